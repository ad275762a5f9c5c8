"""Python binding of the relative-binned likelihood library.

Device memory and streams come from PyTorch (ROCm); every computation runs in
the library's HIP kernels.  Usage:

    ev = Event(data, psd, det_tensor, det_vertex, gmst, f_low, delta_f,
               theta_ref, edges, waveform="taylorf2")
    lnl = ev.loglike(theta)                  # theta: cuda float64 [B, 13]
    lnl, grad = ev.loglike_grad(theta)
    lnl = LogLikeFn.apply(theta, ev)         # autograd-aware
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check

WAVEFORMS = {"taylorf2": _lib.RBL_TAYLORF2, "phenomd_nrtv2": _lib.RBL_PHENOMD_NRTV2}
PRECISIONS = {"fp64": _lib.RBL_FP64, "mixed": _lib.RBL_MIXED}


def _stream_handle(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _host_f64(x, shape=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def check_buffers(theta, outs, workspace, workspace_bytes):
    """Reject, before anything is enqueued, output and workspace buffers the library would
    overrun: the C calls take no buffer sizes.  outs: ((tensor, shape), ...), each a
    contiguous float64 tensor of exactly that shape on theta's device; workspace: a
    contiguous uint8 tensor on that device with at least workspace_bytes bytes (None when
    the call needs none)."""
    dev = theta.device
    for t, shape in outs:
        if not isinstance(t, torch.Tensor):
            raise TypeError("output buffers must be tensors")
        if t.device != dev or t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
            raise ValueError(f"output buffer must be a contiguous float64 tensor of shape {tuple(shape)} on {dev}; "
                             f"got {t.dtype} {tuple(t.shape)} on {t.device}")
    if workspace is not None:
        if not isinstance(workspace, torch.Tensor):
            raise TypeError("workspace must be a tensor")
        if workspace.device != dev or workspace.dtype != torch.uint8 or not workspace.is_contiguous():
            raise ValueError(f"workspace must be a contiguous uint8 tensor on {dev}")
        if workspace.numel() < workspace_bytes:
            raise ValueError(f"workspace holds {workspace.numel()} bytes; this call needs {workspace_bytes}")


def profile_enable(on=True, every=1):
    """Record HIP events around the library's kernels (benchmark timing) on the first and
    every `every`-th likelihood call; on=False turns timing off."""
    check(_lib.lib().rbl_profile_enable(int(every) if on else 0))


def profile_read():
    """(main-kernel ms, setup-kernel ms, timed calls) summed since the last read."""
    m, s, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    check(_lib.lib().rbl_profile_read(ctypes.byref(m), ctypes.byref(s), ctypes.byref(n)))
    return m.value, s.value, n.value


def profile_read_summary():
    """(summary-pass ms, events) summed over events created since the last read."""
    m, n = ctypes.c_double(), ctypes.c_int64()
    check(_lib.lib().rbl_profile_read_summary(ctypes.byref(m), ctypes.byref(n)))
    return m.value, n.value


def bin_edges(f_low, delta_f, n_freq, n_bins):
    """Bin edges from the library's post-Newtonian phase-bound ansatz (host)."""
    out = np.empty(n_bins + 1, dtype=np.int64)
    check(_lib.lib().rbl_bin_edges(float(f_low), float(delta_f), int(n_freq), int(n_bins),
                                   out.ctypes.data_as(ctypes.c_void_p)))
    return out


def strain(waveform, det_tensor, det_vertex, gmst, f_low, delta_f, n_freq, theta, taper=True,
           device="cuda"):
    """Projected strain [n_det, n_freq] complex128 on the device for one theta."""
    tens = _host_f64(det_tensor).reshape(-1, 9)
    vert = _host_f64(det_vertex).reshape(-1, 3)
    nd = tens.shape[0]
    th = _host_f64(theta).reshape(13)
    out = torch.empty((nd, n_freq, 2), dtype=torch.float64, device=device)
    check(_lib.lib().rbl_strain(WAVEFORMS[waveform], nd, tens.ctypes.data_as(ctypes.c_void_p),
                                vert.ctypes.data_as(ctypes.c_void_p), float(gmst), float(f_low),
                                float(delta_f), int(n_freq), th.ctypes.data_as(ctypes.c_void_p),
                                int(bool(taper)), _ptr(out), _stream_handle(out.device)))
    return torch.view_as_complex(out)


class Event:
    """A resident event: summary data and edge tables on the device."""

    def __init__(self, data, psd, det_tensor, det_vertex, gmst, f_low, delta_f, theta_ref, edges,
                 waveform="taylorf2", keep_b2=False, ref_taper=False, keep_grid=False,
                 centre_nodes=False, device="cuda"):
        self.device = torch.device(device)
        tens = _host_f64(det_tensor).reshape(-1, 9)
        vert = _host_f64(det_vertex).reshape(-1, 3)
        nd = tens.shape[0]
        flags = (_lib.RBL_KEEP_B2 if keep_b2 else 0) | (_lib.RBL_REF_TAPER if ref_taper else 0) \
            | (_lib.RBL_KEEP_GRID if keep_grid else 0) | (_lib.RBL_CENTRE_NODES if centre_nodes else 0)
        if isinstance(data, torch.Tensor):
            d = torch.view_as_real(data.to(self.device, torch.complex128).contiguous()).contiguous()
            p = psd.to(self.device, torch.float64).contiguous()
            flags |= _lib.RBL_INPUT_ON_DEVICE
            n_freq = d.shape[-2]
            dptr, pptr = _ptr(d), _ptr(p)
            self._keep = (d, p)
        else:
            d = np.ascontiguousarray(np.asarray(data, dtype=np.complex128).reshape(nd, -1))
            p = _host_f64(psd).reshape(nd, -1)
            n_freq = d.shape[-1]
            dptr = d.ctypes.data_as(ctypes.c_void_p)
            pptr = p.ctypes.data_as(ctypes.c_void_p)
            self._keep = (d, p)
        if isinstance(edges, (int, np.integer)):   # a bin count: edges placed on the device
            n_bins, e, eptr = int(edges), None, None
        else:
            e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64))
            n_bins, eptr = len(e) - 1, e.ctypes.data_as(ctypes.c_void_p)
        th = _host_f64(theta_ref).reshape(13)
        desc = _lib.EventDesc(n_det=nd, waveform=WAVEFORMS[waveform], n_bins=n_bins, flags=flags,
                              n_freq=n_freq, f_low=float(f_low), delta_f=float(delta_f),
                              gmst=float(gmst), data=dptr, psd=pptr,
                              det_tensor=tens.ctypes.data_as(ctypes.c_void_p),
                              det_vertex=vert.ctypes.data_as(ctypes.c_void_p),
                              theta_ref=th.ctypes.data_as(ctypes.c_void_p), edges=eptr)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(_lib.lib().rbl_event_create(ctypes.byref(desc), _stream_handle(self.device),
                                              ctypes.byref(handle)))
        self._h = handle
        self._keep = None
        self.n_det, self.n_bins, self.n_freq = nd, n_bins, n_freq
        self.waveform = waveform

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                _lib.lib().rbl_event_free(h)
            except Exception:
                pass
            self._h = None

    # -- queries ----------------------------------------------------------------
    def summary(self):
        """Summary data [n_det, n_bins, 7] = (ReA0, ImA0, ReA1, ImA1, B0, B1, B2)."""
        out = np.empty((self.n_det, self.n_bins, 7), dtype=np.float64)
        check(_lib.lib().rbl_event_get_summary(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def edges(self):
        """The bin edges (grid indices) [n_bins + 1], given or placed on the device."""
        out = np.empty(self.n_bins + 1, dtype=np.int64)
        check(_lib.lib().rbl_event_get_edges(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def footprint_bytes(self):
        fb = ctypes.c_int64()
        check(_lib.lib().rbl_event_info(self._h, None, None, None, ctypes.byref(fb)))
        return fb.value

    def workspace_bytes(self, B, with_grad=False):
        return int(_lib.lib().rbl_workspace_bytes(self._h, int(B), int(bool(with_grad))))

    def workspace(self, B, with_grad=False):
        return torch.empty(max(self.workspace_bytes(B, with_grad), 256), dtype=torch.uint8, device=self.device)

    # -- evaluation -----------------------------------------------------------------
    def _theta(self, theta):
        if not (isinstance(theta, torch.Tensor) and theta.is_cuda and theta.dtype == torch.float64):
            raise TypeError("theta must be a cuda float64 tensor [B, 13]")
        if theta.dim() != 2 or theta.shape[1] != 13:
            raise ValueError("theta must have shape [B, 13]")
        return theta.contiguous()

    def loglike(self, theta, precision="fp64", out=None, workspace=None):
        theta = self._theta(theta)
        B = theta.shape[0]
        lnl = torch.empty(B, dtype=torch.float64, device=theta.device) if out is None else out
        ws = self.workspace(B) if workspace is None else workspace
        check_buffers(theta, ((lnl, (B,)),), ws, self.workspace_bytes(B))
        check(_lib.lib().rbl_loglike(self._h, _ptr(theta), B, PRECISIONS[precision], _ptr(lnl),
                                     _ptr(ws), _stream_handle(theta.device)))
        return lnl

    def loglike_grad(self, theta, precision="fp64", out=None, workspace=None):
        theta = self._theta(theta)
        B = theta.shape[0]
        if out is None:
            lnl = torch.empty(B, dtype=torch.float64, device=theta.device)
            grad = torch.empty((B, 13), dtype=torch.float64, device=theta.device)
        else:
            lnl, grad = out
        ws = self.workspace(B, True) if workspace is None else workspace
        check_buffers(theta, ((lnl, (B,)), (grad, (B, 13))), ws, self.workspace_bytes(B, True))
        check(_lib.lib().rbl_loglike_grad(self._h, _ptr(theta), B, PRECISIONS[precision], _ptr(lnl),
                                          _ptr(grad), _ptr(ws), _stream_handle(theta.device)))
        return lnl, grad

    def loglike_full(self, theta, out=None, workspace=None):
        theta = self._theta(theta)
        B = theta.shape[0]
        lnl = torch.empty(B, dtype=torch.float64, device=theta.device) if out is None else out
        ws = self.workspace(B) if workspace is None else workspace
        check_buffers(theta, ((lnl, (B,)),), ws, self.workspace_bytes(B))
        check(_lib.lib().rbl_loglike_full(self._h, _ptr(theta), B, _ptr(lnl), _ptr(ws),
                                          _stream_handle(theta.device)))
        return lnl


def ref_search(event, lo, hi, starts, sigma0, normals):
    """CMA-ES reference-parameter search over the full-band lnL (rbl_ref_search): independent
    runs from starts [n_starts, 13] (or one start [13]) advanced together.  normals:
    [n_starts, generations, lambda, 13] (or [generations, lambda, 13] for one start) standard
    normals, the caller's random numbers.  Returns (best theta [13], best lnL, traces): traces
    is a list with one array [generations run, 15] per start."""
    st = np.atleast_2d(_host_f64(starts))
    z = _host_f64(normals)
    if z.ndim == 3:
        z = z[None]
    if st.ndim != 2 or st.shape[1] != 13:
        raise ValueError("starts must have shape [n_starts, 13] or [13]")
    if z.ndim != 4 or z.shape[0] != st.shape[0] or z.shape[3] != 13:
        raise ValueError("normals must have shape [n_starts, generations, lambda, 13]")
    n_starts, gens, lam = z.shape[0], z.shape[1], z.shape[2]
    z = np.ascontiguousarray(z)
    st = np.ascontiguousarray(st)
    lo_, hi_ = (_host_f64(v).reshape(13) for v in (lo, hi))
    best = np.empty(13)
    best_l = ctypes.c_double()
    ran = np.zeros(n_starts, dtype=np.int32)
    trace = np.empty((n_starts, gens, 15))
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    with torch.cuda.device(event.device):
        check(_lib.lib().rbl_ref_search(event._h, vp(lo_), vp(hi_), int(n_starts), vp(st), float(sigma0), int(lam),
                                        int(gens), vp(z), vp(best), ctypes.byref(best_l), vp(trace), vp(ran),
                                        _stream_handle(event.device)))
    return best, best_l.value, [trace[r, :ran[r]] for r in range(n_starts)]


class LogLikeFn(torch.autograd.Function):
    """lnL(theta) with the library's adjoint gradient as its backward."""

    @staticmethod
    def forward(ctx, theta, event, precision="fp64"):
        lnl, grad = event.loglike_grad(theta, precision)
        ctx.save_for_backward(grad)
        return lnl

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g[:, None] * grad, None, None
