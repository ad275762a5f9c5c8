"""Python binding of the device MALA step (argument marshalling only).

    chains = Mala(event, z)                # z: cuda float64 [B, 13] sampled coordinates
    acc = chains.step(step, lo, hi, xi, logu)   # in place on chains.z / .lnl / .gz
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check
from .rbl import PRECISIONS, _ptr, _stream_handle, check_buffers


def _host13(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(13))
    return a, a.ctypes.data


def _is_host13(x):
    return (isinstance(x, np.ndarray) and x.dtype == np.float64 and x.size == 13 and x.flags.c_contiguous)


class Mala:
    """B chains of the MALA local sampler on one event; state lives on the device."""

    def __init__(self, event, z, precision="fp64"):
        if not (isinstance(z, torch.Tensor) and z.is_cuda and z.dtype == torch.float64 and z.dim() == 2
                and z.shape[1] == 13):
            raise TypeError("z must be a cuda float64 tensor [B, 13]")
        self.event = event
        self.precision = precision
        self.z = z.contiguous().clone()
        B = self.z.shape[0]
        self.lnl = torch.empty(B, dtype=torch.float64, device=z.device)
        self.gz = torch.empty((B, 13), dtype=torch.float64, device=z.device)
        self.accepted = torch.zeros(B, dtype=torch.int32, device=z.device)
        n = _lib.lib().rbl_mala_workspace_bytes(event._h, B)
        self._ws = torch.empty(max(n, 256), dtype=torch.uint8, device=z.device)
        # the chain-state buffers never move: their pointers are taken once
        self._p = [_ptr(t) for t in (self.z, self.lnl, self.gz, self.accepted, self._ws)]
        self._box = (None, None, None, None)  # the last (step, lo, hi) arrays passed as they are
        check(_lib.lib().rbl_mala_init(event._h, _ptr(self.z), B, PRECISIONS[precision], _ptr(self.lnl),
                                       _ptr(self.gz), _ptr(self._ws), _stream_handle(z.device)))

    def step(self, step, lo, hi, xi, logu):
        """One MALA step; xi cuda [B, 13] standard normals, logu cuda [B] log-uniforms."""
        B = self.z.shape[0]
        xi = xi.contiguous()
        logu = logu.contiguous()
        check_buffers(self.z, ((xi, (B, 13)), (logu, (B,))), None, 0)
        last = self._box
        if step is last[0] and lo is last[1] and hi is last[2]:
            sp, lp, hp = last[3]  # the same float64 arrays as the last call (read at the call)
        else:
            s, sp = _host13(step)
            l, lp = _host13(lo)
            h, hp = _host13(hi)
            if _is_host13(step) and _is_host13(lo) and _is_host13(hi):
                self._box = (step, lo, hi, (sp, lp, hp))
        pz, pl, pg, pa, pw = self._p
        check(_lib.lib().rbl_mala_step(self.event._h, pz, pl, pg, B, PRECISIONS[self.precision], sp, lp, hp,
                                       _ptr(xi), _ptr(logu), pa, pw, _stream_handle(self.z.device)))
        return self.accepted
