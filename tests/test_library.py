"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every declared symbol, validates arguments before touching the device, and its
bin placement agrees with the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import binning

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2404_11397_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("librbl.so is not built (run __graft_entry__.build())")
    return L


def test_exports_every_declared_symbol():
    L = _lib()
    header = open(os.path.join(ROOT, "include", "rbl.h")).read()
    declared = set(re.findall(r"^\s*(?:int|void|int64_t|const char \*)\s*\*?\s*(rbl_\w+)\s*\(", header, re.M))
    assert declared, "no declarations found"
    lib = L.lib()
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(L.EXPORTS)


@pytest.mark.parametrize("name,nb", [("tf2_1det_32s", 100), ("tf2_3det_128s", 500), ("nrtv2_3det_256s", 1000)])
def test_bin_edges_match_oracle(name, nb):
    from paper_2404_11397_amd import bin_edges
    c = synth.CONFIGS[name]
    f_low, df, n, _ = synth.frequency_grid(c["f_low"], c["f_high"], c["duration"])
    np.testing.assert_array_equal(bin_edges(f_low, df, n, nb), binning.pn_bin_edges(f_low, df, n, nb))


def test_bin_edges_tiny_grid_one_bin_per_point():
    from paper_2404_11397_amd import bin_edges
    np.testing.assert_array_equal(bin_edges(20.0, 1.0, 11, 10), np.arange(11))


def _desc(L, **over):
    nd = over.pop("n_det", 1)
    n = 64
    data = np.zeros((nd, n), complex)
    psd = np.ones((nd, n))
    tens = np.zeros((nd, 9))
    vert = np.zeros((nd, 3))
    th = np.array([1.2, 0.8, 0, 0, 0, 0, 40, 0, 0, 0.3, 0, 0, 0], float)
    edges = np.array([0, 10, 30, 63], np.int64)
    psd = over.get("psd", psd)
    edges = over.get("edges", edges)
    th = over.get("theta", th)
    keep = (data, psd, tens, vert, th, edges)
    d = L.EventDesc(n_det=nd, waveform=over.get("waveform", 0), n_bins=len(edges) - 1, flags=over.get("flags", 0),
                    n_freq=n,
                    f_low=20.0, delta_f=1.0, gmst=0.0,
                    data=data.ctypes.data_as(ctypes.c_void_p), psd=psd.ctypes.data_as(ctypes.c_void_p),
                    det_tensor=tens.ctypes.data_as(ctypes.c_void_p),
                    det_vertex=vert.ctypes.data_as(ctypes.c_void_p),
                    theta_ref=th.ctypes.data_as(ctypes.c_void_p), edges=edges.ctypes.data_as(ctypes.c_void_p))
    return d, keep


@pytest.mark.parametrize("case,code", [
    ({"n_det": 4}, -1),
    ({"edges": np.array([0, 10, 10, 63], np.int64)}, -2),
    ({"edges": np.array([1, 10, 30, 63], np.int64)}, -2),
    ({"edges": np.array([0, 10, 30, 62], np.int64)}, -2),
    ({"psd": np.concatenate([np.ones(63), [0.0]])[None, :]}, -3),
    ({"psd": np.concatenate([np.ones(63), [np.nan]])[None, :]}, -3),
    ({"theta": np.array([1.2, 0.8, 0, 0, 0, 0, -40, 0, 0, 0.3, 0, 0, 0], float)}, -1),
    ({"waveform": 7}, -1),
    ({"flags": 0x10 | 0x1}, -7),
])
def test_event_create_rejects_bad_input_before_device_work(case, code):
    L = _lib()
    d, keep = _desc(L, **case)
    h = ctypes.c_void_p()
    rc = L.lib().rbl_event_create(ctypes.byref(d), None, ctypes.byref(h))
    assert rc == code, L.lib().rbl_last_error()
    assert not h.value
    assert L.lib().rbl_last_error()


def test_null_arguments():
    L = _lib()
    lib = L.lib()
    assert lib.rbl_event_create(None, None, None) == -1
    assert lib.rbl_loglike(None, None, 1, 0, None, None, None) == -1
    assert lib.rbl_loglike_grad(None, None, 1, 0, None, None, None, None) == -1
    assert lib.rbl_bin_edges(20.0, 1.0, 10, 20, None) == -1
    assert lib.rbl_workspace_bytes(None, 10, 0) == 0


def test_profile_sampling_arguments():
    lib = _lib().lib()
    assert lib.rbl_profile_enable(-1) == -1
    assert lib.rbl_profile_enable(8) == 0
    assert lib.rbl_profile_enable(0) == 0
    m, s, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    assert lib.rbl_profile_read(ctypes.byref(m), ctypes.byref(s), ctypes.byref(n)) == 0
    assert n.value == 0


def test_server_argument_errors_without_gpu():
    """Argument checks of the server API are synchronous and need no device."""
    import ctypes
    from paper_2404_11397_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.rbl_server_create(0, 4, 0, ctypes.byref(h)) == -1
    assert L.rbl_server_create(1 << 30, 0, 0, ctypes.byref(h)) == -1
    assert L.rbl_server_create(1 << 30, 17, 0, ctypes.byref(h)) == -1
    assert L.rbl_server_create(1 << 30, 4, 0, None) == -1
    t = ctypes.c_int64()
    assert L.rbl_server_submit(None, 0, None, 1, 0, 1, None, None, 0, ctypes.byref(t)) == -1
    assert L.rbl_server_wait(None, 1, None) == -1
    assert L.rbl_server_add_event(None, None, None) == -1
    L.rbl_server_destroy(None)
    a, b = L.rbl_clock_ns(), L.rbl_clock_ns()
    assert 0 < a <= b
    assert L.rbl_event_footprint_bytes(None) == 0


def test_fault_injection_on_cpu():
    """An injected allocation failure surfaces as RBL_ENOMEM before any device work."""
    from paper_2404_11397_amd import _lib
    L = _lib.lib()
    assert L.rbl_debug_inject_fault(7, 1) == -1
    assert L.rbl_debug_inject_fault(_lib.RBL_FAULT_ALLOC, -1) == -1
    import synth
    f_low, df, n, f = synth.frequency_grid(20.0, 60.0, 4.0)
    psd = synth.analytic_psd(f)[None, :]
    data = np.zeros((1, n), complex)
    geo = synth.detector_geometry(0.1, 0.2, 0.3)
    th0 = np.ascontiguousarray([1.2, 0.8, 0.0, 0.0, 100.0, 100.0, 50.0, 0.0, 0.1, 0.2, 0.3, 0.4, 0.5])
    edges = np.array([0, n // 2, n - 1])
    d = np.ascontiguousarray(data)
    p = np.ascontiguousarray(psd)
    tens = np.ascontiguousarray(geo[0].reshape(1, 9))
    vert = np.ascontiguousarray(geo[1].reshape(1, 3))
    e = np.ascontiguousarray(edges, dtype=np.int64)
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    desc = _lib.EventDesc(n_det=1, waveform=0, n_bins=2, flags=0, n_freq=n, f_low=f_low, delta_f=df, gmst=0.0,
                          data=vp(d), psd=vp(p), det_tensor=vp(tens), det_vertex=vp(vert), theta_ref=vp(th0),
                          edges=vp(e))
    h = ctypes.c_void_p()
    assert L.rbl_debug_inject_fault(_lib.RBL_FAULT_ALLOC, 1) == 0
    try:
        assert L.rbl_event_create(ctypes.byref(desc), None, ctypes.byref(h)) == -4
        assert not h.value
        assert b"allocation" in L.rbl_last_error()
    finally:
        L.rbl_debug_inject_fault(_lib.RBL_FAULT_ALLOC, 0)


def test_binding_rejects_undersized_or_wrong_buffers_before_any_call():
    """The C calls take no buffer sizes, so the binding refuses buffers they would overrun
    (checked with host tensors: the rule is the same on the device)."""
    import torch
    from paper_2404_11397_amd.rbl import check_buffers
    B = 8
    th = torch.zeros((B, 13), dtype=torch.float64)
    ok_l, ok_g = torch.zeros(B, dtype=torch.float64), torch.zeros((B, 13), dtype=torch.float64)
    ws = torch.zeros(1000, dtype=torch.uint8)
    check_buffers(th, ((ok_l, (B,)), (ok_g, (B, 13))), ws, 1000)
    bad = [
        (((ok_l, (B,)),), ws, 1001),                                              # workspace too small
        (((ok_l, (B,)),), torch.zeros(1000, dtype=torch.float32), 10),            # workspace dtype
        (((ok_l, (B,)),), torch.zeros(2000, dtype=torch.uint8)[::2], 10),         # not contiguous
        (((torch.zeros(B - 1, dtype=torch.float64), (B,)),), ws, 10),             # short output
        (((torch.zeros(B, dtype=torch.float32), (B,)),), ws, 10),                 # float32 output
        (((torch.zeros((13, B), dtype=torch.float64).t(), (B, 13)),), ws, 10),    # transposed view
    ]
    for outs, w, need in bad:
        with pytest.raises(ValueError):
            check_buffers(th, outs, w, need)
    with pytest.raises(TypeError):
        check_buffers(th, ((np.zeros(B), (B,)),), ws, 10)
