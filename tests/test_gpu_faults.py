"""Error paths forced from the host (rbl_debug_inject_fault): an injected allocation or
launch failure is reported as RBL_ENOMEM / RBL_EDEVICE, and the library keeps working
(no kernel is made to fail)."""
import numpy as np
import pytest

from gpu_common import gpu_event, oracle_event

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


@pytest.fixture()
def lib():
    from paper_2404_11397_amd import _lib
    L = _lib.lib()
    yield L, _lib
    L.rbl_debug_inject_fault(_lib.RBL_FAULT_ALLOC, 0)
    L.rbl_debug_inject_fault(_lib.RBL_FAULT_LAUNCH, 0)


def test_injected_launch_failure_then_recovery(lib):
    from paper_2404_11397_amd import RblError
    L, _lib = lib
    ev, w = oracle_event("tf2_1det_32s", batch=64)
    gev = gpu_event(ev)
    t = torch.as_tensor(w["theta"], dtype=torch.float64, device="cuda")
    want = gev.loglike(t).cpu().numpy()
    L.rbl_debug_inject_fault(_lib.RBL_FAULT_LAUNCH, 1)
    with pytest.raises(RblError) as ei:
        gev.loglike_grad(t)
    assert ei.value.code == -5
    L.rbl_debug_inject_fault(_lib.RBL_FAULT_LAUNCH, 0)
    got = gev.loglike(t).cpu().numpy()
    assert np.array_equal(got, want)


@pytest.mark.parametrize("which", [1, 3, 6])
def test_injected_allocation_failure_in_event_build(lib, which):
    from paper_2404_11397_amd import RblError
    L, _lib = lib
    ev, w = oracle_event("tf2_1det_32s", batch=8)
    L.rbl_debug_inject_fault(_lib.RBL_FAULT_ALLOC, which)
    with pytest.raises(RblError) as ei:
        gpu_event(ev)
    assert ei.value.code == -4
    L.rbl_debug_inject_fault(_lib.RBL_FAULT_ALLOC, 0)
    gev = gpu_event(ev)  # the next build succeeds
    t = torch.as_tensor(w["theta"], dtype=torch.float64, device="cuda")
    assert torch.isfinite(gev.loglike(t)).all()


def test_injected_allocation_failure_in_server(lib):
    from paper_2404_11397_amd import RblError, Server
    L, _lib = lib
    ev, w = oracle_event("tf2_1det_32s", batch=300)
    gev = gpu_event(ev)
    with Server(1 << 30, n_streams=2) as srv:
        eid = srv.add_event(gev)
        L.rbl_debug_inject_fault(_lib.RBL_FAULT_ALLOC, 1)
        t = srv.submit(eid, w["theta"], precision="fp64")
        with pytest.raises(RblError) as ei:
            srv.wait(t)
        assert ei.value.code == -4
        L.rbl_debug_inject_fault(_lib.RBL_FAULT_ALLOC, 0)
        lnl, grad, _ = srv.wait(srv.submit(eid, w["theta"], precision="fp64"))
        want_l, want_g = gev.loglike_grad(torch.as_tensor(w["theta"], dtype=torch.float64, device="cuda"))
        assert np.array_equal(lnl, want_l.cpu().numpy()) and np.array_equal(grad, want_g.cpu().numpy())


def test_binding_refuses_undersized_workspace_and_short_outputs():
    """A workspace sized for the lnL alone, or a short output, is refused by the binding
    before anything is enqueued; the library then still gives the same results."""
    ev, w = oracle_event("tf2_1det_32s", batch=64)
    gev = gpu_event(ev)
    t = torch.as_tensor(w["theta"], dtype=torch.float64, device="cuda")
    B = t.shape[0]
    want_l, want_g = gev.loglike_grad(t)
    small = gev.workspace(B, with_grad=False)
    with pytest.raises(ValueError):
        gev.loglike_grad(t, workspace=small)
    with pytest.raises(ValueError):
        gev.loglike(t, out=torch.empty(B - 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        gev.loglike_grad(t, out=(torch.empty(B, dtype=torch.float64, device="cuda"),
                                 torch.empty((B, 13), dtype=torch.float32, device="cuda")))
    got_l, got_g = gev.loglike_grad(t)
    assert torch.equal(got_l, want_l) and torch.equal(got_g, want_g)
