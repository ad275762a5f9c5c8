"""Python binding of the request server (continuous batching over resident events).

    srv = Server(hbm_budget_bytes=8 << 30, n_streams=4)
    eid = srv.add_event(ev)                      # ev: a resident Event
    t = srv.submit(eid, theta_host, precision="mixed", grad=True)
    lnl, grad, info = srv.wait(t)                # info: arrival/admit/done times [ns]

theta and the result buffers are host numpy arrays owned by the ticket until wait()
returns; the server copies them through pinned staging buffers of its own.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import check
from .rbl import PRECISIONS


def clock_ns():
    """The server's monotonic clock (CLOCK_MONOTONIC, ns)."""
    return _lib.lib().rbl_clock_ns()


class Ticket:
    __slots__ = ("id", "theta", "lnl", "grad", "event")

    def __init__(self, tid, theta, lnl, grad, event):
        self.id, self.theta, self.lnl, self.grad, self.event = tid, theta, lnl, grad, event


class Server:
    def __init__(self, hbm_budget_bytes, n_streams=4, graphs=True, spin=False, merge=True):
        h = ctypes.c_void_p()
        flags = ((0 if graphs else _lib.RBL_SERVE_NO_GRAPHS) | (_lib.RBL_SERVE_SPIN if spin else 0)
                 | (0 if merge else _lib.RBL_SERVE_NO_MERGE))
        check(_lib.lib().rbl_server_create(int(hbm_budget_bytes), int(n_streams), flags, ctypes.byref(h)))
        self._h = h
        self._events = {}

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib.lib().rbl_server_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def add_event(self, event):
        eid = ctypes.c_int32()
        check(_lib.lib().rbl_server_add_event(self._h, event._h, ctypes.byref(eid)))
        self._events[eid.value] = event
        return eid.value

    def remove_event(self, event_id):
        check(_lib.lib().rbl_server_remove_event(self._h, int(event_id)))
        self._events.pop(event_id, None)

    def submit(self, event_id, theta, precision="mixed", grad=True, t_arrival_ns=0):
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1, 13))
        B = th.shape[0]
        lnl = np.empty(B, dtype=np.float64)
        g = np.empty((B, 13), dtype=np.float64) if grad else None
        tid = ctypes.c_int64()
        check(_lib.lib().rbl_server_submit(
            self._h, int(event_id), th.ctypes.data_as(ctypes.c_void_p), B, PRECISIONS[precision], int(bool(grad)),
            lnl.ctypes.data_as(ctypes.c_void_p), None if g is None else g.ctypes.data_as(ctypes.c_void_p),
            int(t_arrival_ns), ctypes.byref(tid)))
        return Ticket(tid.value, th, lnl, g, event_id)

    def wait(self, ticket):
        info = _lib.RequestInfo()
        check(_lib.lib().rbl_server_wait(self._h, ticket.id, ctypes.byref(info)))
        return ticket.lnl, ticket.grad, {"t_arrival_ns": info.t_arrival_ns, "t_admit_ns": info.t_admit_ns,
                                         "t_done_ns": info.t_done_ns, "stream": info.stream}

    def stats(self):
        st = _lib.ServerStats()
        check(_lib.lib().rbl_server_get_stats(self._h, ctypes.byref(st)))
        return {n: getattr(st, n) for n, _ in _lib.ServerStats._fields_}
