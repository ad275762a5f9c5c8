"""ctypes binding of librbl.so (argument marshalling only).

The library is the HIP build in this directory.  If it is missing or cannot
be loaded, every call raises: there is no fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbl.so")

RBL_OK = 0
RBL_TAYLORF2, RBL_PHENOMD_NRTV2 = 0, 1
RBL_FP64, RBL_MIXED = 0, 1
RBL_KEEP_B2, RBL_REF_TAPER, RBL_KEEP_GRID, RBL_INPUT_ON_DEVICE, RBL_CENTRE_NODES = 0x1, 0x2, 0x4, 0x8, 0x10
ERROR_NAMES = {-1: "RBL_EINVAL", -2: "RBL_EEDGES", -3: "RBL_EPSD", -4: "RBL_ENOMEM",
               -5: "RBL_EDEVICE", -6: "RBL_EREF", -7: "RBL_EUNSUPPORTED"}

EXPORTS = ("rbl_event_create", "rbl_event_free", "rbl_workspace_bytes", "rbl_loglike",
           "rbl_loglike_grad", "rbl_loglike_full", "rbl_strain", "rbl_event_get_summary",
           "rbl_event_info", "rbl_bin_edges", "rbl_profile_enable", "rbl_profile_read", "rbl_profile_read_summary",
           "rbl_last_error", "rbl_server_create", "rbl_server_add_event", "rbl_server_remove_event",
           "rbl_server_submit", "rbl_server_wait", "rbl_server_get_stats", "rbl_server_destroy", "rbl_clock_ns",
           "rbl_event_footprint_bytes", "rbl_debug_inject_fault", "rbl_mala_workspace_bytes", "rbl_mala_init",
           "rbl_mala_step", "rbl_loglike_grad_noalloc", "rbl_ref_search", "rbl_event_get_edges")
RBL_FAULT_ALLOC, RBL_FAULT_LAUNCH = 0, 1
RBL_NOALLOC_MAX_CHAINS = 16384
RBL_SERVE_NO_GRAPHS, RBL_SERVE_SPIN, RBL_SERVE_NO_MERGE = 0x1, 0x2, 0x4


class RblError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class EventDesc(ctypes.Structure):
    _fields_ = [("n_det", ctypes.c_int32), ("waveform", ctypes.c_int32), ("n_bins", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("n_freq", ctypes.c_int64), ("f_low", ctypes.c_double),
                ("delta_f", ctypes.c_double), ("gmst", ctypes.c_double),
                ("data", ctypes.c_void_p), ("psd", ctypes.c_void_p),
                ("det_tensor", ctypes.c_void_p), ("det_vertex", ctypes.c_void_p),
                ("theta_ref", ctypes.c_void_p), ("edges", ctypes.c_void_p)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("t_arrival_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64),
                ("status", ctypes.c_int32), ("stream", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "budget_bytes", "resident_bytes", "buffer_bytes", "submitted", "completed", "queued", "in_flight",
        "max_in_flight", "graphs", "graph_launches", "plain_launches", "buffer_allocs", "buffer_releases",
        "admission_waits", "merged_launches", "merged_requests")]


_lib = None


def lib():
    """Load librbl.so once (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"librbl.so not built at {LIB_PATH}; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.rbl_event_create.argtypes = [ctypes.POINTER(EventDesc), vp, ctypes.POINTER(vp)]
    L.rbl_event_create.restype = ctypes.c_int
    L.rbl_event_free.argtypes = [vp]
    L.rbl_event_free.restype = None
    L.rbl_workspace_bytes.argtypes = [vp, i64, i32]
    L.rbl_workspace_bytes.restype = i64
    L.rbl_loglike.argtypes = [vp, vp, i64, i32, vp, vp, vp]
    L.rbl_loglike.restype = ctypes.c_int
    L.rbl_loglike_grad.argtypes = [vp, vp, i64, i32, vp, vp, vp, vp]
    L.rbl_loglike_grad.restype = ctypes.c_int
    L.rbl_loglike_grad_noalloc.argtypes = [vp, vp, i64, i32, vp, vp, vp]
    L.rbl_loglike_grad_noalloc.restype = ctypes.c_int
    L.rbl_loglike_full.argtypes = [vp, vp, i64, vp, vp, vp]
    L.rbl_loglike_full.restype = ctypes.c_int
    L.rbl_ref_search.argtypes = [vp, vp, vp, i32, vp, dbl, i32, i32, vp, vp, vp, vp, vp, vp]
    L.rbl_ref_search.restype = ctypes.c_int
    L.rbl_strain.argtypes = [i32, i32, vp, vp, dbl, dbl, dbl, i64, vp, i32, vp, vp]
    L.rbl_strain.restype = ctypes.c_int
    L.rbl_event_get_summary.argtypes = [vp, vp]
    L.rbl_event_get_summary.restype = ctypes.c_int
    L.rbl_event_get_edges.argtypes = [vp, vp]
    L.rbl_event_get_edges.restype = ctypes.c_int
    L.rbl_event_info.argtypes = [vp, vp, vp, vp, vp]
    L.rbl_event_info.restype = ctypes.c_int
    L.rbl_bin_edges.argtypes = [dbl, dbl, i64, i32, vp]
    L.rbl_bin_edges.restype = ctypes.c_int
    L.rbl_profile_enable.argtypes = [i32]
    L.rbl_profile_enable.restype = ctypes.c_int
    L.rbl_profile_read.argtypes = [vp, vp, vp]
    L.rbl_profile_read.restype = ctypes.c_int
    L.rbl_profile_read_summary.argtypes = [vp, vp]
    L.rbl_profile_read_summary.restype = ctypes.c_int
    L.rbl_last_error.argtypes = []
    L.rbl_last_error.restype = ctypes.c_char_p
    L.rbl_server_create.argtypes = [i64, i32, ctypes.c_uint32, ctypes.POINTER(vp)]
    L.rbl_server_create.restype = ctypes.c_int
    L.rbl_server_add_event.argtypes = [vp, vp, ctypes.POINTER(i32)]
    L.rbl_server_add_event.restype = ctypes.c_int
    L.rbl_server_remove_event.argtypes = [vp, i32]
    L.rbl_server_remove_event.restype = ctypes.c_int
    L.rbl_server_submit.argtypes = [vp, i32, vp, i64, i32, i32, vp, vp, i64, ctypes.POINTER(i64)]
    L.rbl_server_submit.restype = ctypes.c_int
    L.rbl_server_wait.argtypes = [vp, i64, ctypes.POINTER(RequestInfo)]
    L.rbl_server_wait.restype = ctypes.c_int
    L.rbl_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    L.rbl_server_get_stats.restype = ctypes.c_int
    L.rbl_server_destroy.argtypes = [vp]
    L.rbl_server_destroy.restype = None
    L.rbl_clock_ns.argtypes = []
    L.rbl_clock_ns.restype = i64
    L.rbl_event_footprint_bytes.argtypes = [vp]
    L.rbl_event_footprint_bytes.restype = i64
    L.rbl_debug_inject_fault.argtypes = [i32, i32]
    L.rbl_debug_inject_fault.restype = ctypes.c_int
    L.rbl_mala_workspace_bytes.argtypes = [vp, i64]
    L.rbl_mala_workspace_bytes.restype = i64
    L.rbl_mala_init.argtypes = [vp, vp, i64, i32, vp, vp, vp, vp]
    L.rbl_mala_init.restype = ctypes.c_int
    L.rbl_mala_step.argtypes = [vp, vp, vp, vp, i64, i32, vp, vp, vp, vp, vp, vp, vp, vp]
    L.rbl_mala_step.restype = ctypes.c_int
    _lib = L
    return L


def check(rc):
    if rc != RBL_OK:
        raise RblError(rc, lib().rbl_last_error().decode())
    return rc
