"""ctypes binding of include/inc.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libinc.so")

INC_OK = 0
INC_ERR_ARG = -1
INC_ERR_RANGE = -2
INC_ERR_CAPACITY = -3
INC_ERR_NO_DEVICE = -4
INC_ERR_OOM = -5
INC_ERR_DEVICE = -6
INC_ERR_BUSY = -7
INC_ERR_TOO_LARGE = -8
NOALLOC_MAX_EVENTS = 1048576
MODE_PLAIN = 0
MODE_PERSISTENT = 1
MODE_STAGED = 2
MODE_VERTEX = 3

# exported symbols, in the order include/inc.h declares them
SYMBOLS = (
    "inc_strerror", "inc_ctx_create", "inc_ctx_destroy", "inc_ctx_tables", "inc_ctx_xs_table",
    "inc_simulate_dev", "inc_simulate_dev_noalloc", "inc_evaporate_dev", "inc_simulate", "inc_server_create", "inc_server_destroy",
    "inc_server_submit", "inc_server_poll", "inc_server_wait", "inc_server_fetch",
    "inc_server_stats_get", "inc_server_stats_reset", "inc_server_hold", "inc_server_replay", "inc_ring_create",
    "inc_ring_create_device",
    "inc_ring_destroy",
    "inc_ring_simulate", "inc_ring_simulate_to", "inc_ctx_tally_shape", "inc_tally_residuals", "inc_contract_version",
)


class Nucleus(C.Structure):
    _fields_ = [("A", C.c_int), ("Z", C.c_int)]


class Options(C.Structure):
    _fields_ = [
        ("uniform_density", C.c_int), ("zero_fermi", C.c_int), ("zero_binding", C.c_int),
        ("no_pauli", C.c_int), ("no_evaporation", C.c_int), ("stop_after_first", C.c_int),
        ("const_sigma_mb", C.c_float), ("fixed_b_on", C.c_int), ("fixed_b", C.c_float),
        ("block_size", C.c_int), ("evap_threshold", C.c_int), ("tent_threshold", C.c_int),
        ("kin_threshold", C.c_int), ("waves_per_cu", C.c_int), ("stack_levels", C.c_int),
        ("same_stream", C.c_int), ("fast_math", C.c_int), ("start_threshold", C.c_int),
        ("input_order", C.c_int),
        ("photon_evaporation", C.c_int),
        ("table_layout", C.c_int),
        ("chunk_events", C.c_int),
        ("heavy_fragments", C.c_int),
        ("vertex_window", C.c_int),
        ("vertex_launch", C.c_int),
    ]


class Output(C.Structure):
    _fields_ = [
        ("res", C.c_void_p), ("sec_event", C.c_void_p), ("sec_species", C.c_void_p),
        ("sec_stage", C.c_void_p), ("sec_T", C.c_void_p), ("sec_ux", C.c_void_p),
        ("sec_uy", C.c_void_p), ("sec_uz", C.c_void_p), ("sec_capacity", C.c_size_t),
        ("counters", C.c_void_p), ("history", C.c_void_p),
    ]


class Batch(C.Structure):
    _fields_ = [
        ("n", C.c_size_t), ("target_idx", C.c_void_p), ("T0", C.c_void_p),
        ("seed", C.c_uint64), ("first_event_id", C.c_uint64),
    ]


class Excited(C.Structure):
    _fields_ = [
        ("n", C.c_size_t), ("A", C.c_void_p), ("Z", C.c_void_p), ("Ex", C.c_void_p), ("P", C.c_void_p),
        ("seed", C.c_uint64), ("first_event_id", C.c_uint64),
    ]


class Request(C.Structure):
    _fields_ = [
        ("n", C.c_size_t), ("target_idx", C.c_void_p), ("T0", C.c_void_p),
        ("seed", C.c_uint64), ("first_event_id", C.c_uint64), ("sec_capacity", C.c_size_t),
    ]


class HostOutput(C.Structure):
    _fields_ = [
        ("res", C.c_void_p), ("sec_event", C.c_void_p), ("sec_species", C.c_void_p),
        ("sec_stage", C.c_void_p), ("sec_T", C.c_void_p), ("sec_ux", C.c_void_p),
        ("sec_uy", C.c_void_p), ("sec_uz", C.c_void_p), ("sec_capacity", C.c_size_t),
        ("n_sec", C.POINTER(C.c_ulonglong)), ("latency_s", C.POINTER(C.c_double)),
    ]


class ServerStats(C.Structure):
    _fields_ = [
        ("submitted", C.c_ulonglong), ("completed", C.c_ulonglong), ("rejected_busy", C.c_ulonglong),
        ("events", C.c_ulonglong), ("secondaries", C.c_ulonglong), ("in_flight", C.c_ulonglong),
        ("pool_free_largest", C.c_size_t), ("launches", C.c_ulonglong), ("latency_p50_s", C.c_double),
        ("latency_p99_s", C.c_double), ("events_per_s", C.c_double),
    ]


class RingStats(C.Structure):
    _fields_ = [
        ("records", C.c_ulonglong), ("slots", C.c_ulonglong), ("wraps", C.c_ulonglong),
        ("consumer_idle_polls", C.c_ulonglong), ("seconds", C.c_double), ("producer_gave_up", C.c_uint),
    ]


class RingChunk(C.Structure):
    _fields_ = [
        ("first", C.c_ulonglong), ("n", C.c_size_t), ("event", C.POINTER(C.c_uint32)),
        ("kind", C.POINTER(C.c_uint32)), ("T", C.POINTER(C.c_float)), ("ux", C.POINTER(C.c_float)),
        ("uy", C.POINTER(C.c_float)), ("uz", C.POINTER(C.c_float)),
    ]


RING_CONSUMER = C.CFUNCTYPE(None, C.POINTER(RingChunk), C.c_void_p)


RESIDUAL_DTYPE = np.dtype(
    [("A_f", "<u2"), ("Z_f", "<u2"), ("n_sec", "<u2"), ("flags", "<u2"),
     ("Ex_casc", "<f4"), ("Ex_f", "<f4"), ("p_f", "<f4", 3),
     ("n_coll", "<u2"), ("n_retry", "<u2")]
)
assert RESIDUAL_DTYPE.itemsize == 32

_lib = None


class IncError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = load().inc_strerror(code).decode() if _lib is not None else str(code)
        super().__init__("%s: %s (%d)" % (what, msg, code) if what else "%s (%d)" % (msg, code))


def load():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        # One HIP runtime per process: torch ships its own libamdhip64.so.7 and
        # the dynamic linker binds libinc.so to whichever copy is loaded
        # first, so torch (which owns the device memory and streams) goes
        # first.
        import torch  # noqa: F401

        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libinc.so is not built: run `python -m paper_1309_7963_amd.build` "
                "(the GPU path has no fallback)"
            )
        L = C.CDLL(LIB_PATH)
        L.inc_strerror.argtypes = [C.c_int]
        L.inc_strerror.restype = C.c_char_p
        L.inc_ctx_create.argtypes = [C.POINTER(Nucleus), C.c_int, C.POINTER(Options), C.POINTER(C.c_void_p)]
        L.inc_ctx_create.restype = C.c_int
        L.inc_ctx_destroy.argtypes = [C.c_void_p]
        L.inc_ctx_destroy.restype = C.c_int
        L.inc_ctx_tables.argtypes = [C.c_void_p, C.c_void_p]
        L.inc_ctx_tables.restype = C.c_int
        L.inc_ctx_xs_table.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_float),
                                       C.POINTER(C.c_float)]
        L.inc_ctx_xs_table.restype = C.c_int
        L.inc_simulate_dev.argtypes = [C.c_void_p, C.POINTER(Batch), C.POINTER(Output), C.c_void_p, C.c_int]
        L.inc_simulate_dev.restype = C.c_int
        L.inc_simulate_dev_noalloc.argtypes = [C.c_void_p, C.POINTER(Batch), C.POINTER(Output), C.c_void_p, C.c_int]
        L.inc_simulate_dev_noalloc.restype = C.c_int
        L.inc_evaporate_dev.argtypes = [C.c_void_p, C.POINTER(Excited), C.POINTER(Output), C.c_void_p]
        L.inc_evaporate_dev.restype = C.c_int
        L.inc_simulate.argtypes = [
            C.c_int, C.c_int, C.c_void_p, C.c_size_t, C.c_uint64, C.c_void_p,
            C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
            C.c_size_t, C.POINTER(C.c_size_t),
        ]
        L.inc_simulate.restype = C.c_int
        vp = C.c_void_p
        L.inc_server_create.argtypes = [vp, C.c_size_t, C.c_int, C.POINTER(vp)]
        L.inc_server_create.restype = C.c_int
        L.inc_server_destroy.argtypes = [vp]
        L.inc_server_destroy.restype = C.c_int
        L.inc_server_submit.argtypes = [vp, C.POINTER(Request), C.POINTER(C.c_uint64)]
        L.inc_server_submit.restype = C.c_int
        L.inc_server_poll.argtypes = [vp, C.c_uint64]
        L.inc_server_poll.restype = C.c_int
        L.inc_server_wait.argtypes = [vp, C.c_uint64]
        L.inc_server_wait.restype = C.c_int
        L.inc_server_fetch.argtypes = [vp, C.c_uint64, C.POINTER(HostOutput)]
        L.inc_server_fetch.restype = C.c_int
        L.inc_server_stats_get.argtypes = [vp, C.POINTER(ServerStats)]
        L.inc_server_stats_get.restype = C.c_int
        L.inc_server_stats_reset.argtypes = [vp]
        L.inc_server_stats_reset.restype = C.c_int
        L.inc_server_hold.argtypes = [vp, C.c_int]
        L.inc_server_hold.restype = C.c_int
        L.inc_server_replay.argtypes = [vp, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]
        L.inc_server_replay.restype = C.c_int
        L.inc_ring_create.argtypes = [vp, C.c_size_t, C.POINTER(vp)]
        L.inc_ring_create.restype = C.c_int
        L.inc_ring_create_device.argtypes = [vp, C.c_size_t, C.c_size_t, C.POINTER(vp)]
        L.inc_ring_create_device.restype = C.c_int
        L.inc_ring_destroy.argtypes = [vp]
        L.inc_ring_destroy.restype = C.c_int
        L.inc_ring_simulate.argtypes = [vp, C.POINTER(Batch), vp, C.POINTER(HostOutput), vp, C.c_int,
                                        C.POINTER(RingStats)]
        L.inc_ring_simulate.restype = C.c_int
        L.inc_ring_simulate_to.argtypes = [vp, C.POINTER(Batch), vp, vp, RING_CONSUMER, vp, C.POINTER(C.c_ulonglong),
                                           vp, C.c_int, C.POINTER(RingStats)]
        L.inc_ring_simulate_to.restype = C.c_int
        L.inc_ctx_tally_shape.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.inc_ctx_tally_shape.restype = C.c_int
        L.inc_tally_residuals.argtypes = [vp, C.POINTER(Batch), vp, C.c_int, vp, vp]
        L.inc_tally_residuals.restype = C.c_int
        L.inc_contract_version.argtypes = []
        L.inc_contract_version.restype = C.c_int
        _lib = L
    return _lib


def check(code: int, what: str = ""):
    if code != INC_OK:
        raise IncError(code, what)
