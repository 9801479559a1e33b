"""ctypes loader for libtebd.so (the HIP library).  Fails loudly when it is missing."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libtebd.so")

# every exported symbol of include/tebd.h
EXPORTS = [
    "mps_arena_bytes", "mps_alloc", "tebd_step", "apply_jumps", "measure_corr", "mps_free",
    "mps_last_error", "mps_instance_tensor_capacity", "mps_instance_lambda_capacity",
    "mps_get_instance", "mps_set_instance", "mps_replicate", "tn_gate", "tn_tuning", "tn_graph_enable", "tn_overlap", "tn_schedule", "tn_prof_enable",
    "tn_prof_query", "tn_prof_busy", "tn_measure_async_bytes", "tn_measure_async_enable", "measure_corr_start",
    "measure_corr_finish", "measure_corr_noalloc", "tn_stats", "tn_theta_precision", "tn_buckets",
]


class TnModel(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int),
        ("d", ctypes.c_int),
        ("h_bond", ctypes.POINTER(ctypes.c_double)),
        ("n_jumps", ctypes.c_int),
        ("jump_site", ctypes.POINTER(ctypes.c_int)),
        ("jump_op", ctypes.POINTER(ctypes.c_double)),
        ("gamma", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None


def load():
    """Load the built library (build it with paper_2609_18841_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run paper_2609_18841_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, dp, ip, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), ctypes.c_size_t
    ubp = ctypes.POINTER(ctypes.c_ubyte)
    lib.mps_arena_bytes.restype = sz
    lib.mps_arena_bytes.argtypes = [ctypes.c_int] * 7
    lib.mps_alloc.restype = ctypes.c_int
    lib.mps_alloc.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(TnModel), ctypes.c_int, ctypes.c_int,
                              ctypes.c_int, ctypes.c_int, ip, ctypes.c_double, vp, sz, vp]
    lib.tebd_step.restype = ctypes.c_int
    lib.tebd_step.argtypes = [vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, ubp, dp]
    lib.apply_jumps.restype = ctypes.c_int
    lib.apply_jumps.argtypes = [vp, ctypes.c_int, ctypes.c_double, dp, ctypes.c_int, ip, ubp]
    lib.measure_corr.restype = ctypes.c_int
    lib.measure_corr.argtypes = [vp, ctypes.c_int, dp, dp, dp, dp]
    lib.tn_measure_async_bytes.restype = sz
    lib.tn_measure_async_bytes.argtypes = [vp]
    lib.tn_measure_async_enable.restype = ctypes.c_int
    lib.tn_measure_async_enable.argtypes = [vp, vp, sz]
    lib.measure_corr_start.restype = ctypes.c_int
    lib.measure_corr_start.argtypes = [vp, ctypes.c_int]
    lib.measure_corr_finish.restype = ctypes.c_int
    lib.measure_corr_finish.argtypes = [vp, dp, dp, dp, dp]
    lib.tn_buckets.restype = ctypes.c_int
    lib.tn_buckets.argtypes = [vp, ctypes.c_int, ctypes.c_int, ip, ip, ip, ip]
    lib.tn_theta_precision.restype = ctypes.c_int
    lib.tn_theta_precision.argtypes = [vp, ctypes.c_int]
    lib.tn_stats.restype = ctypes.c_int
    lib.tn_stats.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]
    lib.measure_corr_noalloc.restype = ctypes.c_int
    lib.measure_corr_noalloc.argtypes = [vp, ctypes.c_int, dp, dp, dp, dp]
    lib.mps_free.restype = ctypes.c_int
    lib.mps_free.argtypes = [vp]
    lib.mps_last_error.restype = ctypes.c_char_p
    lib.mps_last_error.argtypes = []
    lib.mps_instance_tensor_capacity.restype = sz
    lib.mps_instance_tensor_capacity.argtypes = [vp]
    lib.mps_instance_lambda_capacity.restype = sz
    lib.mps_instance_lambda_capacity.argtypes = [vp]
    lib.mps_get_instance.restype = ctypes.c_int
    lib.mps_get_instance.argtypes = [vp, ctypes.c_int, ip, dp, dp, dp, dp]
    lib.mps_set_instance.restype = ctypes.c_int
    lib.mps_set_instance.argtypes = [vp, ctypes.c_int, ip, dp, dp, ctypes.c_double]
    lib.mps_replicate.restype = ctypes.c_int
    lib.mps_replicate.argtypes = [vp, ctypes.c_int]
    lib.tn_gate.restype = ctypes.c_int
    lib.tn_gate.argtypes = [ctypes.c_int, ctypes.POINTER(TnModel), ctypes.c_int, ctypes.c_double, dp]
    lib.tn_prof_enable.restype = ctypes.c_int
    lib.tn_prof_enable.argtypes = [vp, ctypes.c_int]
    lib.tn_graph_enable.restype = ctypes.c_int
    lib.tn_graph_enable.argtypes = [vp, ctypes.c_int]
    lib.tn_overlap.restype = ctypes.c_int
    lib.tn_overlap.argtypes = [vp, ctypes.c_int]
    lib.tn_schedule.restype = ctypes.c_int
    lib.tn_schedule.argtypes = [vp, ctypes.c_int]
    lib.tn_tuning.restype = ctypes.c_int
    lib.tn_tuning.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_float)]
    lib.tn_prof_query.restype = ctypes.c_int
    lib.tn_prof_query.argtypes = [vp, ctypes.c_int, dp, ctypes.POINTER(ctypes.c_longlong)]
    lib.tn_prof_busy.restype = ctypes.c_int
    lib.tn_prof_busy.argtypes = [vp, ctypes.c_int, dp]
    _lib = lib
    return lib
