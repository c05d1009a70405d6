"""ctypes declarations of the C ABI in include/muca.h (argument marshalling only).

The product path has no fallback: if libmuca.so is missing this module
raises, and nothing in the package computes any step of the method itself.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmuca.so")

MUCA_OK = 0
MUCA_ERR_INVALID_ARG = 1
MUCA_ERR_OUT_OF_MEMORY = 2
MUCA_ERR_DEVICE = 3
MUCA_ERR_OVERFLOW = 4
MUCA_ERR_NOT_CONVERGED = 5
MUCA_ERR_STATE = 6
MUCA_PENDING = 7
STATUS_NAMES = {
    0: "MUCA_OK", 1: "MUCA_ERR_INVALID_ARG", 2: "MUCA_ERR_OUT_OF_MEMORY", 3: "MUCA_ERR_DEVICE",
    4: "MUCA_ERR_OVERFLOW", 5: "MUCA_ERR_NOT_CONVERGED", 6: "MUCA_ERR_STATE", 7: "MUCA_PENDING",
}
MUCA_MAX_L = 128
MUCA_FLAG_GENERIC_KERNEL = 0x10000
MUCA_FLAG_FAST_KERNEL = 0x20000
KERNEL_GENERIC, KERNEL_FAST, KERNEL_SPLIT, KERNEL_WIDE, KERNEL_WIDE_SPLIT = 0, 1, 2, 3, 4


class MucaParams(ctypes.Structure):
    _fields_ = [("L", ctypes.c_uint32), ("walkers", ctypes.c_uint32),
                ("seed", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class MucaInfo(ctypes.Structure):
    _fields_ = [("attempts", ctypes.c_uint64), ("hist_sum", ctypes.c_uint64),
                ("sweep_counter", ctypes.c_uint64), ("position", ctypes.c_uint64),
                ("iteration", ctypes.c_uint32),
                ("visited_bins", ctypes.c_uint32), ("flatness", ctypes.c_double),
                ("kl_divergence", ctypes.c_double), ("chebyshev", ctypes.c_double),
                ("kernel_ms", ctypes.c_double), ("kernel_launches", ctypes.c_uint32),
                ("kernel_variant", ctypes.c_uint32), ("width", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_P = ctypes.c_void_p
_SZ = ctypes.c_size_t
_U32 = ctypes.c_uint32
_INT = ctypes.c_int

class Schedule(ctypes.Structure):
    _fields_ = [("z", ctypes.c_double), ("growth", ctypes.c_double), ("dk_flat", ctypes.c_double),
                ("dc_flat", ctypes.c_double), ("f_therm", ctypes.c_uint32), ("w_min", ctypes.c_uint32),
                ("max_iterations", ctypes.c_uint32), ("stop_rule", ctypes.c_uint32)]


class ScheduleStep(ctypes.Structure):
    _fields_ = [("therm_attempts", ctypes.c_uint64), ("update_attempts", ctypes.c_uint64),
                ("kl_divergence", ctypes.c_double), ("chebyshev", ctypes.c_double),
                ("flatness", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("width", ctypes.c_uint32), ("covered", ctypes.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerConfig(ctypes.Structure):
    _fields_ = [("mem_cap_bytes", ctypes.c_uint64), ("max_active_walkers", ctypes.c_uint64),
                ("batch_flags", ctypes.c_uint32), ("policy", ctypes.c_uint32),
                ("max_wait_s", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("min_flatness", ctypes.c_double),
                ("L", ctypes.c_uint32), ("walkers", ctypes.c_uint32), ("seed", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("iter_therm", ctypes.c_uint32),
                ("iter_sweeps", ctypes.c_uint32), ("max_iterations", ctypes.c_uint32),
                ("prod_therm", ctypes.c_uint32), ("prod_sweeps", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class Result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("attempts", ctypes.c_uint64),
                ("flatness", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_weights", ctypes.c_double),
                ("t_done", ctypes.c_double), ("status", ctypes.c_int32),
                ("iterations", ctypes.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerCounters(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("resident_bytes", ctypes.c_uint64), ("active_walkers", ctypes.c_uint64),
                ("attempts", ctypes.c_uint64), ("clock_s", ctypes.c_double),
                ("queued", ctypes.c_uint32), ("active", ctypes.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (restype, argtypes); every function declared in include/muca.h
PROTOTYPES = {
    "muca_state_bytes": (_SZ, [ctypes.POINTER(MucaParams)]),
    "muca_create": (_INT, [ctypes.POINTER(MucaParams), _P, _P, _SZ, ctypes.POINTER(_P)]),
    "muca_destroy": (_INT, [_P]),
    "muca_iterate": (_INT, [_P, _U32, _U32, ctypes.POINTER(MucaInfo)]),
    "muca_production": (_INT, [_P, _U32, _U32, ctypes.POINTER(MucaInfo)]),
    "muca_histogram": (_INT, [_P, _P, _SZ]),
    "muca_log_weights": (_INT, [_P, _P, _SZ]),
    "muca_set_log_weights": (_INT, [_P, _P, _SZ]),
    "muca_thresholds": (_INT, [_P, _P, _SZ]),
    "muca_energies": (_INT, [_P, _P, _SZ]),
    "muca_spins": (_INT, [_P, _P, _SZ]),
    "muca_log_dos": (_INT, [_P, _INT, _P, _SZ]),
    "muca_last_info": (_INT, [_P, ctypes.POINTER(MucaInfo)]),
    "muca_last_error": (ctypes.c_char_p, [_P]),
    "muca_checkpoint_bytes": (_SZ, [_P]),
    "muca_checkpoint": (_INT, [_P, _P, _SZ]),
    "muca_restore": (_INT, [_P, _P, _SZ]),
    "muca_iterate_attempts": (_INT, [_P, ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(MucaInfo)]),
    "muca_production_attempts": (_INT, [_P, ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.POINTER(MucaInfo)]),
    "muca_run_schedule": (_INT, [_P, ctypes.POINTER(Schedule), ctypes.POINTER(ScheduleStep), _U32,
                                 ctypes.POINTER(_U32)]),
    "muca_jackknife_log_dos": (_INT, [_U32, _U32, _P, _P, _INT, _P, _P]),
    "muca_canonical": (_INT, [_U32, _U32, _P, _P, _U32, _P, _P, _P, _P, _P]),
    "muca_batch_create": (_INT, [ctypes.POINTER(_P), _U32, _P, _U32, ctypes.POINTER(_P)]),
    "muca_batch_run": (_INT, [_P, _P, _P, _P, ctypes.POINTER(MucaInfo)]),
    "muca_batch_set_members": (_INT, [_P, ctypes.POINTER(_P), _U32]),
    "muca_batch_submit": (_INT, [_P, _P, _P, _P]),
    "muca_batch_query": (_INT, [_P]),
    "muca_batch_finish": (_INT, [_P, ctypes.POINTER(MucaInfo)]),
    "muca_batch_destroy": (_INT, [_P]),
    "muca_batch_last_error": (ctypes.c_char_p, [_P]),
    "muca_server_create": (_INT, [ctypes.POINTER(ServerConfig), ctypes.POINTER(_P)]),
    "muca_server_submit": (_INT, [_P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
    "muca_server_progress": (_INT, [_P, ctypes.POINTER(_U32)]),
    "muca_server_take": (_INT, [_P, ctypes.c_uint64, ctypes.POINTER(Result), _P, ctypes.c_size_t]),
    "muca_server_stats": (_INT, [_P, ctypes.POINTER(ServerCounters)]),
    "muca_server_destroy": (_INT, [_P]),
    "muca_server_last_error": (ctypes.c_char_p, [_P]),
    "muca_probe_issue_rate": (_INT, [_U32, _U32, _U32, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_uint64)]),
    "muca_production_static": (_INT, [ctypes.POINTER(MucaParams), ctypes.c_uint64, _U32, _U32, _P, _P, _P, _P,
                                      _P]),
}
MUCA_STATIC_SCRATCH_BYTES = 655872

MUCA_BATCH_SKIP = 0
MUCA_BATCH_ITERATE = 1
MUCA_BATCH_PRODUCTION = 2
MUCA_SERVE_FIFO = 0
MUCA_SERVE_SMALLEST_FIRST = 1
MUCA_STOP_KL = 0
MUCA_STOP_CHEBYSHEV = 1
MUCA_PROBE_OPS = {"v_add_u32": 0, "v_bitop3_b32 (xor3)": 1, "v_mul_lo_u32": 2, "v_mul_hi_u32": 3,
                  "v_mad_u64_u32": 4}
MUCA_BATCH_GRAPH = 0x1
MUCA_BATCH_AUTOTUNE = 0x2

_lib = None


def _share_torch_runtime():
    """Load torch (when installed) before libmuca.so.

    torch ships its own HIP runtime, which its libraries find under the name
    libamdhip64.so.  libmuca.so asks for libamdhip64.so.7, the soname torch's
    copy also carries: loaded after torch, libmuca binds to torch's runtime;
    loaded first, it would pull in the system runtime and torch would then
    load its own beside it -- two HIP runtimes in one process, and the second
    to open the device finds none.  Loading torch first keeps one runtime,
    whose device memory and streams both sides then share.
    """
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def lib():
    """Load libmuca.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmuca.so not found at %s; build it with "
                              "`python -m paper_1707_00919_amd.build`" % LIB_PATH)
        _share_torch_runtime()
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib
