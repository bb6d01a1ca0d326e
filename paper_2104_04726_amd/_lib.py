"""ctypes declarations for libtucker_mi355x.so (the C ABI of include/tucker.h).

The library is loaded from this package directory; there is no fallback implementation:
a missing or unloadable library raises at first use.
"""

from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("TUCKER_LIB") or os.path.join(HERE, "libtucker_mi355x.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "tucker.h")

OK, ERR_INVALID_ARG, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_NUMERICAL, ERR_UNSUPPORTED, ERR_TIMEOUT = range(7)
FP32, BF16, FP16, FP8_E4M3 = range(4)
START_THOSVD, START_STHOSVD = range(2)


class Options(C.Structure):
    _fields_ = [
        ("device", C.c_int),
        ("stream", C.c_void_p),
        ("precision", C.c_int),
        ("refine_sweeps", C.c_int),
        ("inner_iters", C.c_int),
        ("init_iters", C.c_int),
        ("inner_tol", C.c_double),
        ("use_graphs", C.c_int),
        ("hbm_budget_bytes", C.c_size_t),
        ("seed", C.c_uint64),
        ("timing", C.c_int),
        ("wait_spin_limit", C.c_int64),
        ("start", C.c_int),
        ("autotune", C.c_int),
        ("pp_tol", C.c_double),
        ("timing_stages", C.c_uint32),
        ("oversample", C.c_int),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("init_ms", C.c_double),
        ("sweeps_ms", C.c_double),
        ("final_fit_ms", C.c_double),
        ("fit_gram", C.c_double),
        ("sweeps", C.c_int),
        ("refine_sweeps", C.c_int),
        ("chol_shifts", C.c_int),
        ("orth_second_passes", C.c_int),
        ("wait_timeouts", C.c_int),
        ("oi_steps_init", C.c_int),
        ("oi_steps_sweeps", C.c_int),
        ("oi_residual_max", C.c_double),
        ("pp_sweeps", C.c_int),
        ("pp_refs", C.c_int),
        ("rr_sweeps", C.c_int),
        ("workspace_bytes", C.c_size_t),
        ("stage_ms", C.c_double * 12),
        ("stage_calls", C.c_int * 12),
    ]


MAX_ORDER = 8


class ServerOptions(C.Structure):
    _fields_ = [
        ("device", C.c_int),
        ("slots", C.c_int),
        ("hbm_budget_bytes", C.c_size_t),
        ("inner_iters", C.c_int),
        ("init_iters", C.c_int),
        ("seed", C.c_uint64),
        ("use_graphs", C.c_int),
        ("autotune", C.c_int),
        ("group_requests", C.c_int),
    ]


class Request(C.Structure):
    _fields_ = [
        ("host_tensor", C.c_void_p),
        ("ndim", C.c_int),
        ("dims", C.c_int64 * MAX_ORDER),
        ("ranks", C.c_int64 * MAX_ORDER),
        ("max_iters", C.c_int),
        ("tol", C.c_double),
        ("precision", C.c_int),
        ("refine_sweeps", C.c_int),
        ("tag", C.c_uint64),
        ("host_core", C.c_void_p),
        ("host_factors", C.c_void_p * MAX_ORDER),
    ]


class ServedResult(C.Structure):
    _fields_ = [
        ("status", C.c_int),
        ("fit", C.c_double),
        ("sweeps", C.c_int),
        ("tag", C.c_uint64),
        ("slot", C.c_int),
        ("footprint_bytes", C.c_size_t),
        ("t_submit", C.c_double),
        ("t_admit", C.c_double),
        ("t_start", C.c_double),
        ("t_finish", C.c_double),
        ("error", C.c_char * 160),
    ]


class ServerStats(C.Structure):
    _fields_ = [
        ("submitted", C.c_int64),
        ("completed", C.c_int64),
        ("failed", C.c_int64),
        ("budget_bytes", C.c_size_t),
        ("peak_admitted_bytes", C.c_size_t),
        ("peak_running", C.c_int),
        ("grouped_requests", C.c_int64),
        ("group_launches", C.c_int64),
        ("grouped_products", C.c_int64),
    ]


STAGES = ["pass_a", "ttm_y1", "gram_1", "oi_1", "ttm_y2", "gram_2", "oi_2", "pass_c1", "ttm_c2", "small",
          "core", "reduce"]


_lib = None

I64P = C.POINTER(C.c_int64)
FPP = C.POINTER(C.c_void_p)


def _declare(lib):
    v = C.c_void_p
    lib.tucker_default_options.argtypes = [C.POINTER(Options)]
    lib.tucker_default_options.restype = None
    lib.tucker_validate.argtypes = [C.c_int, I64P, I64P, C.c_int, C.c_double]
    lib.tucker_workspace_size.argtypes = [C.c_int, I64P, I64P, C.c_int, C.POINTER(C.c_size_t)]
    lib.tucker_create.argtypes = [C.POINTER(Options), C.POINTER(v)]
    lib.tucker_destroy.argtypes = [v]
    lib.tucker_decompose.argtypes = [v, v, C.c_int, I64P, I64P, C.c_int, C.c_double, v, FPP,
                                     C.POINTER(C.c_double), C.POINTER(C.c_int)]
    lib.tucker_decompose_ex.argtypes = [v, v, C.c_int, I64P, I64P, C.c_int, C.c_double, FPP, v, FPP,
                                        C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int)]
    lib.tucker_reconstruct.argtypes = [v, v, FPP, C.c_int, I64P, I64P, v]
    lib.tucker_ttm.argtypes = [v, v, C.c_int, I64P, C.c_int, v, C.c_int64, v]
    lib.tucker_order_core.argtypes = [v, v, FPP, C.c_int, I64P, I64P, v, FPP, v]
    lib.tucker_quantize_core.argtypes = [v, v, C.c_int, I64P, I64P, C.c_int, v, v, C.POINTER(C.c_float)]
    lib.tucker_gram.argtypes = [v, v, C.c_int, I64P, C.c_int, v]
    lib.tucker_orthonormalize.argtypes = [v, v, C.c_int64, C.c_int64, v]
    lib.tucker_gram_tn64.argtypes = [v, v, C.c_int64, C.c_int64, v]
    lib.tucker_chol_inv.argtypes = [v, v, C.c_int64, v]
    lib.tucker_chol_inv_noalloc.argtypes = [v, v, C.c_int64, v]
    lib.tucker_sym_eig.argtypes = [v, v, C.c_int64, C.c_int64, v, v]
    lib.tucker_sumsq.argtypes = [v, v, C.c_int64, C.POINTER(C.c_double)]
    lib.tucker_set_timing.argtypes = [v, C.c_int, C.c_uint32]
    lib.tucker_autotune_dump.argtypes = [C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]
    lib.tucker_autotune_dump.restype = C.c_int
    lib.tucker_autotune_clear.argtypes = []
    lib.tucker_autotune_clear.restype = C.c_int
    lib.tucker_autotune_force.argtypes = [C.c_int, C.c_int]
    lib.tucker_autotune_force.restype = C.c_int
    lib.tucker_status_string.argtypes = [C.c_int]
    lib.tucker_status_string.restype = C.c_char_p
    lib.tucker_last_error.argtypes = [v]
    lib.tucker_last_error.restype = C.c_char_p
    lib.tucker_get_stats.argtypes = [v, C.POINTER(Stats)]
    lib.tucker_quantize.argtypes = [v, v, C.c_int64, C.c_int64, C.c_int, v, v]
    lib.tucker_ttm_lowp.argtypes = [v, v, C.c_int, I64P, C.c_int, v, C.c_int64, C.c_int, v]
    lib.tucker_gram_lowp.argtypes = [v, v, C.c_int, I64P, C.c_int, C.c_int, v]
    lib.tucker_default_server_options.argtypes = [C.POINTER(ServerOptions)]
    lib.tucker_default_server_options.restype = None
    lib.tucker_server_create.argtypes = [C.POINTER(ServerOptions), C.POINTER(v)]
    lib.tucker_server_submit.argtypes = [v, C.POINTER(Request), C.POINTER(C.c_uint64)]
    lib.tucker_server_wait.argtypes = [v, C.c_uint64, C.c_double, C.POINTER(ServedResult)]
    lib.tucker_server_get_stats.argtypes = [v, C.POINTER(ServerStats)]
    lib.tucker_server_destroy.argtypes = [v]
    for name in ("tucker_server_create", "tucker_server_submit", "tucker_server_wait", "tucker_server_get_stats",
                 "tucker_server_destroy"):
        getattr(lib, name).restype = C.c_int
    for name in ("tucker_validate", "tucker_workspace_size", "tucker_create", "tucker_destroy", "tucker_decompose",
                 "tucker_decompose_ex", "tucker_reconstruct", "tucker_ttm", "tucker_gram",
                 "tucker_order_core", "tucker_quantize_core",
                 "tucker_quantize", "tucker_ttm_lowp", "tucker_gram_lowp",
                 "tucker_orthonormalize", "tucker_gram_tn64", "tucker_chol_inv", "tucker_chol_inv_noalloc",
                 "tucker_sym_eig", "tucker_sumsq", "tucker_get_stats"):
        getattr(lib, name).restype = C.c_int


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run `python -m paper_2104_04726_amd.build`)")
        handle = C.CDLL(LIB_PATH)
        _declare(handle)
        _lib = handle
    return _lib


def header_functions():
    """Names of the functions declared in include/tucker.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tucker_[a-z0-9_]+)\s*\(", text)))


def i64(vals):
    arr = (C.c_int64 * len(vals))(*[int(v) for v in vals])
    return arr


def status_name(code: int) -> str:
    return lib().tucker_status_string(int(code)).decode()
