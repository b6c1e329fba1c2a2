"""ctypes declarations of the C ABI in include/ipfp.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libipfp.so")

F64, F32, BF16, FP8E4M3 = 0, 1, 2, 3
PATH_FUSED, PATH_PLAIN = 0, 1
NOALLOC_BYTES = 64 << 20     # IPFP_NOALLOC_BYTES

OK, NOT_CONVERGED = 0, 1
EINVAL, EBUDGET, EHIP, ENONFINITE, ECANCELLED, EBUSY, ENOTFOUND = -1, -2, -3, -4, -5, -6, -7

c_dp = ctypes.POINTER(ctypes.c_double)


class Market(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64), ("M", ctypes.c_int64), ("d", ctypes.c_int64),
        ("in_dtype", ctypes.c_int),
        ("U", ctypes.c_void_p), ("Q", ctypes.c_void_p),
        ("V", ctypes.c_void_p), ("P", ctypes.c_void_p),
        ("ld_x", ctypes.c_int64), ("ld_y", ctypes.c_int64),
        ("n", ctypes.c_void_p), ("m", ctypes.c_void_p),
        ("sigma", ctypes.c_double),
        ("scale_x", ctypes.c_void_p), ("scale_y", ctypes.c_void_p),
    ]


class Options(ctypes.Structure):
    _fields_ = [
        ("path", ctypes.c_int), ("compute", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("max_sweeps", ctypes.c_int32), ("check_every", ctypes.c_int32),
        ("splits", ctypes.c_int32), ("splits_col", ctypes.c_int32),
        ("tile_rows", ctypes.c_int32),
        ("b0", ctypes.c_void_p),
        ("use_graph", ctypes.c_int32), ("time_passes", ctypes.c_int32),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("a", ctypes.c_void_p), ("b", ctypes.c_void_p),
        ("res_hist", c_dp), ("res_cap", ctypes.c_int32),
        ("sweeps", ctypes.c_int32), ("n_res", ctypes.c_int32),
        ("final_res", ctypes.c_double), ("setup_ms", ctypes.c_double),
        ("loop_ms", ctypes.c_double), ("pass_ms", ctypes.c_double),
        ("pass_launches", ctypes.c_int32), ("fixups", ctypes.c_int32),
    ]


class Plan(ctypes.Structure):
    _fields_ = [
        ("kpad", ctypes.c_int64), ("rows_per_workgroup", ctypes.c_int32),
        ("auto_splits_row", ctypes.c_int32), ("auto_splits_col", ctypes.c_int32),
        ("splits_row", ctypes.c_int32), ("splits_col", ctypes.c_int32),
        ("blocks_row", ctypes.c_int64), ("blocks_col", ctypes.c_int64),
        ("footprint_bytes", ctypes.c_size_t),
    ]


class ServerOptions(ctypes.Structure):
    _fields_ = [
        ("arena_bytes", ctypes.c_size_t), ("max_active", ctypes.c_int32),
        ("lanes", ctypes.c_int32), ("chunk", ctypes.c_int32), ("compute", ctypes.c_int),
        ("tile_rows", ctypes.c_int32), ("lane_pairs", ctypes.c_double * 3),
        ("lane_blocks", ctypes.c_int32), ("aging_ms", ctypes.c_double),
    ]


REQ_QUEUED, REQ_RUNNING, REQ_FINISHED = 0, 1, 2


class RequestInfo(ctypes.Structure):
    _fields_ = [
        ("state", ctypes.c_int32), ("code", ctypes.c_int32), ("lane", ctypes.c_int32),
        ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
        ("t_done", ctypes.c_double),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64),
        ("finished", ctypes.c_int64), ("queued", ctypes.c_int64),
        ("active", ctypes.c_int64), ("rounds", ctypes.c_int64),
        ("arena_bytes", ctypes.c_size_t), ("arena_used", ctypes.c_size_t),
        ("arena_peak", ctypes.c_size_t), ("pair_evals", ctypes.c_double),
    ]


# name -> (restype, argtypes); every symbol the header declares
SIGNATURES = {
    "ipfp_abi_version": (ctypes.c_int, []),
    "ipfp_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "ipfp_default_options": (None, [ctypes.POINTER(Options)]),
    "ipfp_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                   ctypes.c_size_t]),
    "ipfp_destroy": (None, [ctypes.c_void_p]),
    "ipfp_footprint": (ctypes.c_int, [ctypes.POINTER(Market), ctypes.POINTER(Options),
                                      ctypes.POINTER(ctypes.c_size_t)]),
    "ipfp_plan_market": (ctypes.c_int, [ctypes.POINTER(Market), ctypes.POINTER(Options),
                                        ctypes.POINTER(Plan)]),
    "ipfp_solve_market": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Market),
                                         ctypes.POINTER(Options), ctypes.POINTER(Result),
                                         ctypes.c_void_p]),
    "ipfp_solve_market_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Market),
                                                 ctypes.POINTER(Options),
                                                 ctypes.POINTER(Result), ctypes.c_void_p]),
    "ipfp_solve_market_phi": (ctypes.c_int, [
        ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
        ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
        ctypes.POINTER(Options), ctypes.POINTER(Result), ctypes.c_void_p]),
    "ipfp_market_open": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Market),
                                        ctypes.POINTER(Options),
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]),
    "ipfp_market_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int), ctypes.c_void_p]),
    "ipfp_market_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.POINTER(Result), ctypes.c_void_p]),
    "ipfp_market_close": (None, [ctypes.c_void_p]),
    "ipfp_mu_pairs": (ctypes.c_int, [
        ctypes.c_void_p, ctypes.POINTER(Market), ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
        ctypes.c_void_p]),
    "ipfp_pack_side": (ctypes.c_int, [
        ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
    "ipfp_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Market),
                                 ctypes.POINTER(Options), ctypes.POINTER(Options),
                                 ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "ipfp_margin_residuals": (ctypes.c_int, [
        ctypes.c_void_p, ctypes.POINTER(Market), ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
        ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "ipfp_stable_factors": (ctypes.c_int, [
        ctypes.c_void_p, ctypes.POINTER(Market), ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "ipfp_market_topk": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ipfp_market_gradient": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                            ctypes.c_int64, ctypes.c_void_p]),
    "ipfp_default_server_options": (None, [ctypes.POINTER(ServerOptions)]),
    "ipfp_server_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerOptions),
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "ipfp_server_destroy": (None, [ctypes.c_void_p]),
    "ipfp_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Market),
                                   ctypes.POINTER(Options), ctypes.POINTER(Result),
                                   ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p]),
    "ipfp_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64,
                                 ctypes.POINTER(RequestInfo)]),
    "ipfp_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double,
                                 ctypes.POINTER(RequestInfo)]),
    "ipfp_cancel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "ipfp_server_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerStats)]),
    "ipfp_clock_ms": (ctypes.c_double, []),
    "ipfp_probe": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                                  ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
}

PROBE_EXP2, PROBE_MFMA_BF16, PROBE_MFMA_FP8, PROBE_MFMA_F32, PROBE_HBM_READ = 0, 1, 2, 3, 4
PROBE_MFMA_BF16_2W, PROBE_MFMA_BF16_EPI, PROBE_MFMA_FP8_EPI = 5, 6, 7

_LIB = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libipfp.so and declare every entry point. Raises when the library
    has not been built: there is no fallback implementation."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_2411_19214_amd.build`"
            " (the IPFP kernels exist only as HIP code)")
    # The library must share the HIP runtime torch uses (device pointers and
    # streams cross the boundary). torch ships its own libamdhip64 under the
    # same soname; loading torch first makes the dynamic linker reuse it, where
    # loading this library first would map a second runtime from /opt/rocm.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib
