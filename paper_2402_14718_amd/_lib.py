"""ctypes declarations of the sbtrack C ABI (include/sbtrack.h).

Only marshalling lives here.  Loading fails loudly if the in-tree
libsbtrack.so has not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsbtrack.so")

SBT_OK = 0
SBT_EINVAL = -1
SBT_ENOMEM = -2
SBT_EDEVICE = -3
SBT_EUNSUPPORTED = -4

SBT_BSB = 0
SBT_DSB = 1
SBT_ASB = 2

SBT_KERNEL_AUTO = 0
SBT_KERNEL_RESIDENT = 1
SBT_KERNEL_STREAM = 2
SBT_KERNEL_STREAM_TILE = 3
SBT_KERNEL_STREAM_ROWS = 4
SBT_KERNEL_STREAM_MFMA = 5


class SbtHit(C.Structure):
    _fields_ = [("hit_id", C.c_int64), ("layer", C.c_int32), ("pad", C.c_int32),
                ("x", C.c_double), ("y", C.c_double), ("z", C.c_double)]


class SbtBuildParams(C.Structure):
    _fields_ = [("dphi_tan", C.c_double), ("z0_max", C.c_double), ("curv_max", C.c_double),
                ("dtheta_tan", C.c_double), ("dcurv_max", C.c_double), ("s_min", C.c_double),
                ("max_holes", C.c_int32), ("min_track_hits", C.c_int32),
                ("alpha", C.c_double), ("beta", C.c_double), ("gamma_", C.c_double),
                ("lambda_", C.c_double)]


class SbtQubo(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("a", C.POINTER(C.c_double)),
                ("row_ptr", C.POINTER(C.c_int64)), ("col", C.POINTER(C.c_int32)),
                ("b", C.POINTER(C.c_double)), ("trip_hits", C.POINTER(C.c_int64))]


class SbtSolveParams(C.Structure):
    _fields_ = [("a0", C.c_double), ("dt", C.c_double), ("c0", C.c_double),
                ("agents", C.c_int32), ("steps", C.c_int32), ("seed", C.c_uint64),
                ("event", C.c_int32), ("kernel", C.c_int32), ("energy_every", C.c_int32),
                ("tpb", C.c_int32), ("precision", C.c_int32), ("reserved", C.c_int32)]


class SbtAnnealParams(C.Structure):
    _fields_ = [("shots", C.c_int32), ("sweeps", C.c_int32), ("beta_hot", C.c_double),
                ("beta_cold", C.c_double), ("seed", C.c_uint64), ("threads", C.c_int32),
                ("reserved", C.c_int32)]


class SbtResult(C.Structure):
    _fields_ = [("T", C.POINTER(C.c_int8)), ("agent_energy", C.POINTER(C.c_double)),
                ("trace", C.POINTER(C.c_double)), ("x_final", C.POINTER(C.c_float)),
                ("y_final", C.POINTER(C.c_float)), ("energy", C.c_double),
                ("ising_offset", C.c_double), ("c0", C.c_double), ("best_agent", C.c_int32),
                ("kernel_used", C.c_int32), ("elapsed_s", C.c_double),
                ("agent_trace", C.POINTER(C.c_double)), ("trace_len", C.c_int32)]


class SbtDevQubo(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("a", C.c_void_p), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("b", C.c_void_p)]


class SbtDevResult(C.Structure):
    _fields_ = [("T", C.c_void_p), ("agent_energy", C.c_void_p), ("best_energy", C.c_void_p),
                ("best_agent", C.c_void_p), ("scalars", C.c_void_p), ("x_final", C.c_void_p),
                ("y_final", C.c_void_p), ("trace", C.c_void_p), ("step_begin", C.c_void_p),
                ("step_end", C.c_void_p), ("agent_trace", C.c_void_p)]


SBT_PREC_FP32 = 0
SBT_PREC_FP16 = 1
SBT_PREC_BF16 = 2
SBT_PREC_FP8 = 3
SBT_PREC_FP8_BLOCK = 4
SBT_PREC_BF16X2 = 5


class SbtDevBatch(C.Structure):
    _fields_ = [("n_events", C.c_int32), ("n", C.POINTER(C.c_int32)), ("nnz", C.POINTER(C.c_int64)),
                ("a", C.c_void_p), ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("b", C.c_void_p),
                ("target", C.c_void_p)]


class SbtDevBatchResult(C.Structure):
    _fields_ = [("best_energy", C.c_void_p), ("best_agent", C.c_void_p), ("best_T", C.c_void_p),
                ("agent_energy", C.c_void_p), ("offset", C.c_void_p), ("trace", C.c_void_p),
                ("step_begin", C.c_void_p), ("step_end", C.c_void_p), ("agent_T", C.c_void_p),
                ("agent_x", C.c_void_p), ("agent_trace", C.c_void_p),
                ("ckpt_clock", C.c_void_p)]


class SbtBatchTuning(C.Structure):
    _fields_ = [("split_n", C.c_int32), ("tail_words", C.c_int32), ("fill", C.c_double),
                ("band_rows", C.c_int32), ("from_cache", C.c_int32), ("reserved", C.c_int32)]


class SbtBatchResult(C.Structure):
    _fields_ = [("energy", C.POINTER(C.c_double)), ("best_agent", C.POINTER(C.c_int32)),
                ("T", C.POINTER(C.c_int8)), ("agent_energy", C.POINTER(C.c_double)),
                ("trace", C.POINTER(C.c_double)), ("elapsed_s", C.c_double),
                ("agent_trace", C.POINTER(C.c_double))]


# (name, restype, argtypes) of every exported function, as in sbtrack.h
EXPORTS = [
    ("sbt_last_error", C.c_char_p, []),
    ("sbt_version", C.c_char_p, []),
    ("sbt_build_params_default", None, [C.POINTER(SbtBuildParams)]),
    ("sbt_build_qubo", C.c_int, [C.POINTER(SbtHit), C.c_int64, C.POINTER(SbtBuildParams),
                                 C.POINTER(C.POINTER(SbtQubo))]),
    ("sbt_qubo_free", None, [C.POINTER(SbtQubo)]),
    ("sbt_energy", C.c_int, [C.POINTER(SbtQubo), C.POINTER(C.c_int8), C.POINTER(C.c_double)]),
    ("sbt_build_qubo_gpu", C.c_int, [C.POINTER(SbtHit), C.c_int64, C.POINTER(SbtBuildParams),
                                     C.POINTER(C.POINTER(SbtQubo)), C.POINTER(C.c_double)]),
    ("sbt_anneal_params_default", None, [C.POINTER(SbtAnnealParams)]),
    ("sbt_anneal_cpu", C.c_int, [C.POINTER(SbtQubo), C.POINTER(SbtAnnealParams),
                                 C.POINTER(C.c_int8), C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("sbt_phi_order", C.c_int, [C.POINTER(SbtQubo), C.POINTER(SbtHit), C.c_int64,
                                C.POINTER(C.c_int32)]),
    ("sbt_qubo_permute", C.c_int, [C.POINTER(SbtQubo), C.POINTER(C.c_int32),
                                   C.POINTER(C.POINTER(SbtQubo))]),
    ("sbt_solve_params_default", None, [C.POINTER(SbtSolveParams)]),
    ("sbt_solve", C.c_int, [C.POINTER(SbtQubo), C.c_int, C.POINTER(SbtSolveParams),
                            C.POINTER(SbtResult)]),
    ("sbt_workspace_bytes", C.c_size_t, [C.c_int32, C.c_int64, C.c_int,
                                         C.POINTER(SbtSolveParams)]),
    ("sbt_select_kernel", C.c_int, [C.c_int32, C.c_int64, C.c_int32, C.c_int,
                                    C.POINTER(SbtSolveParams)]),
    ("sbt_solve_dev", C.c_int, [C.POINTER(SbtDevQubo), C.c_int32, C.c_int,
                                C.POINTER(SbtSolveParams), C.c_void_p, C.c_size_t,
                                C.POINTER(SbtDevResult), C.c_void_p]),
    ("sbt_solve_dev_noalloc", C.c_int, [C.POINTER(SbtDevQubo), C.c_int32, C.c_int,
                                        C.POINTER(SbtSolveParams), C.POINTER(SbtDevResult),
                                        C.c_void_p]),
    ("sbt_top_k_dev", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                C.c_void_p]),
    ("sbt_batch_workspace_bytes", C.c_size_t, [C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                               C.c_int32, C.POINTER(SbtSolveParams)]),
    ("sbt_batch_workspace_bytes_tuned", C.c_size_t,
     [C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.c_int32, C.POINTER(SbtSolveParams),
      C.POINTER(SbtBatchTuning)]),
    ("sbt_batch_tuning_default", None, [C.POINTER(SbtBatchTuning)]),
    ("sbt_batch_tuning_key", C.c_int, [C.POINTER(C.c_int32), C.c_int32, C.c_int, C.c_int,
                                       C.c_int32, C.c_char_p, C.c_size_t]),
    ("sbt_batch_tuning_lookup", C.c_int, [C.POINTER(C.c_int32), C.c_int32, C.c_int, C.c_int,
                                          C.c_int32, C.POINTER(SbtBatchTuning)]),
    ("sbt_batch_plan_tuned", C.c_int, [C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.c_int32,
                                       C.POINTER(C.c_double), C.c_int32,
                                       C.POINTER(SbtSolveParams), C.POINTER(SbtBatchTuning),
                                       C.c_void_p, C.c_size_t, C.c_void_p]),
    ("sbt_batch_run_tuned", C.c_int, [C.POINTER(SbtDevBatch), C.c_int, C.c_int,
                                      C.POINTER(SbtSolveParams), C.POINTER(SbtBatchTuning),
                                      C.c_void_p, C.c_size_t, C.POINTER(SbtDevBatchResult),
                                      C.c_void_p]),
    ("sbt_batch_plan", C.c_int, [C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.c_int32,
                                 C.POINTER(C.c_double), C.c_int32, C.POINTER(SbtSolveParams),
                                 C.c_void_p, C.c_size_t, C.c_void_p]),
    ("sbt_batch_run", C.c_int, [C.POINTER(SbtDevBatch), C.c_int, C.c_int,
                                C.POINTER(SbtSolveParams), C.c_void_p, C.c_size_t,
                                C.POINTER(SbtDevBatchResult), C.c_void_p]),
    ("sbt_wall_clock_hz", C.c_int, [C.POINTER(C.c_double)]),
    ("sbt_solve_batch", C.c_int, [C.POINTER(C.POINTER(SbtQubo)), C.c_int32, C.c_int, C.c_int,
                                  C.POINTER(SbtSolveParams), C.POINTER(SbtBatchResult)]),
    ("sbt_c0_scan", C.c_int, [C.POINTER(SbtQubo), C.c_int, C.c_int, C.POINTER(SbtSolveParams),
                              C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_double),
                              C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
]

_LIB = None


class SbtError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"sbtrack error {code}: {message}")
        self.code = code


def load() -> C.CDLL:
    """Load the in-tree library (build it with paper_2402_14718_amd.build)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2402_14718_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, res, args in EXPORTS:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def check(rc: int) -> None:
    if rc != SBT_OK:
        msg = load().sbt_last_error().decode("utf-8", "replace")
        raise SbtError(rc, msg)
