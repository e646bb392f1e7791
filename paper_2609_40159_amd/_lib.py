"""ctypes declarations for librwtrsv.so (the C ABI in include/rwtrsv.h).

Argument marshalling only: every step of the solve path runs in the HIP
library.  Importing this module fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librwtrsv.so")

OK = 0
STATUS = {
    0: "OK", -1: "INVALID_ARG", -2: "NOT_LOWER", -3: "UNSORTED_OR_DUP", -4: "MISSING_DIAG",
    -5: "ZERO_DIAG", -6: "BAD_ROWSET", -7: "BUFFER_TOO_SMALL", -8: "TOO_LARGE", -9: "DEADLOCK",
    -10: "HIP",
}
F64, F32 = 0, 1
ALGO = {"auto": 0, "level": 1, "syncfree": 2, "walk": 3}
ALGO_NAME = {v: k for k, v in ALGO.items()}


class RwtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


class Csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("pad_", C.c_int32), ("nnz", C.c_int64),
                ("rowptr", C.c_void_p), ("colidx", C.c_void_p), ("vals", C.c_void_p),
                ("dt", C.c_int32), ("pad2_", C.c_int32)]


class LevelStats(C.Structure):
    _fields_ = [("num_levels", C.c_int32), ("thin_count", C.c_int32), ("S1", C.c_uint64),
                ("S2_lo", C.c_uint64), ("S2_hi", C.c_uint64), ("cv", C.c_double),
                ("cv_rows", C.c_double), ("alc", C.c_double), ("arl", C.c_double),
                ("air", C.c_double), ("thin_threshold", C.c_double),
                ("max_level_rows", C.c_int32), ("pad_", C.c_int32)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_ if not f.startswith("pad")}
        d["S2"] = int(self.S2_lo) | (int(self.S2_hi) << 64)
        return d


class PlanOpts(C.Structure):
    _fields_ = [("algo", C.c_int32), ("block_rows", C.c_int32), ("lanes_per_row", C.c_int32),
                ("narrow_rows", C.c_int32), ("kmax", C.c_int32), ("watchdog_ms", C.c_int32),
                ("rhs_chunk", C.c_int32), ("tune_cols", C.c_int32),
                ("stage_outside", C.c_int32)]


class PlanInfo(C.Structure):
    _fields_ = [("stats", LevelStats), ("algo_fwd", C.c_int32), ("algo_bwd", C.c_int32),
                ("block_rows", C.c_int32), ("lanes_per_row", C.c_int32),
                ("narrow_rows", C.c_int32), ("num_blocks", C.c_int32), ("grid", C.c_int32),
                ("rhs_chunk", C.c_int32), ("stage_outside", C.c_int32),
                ("tuned_ms_level", C.c_double),
                ("tuned_ms_syncfree", C.c_double), ("tuned_ms_walk", C.c_double),
                ("chunk_rounds", C.c_double)]


class BatchMatrix(C.Structure):
    _fields_ = [("L", Csr), ("B", C.c_void_p), ("X", C.c_void_p), ("k", C.c_int32),
                ("block_rows", C.c_int32), ("ldb", C.c_int64), ("ldx", C.c_int64)]


class BatchDesc(C.Structure):
    _fields_ = [("count", C.c_int32), ("num_cand", C.c_int32), ("mats", C.c_void_p),
                ("h_cand_mat", C.c_void_p), ("d_cand_ptr", C.c_void_p),
                ("d_cand_rows", C.c_void_p), ("d_cand_targets", C.c_void_p),
                ("cand_rows_cap", C.c_int32), ("pattern_cap", C.c_int32),
                ("watchdog_ms", C.c_int32), ("cand_mode", C.c_int32)]


class CandStats(C.Structure):
    _fields_ = [("num_levels", C.c_int32), ("valid", C.c_int32), ("S1", C.c_uint64),
                ("S2_lo", C.c_uint64), ("S2_hi", C.c_uint64), ("cv", C.c_double)]


class BatchInfo(C.Structure):
    _fields_ = [("tasks", C.c_int32), ("solve_tasks", C.c_int32), ("grid", C.c_int32),
                ("captured", C.c_int32), ("create_ms", C.c_double), ("sweep_cands", C.c_int32),
                ("pattern_slot", C.c_int32)]


class GenParams(C.Structure):
    _fields_ = [("alpha", C.c_double), ("thin_stop", C.c_double), ("max_dist", C.c_int32),
                ("max_moves", C.c_int32), ("max_steps", C.c_int32), ("pad_", C.c_int32)]


class GenResult(C.Structure):
    _fields_ = [("moves", C.c_int32), ("steps", C.c_int32), ("stop", C.c_int32),
                ("levels", C.c_int32), ("thin", C.c_int32), ("thin0", C.c_int32),
                ("rejected", C.c_int32), ("pad_", C.c_int32), ("threshold", C.c_double),
                ("S1", C.c_uint64), ("S2_lo", C.c_uint64), ("S2_hi", C.c_uint64),
                ("cv", C.c_double)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("pad_", "S2_lo", "S2_hi")}
        d["S2"] = int(self.S2_lo) | (int(self.S2_hi) << 64)
        return d


class EnvParams(C.Structure):
    _fields_ = [("alpha", C.c_double), ("thin_stop", C.c_double), ("reward_alpha", C.c_double),
                ("eps", C.c_double), ("decay", C.c_double), ("max_dist", C.c_int32),
                ("search_window", C.c_int32), ("dist_threshold", C.c_int32),
                ("max_steps", C.c_int32), ("stall_steps", C.c_int32), ("keep_top", C.c_int32)]


class EnvResult(C.Structure):
    _fields_ = [("outcome", C.c_int32), ("node", C.c_int32), ("src", C.c_int32),
                ("tgt", C.c_int32), ("collapsed", C.c_int32), ("done", C.c_int32),
                ("steps", C.c_int32), ("moves", C.c_int32), ("levels", C.c_int32),
                ("thin", C.c_int32), ("thin0", C.c_int32), ("pad_", C.c_int32),
                ("reward", C.c_double), ("r_cv", C.c_double), ("r_cp", C.c_double),
                ("r_rwdist", C.c_double), ("r_abandon", C.c_double), ("cv", C.c_double),
                ("cv_rows", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


P = C.c_void_p
I32 = C.c_int32
I64 = C.c_int64
SZ = C.c_size_t
# largest n of rwt_apply_M_noalloc (RWT_APPLY_M_NOALLOC_MAX_N)
APPLY_M_NOALLOC_MAX_N = 1 << 22

# name -> (restype, argtypes); every symbol include/rwtrsv.h declares
SIGNATURES = {
    "rwt_last_error_string": (C.c_char_p, []),
    "rwt_last_hip_error": (C.c_int, []),
    "rwt_version": (C.c_char_p, []),
    "rwt_source_hash": (C.c_char_p, []),
    "rwt_validate_ws": (SZ, []),
    "rwt_validate": (C.c_int, [C.POINTER(Csr), P, SZ, C.POINTER(I32), P]),
    "rwt_analyze_ws": (C.c_int, [C.POINTER(Csr), C.POINTER(SZ)]),
    "rwt_analyze": (C.c_int, [C.POINTER(Csr), P, SZ, P, P, P, P, P, P, C.POINTER(LevelStats), P]),
    "rwt_rewrite_ws": (C.c_int, [C.POINTER(Csr), I32, C.POINTER(SZ)]),
    "rwt_rewrite_symbolic": (C.c_int, [C.POINTER(Csr), P, P, P, I32, P, SZ, P, P,
                                       C.POINTER(I64), P]),
    "rwt_rewrite_numeric": (C.c_int, [C.POINTER(Csr), P, P, P, I32, P, I32, I64,
                                      C.POINTER(Csr), P, I64, P, P, P, P, SZ, P]),
    "rwt_tall_block_order": (C.c_int, [C.c_int32, P, P, C.c_int32, C.c_int32, P]),
    "rwt_plan_ws": (C.c_int, [C.POINTER(Csr), C.POINTER(PlanOpts), C.POINTER(SZ)]),
    "rwt_plan_create": (C.c_int, [C.POINTER(Csr), C.POINTER(PlanOpts), P, SZ, C.POINTER(P), P]),
    "rwt_plan_get_info": (C.c_int, [P, C.POINTER(PlanInfo)]),
    "rwt_plan_levels": (C.c_int, [P, C.POINTER(P), C.POINTER(P), C.POINTER(P)]),
    "rwt_plan_destroy": (C.c_int, [P]),
    "rwt_solve": (C.c_int, [P, P, I32, I64, P, I64, P]),
    "rwt_solve_transpose": (C.c_int, [P, P, I32, I64, P, I64, P]),
    "rwt_plan_check": (C.c_int, [P, P]),
    "rwt_solve_withhold": (C.c_int, [P, I32, P, I32, I64, P, I64, P]),
    "rwt_apply_MT_ws": (C.c_int, [I32, I64, C.POINTER(SZ)]),
    "rwt_apply_MT": (C.c_int, [I32, I64, P, P, P, I32, P, I32, I64, P, I64, P, SZ, P]),
    "rwt_apply_MT_prepare": (C.c_int, [I32, I64, P, P, SZ, P]),
    "rwt_apply_MT_apply": (C.c_int, [I32, I64, P, P, I32, P, I32, I64, P, I64, P, SZ, P]),
    "rwt_grad_vals": (C.c_int, [C.POINTER(Csr), P, I64, P, I64, I32, P, P]),
    "rwt_apply_M_ws": (C.c_int, [I32, C.POINTER(SZ)]),
    "rwt_apply_M": (C.c_int, [I32, I64, P, P, P, I32, P, I32, I64, P, I64, P, SZ, P]),
    "rwt_apply_M_noalloc": (C.c_int, [I32, I64, P, P, P, I32, P, I32, I64, P, I64, P]),
    "rwt_batch_ws": (C.c_int, [C.POINTER(BatchDesc), C.POINTER(SZ)]),
    "rwt_batch_create": (C.c_int, [C.POINTER(BatchDesc), P, SZ, C.POINTER(P), P]),
    "rwt_batch_run": (C.c_int, [P, P]),
    "rwt_batch_run_setup": (C.c_int, [P, P]),
    "rwt_batch_run_main": (C.c_int, [P, P]),
    "rwt_batch_capture": (C.c_int, [P, P]),
    "rwt_batch_launch": (C.c_int, [P, P]),
    "rwt_batch_stats": (C.c_int, [P, P, P]),
    "rwt_batch_get_info": (C.c_int, [P, C.POINTER(BatchInfo)]),
    "rwt_batch_plan": (C.c_int, [P, I32, C.POINTER(P)]),
    "rwt_batch_destroy": (C.c_int, [P]),
    "rwt_upper_ws": (C.c_int, [C.POINTER(Csr), C.POINTER(PlanOpts), C.POINTER(SZ)]),
    "rwt_upper_create": (C.c_int, [C.POINTER(Csr), C.POINTER(PlanOpts), P, SZ, C.POINTER(P), P]),
    "rwt_upper_refresh": (C.c_int, [P, P]),
    "rwt_upper_get_info": (C.c_int, [P, C.POINTER(PlanInfo)]),
    "rwt_upper_levels": (C.c_int, [P, C.POINTER(P), C.POINTER(P), C.POINTER(P)]),
    "rwt_upper_solve": (C.c_int, [P, P, I32, I64, P, I64, P]),
    "rwt_upper_solve_transpose": (C.c_int, [P, P, I32, I64, P, I64, P]),
    "rwt_solve_pair": (C.c_int, [P, P, P, I32, I64, P, I64, P]),
    "rwt_upper_check": (C.c_int, [P, P]),
    "rwt_upper_destroy": (C.c_int, [P]),
    "rwt_probe_handoff_ws": (SZ, [I32]),
    "rwt_probe_handoff": (C.c_int, [I32, P, SZ, C.POINTER(C.c_double), P]),
    "rwt_generate_ws": (C.c_int, [I32, I32, I32, C.POINTER(SZ)]),
    "rwt_generate": (C.c_int, [C.POINTER(Csr), P, P, P, P, I32, I32, C.POINTER(GenParams), I32,
                               P, P, P, P, P, P, P, P, SZ, P]),
    "rwt_gen_rowsets_ws": (C.c_int, [I32, I32, C.POINTER(SZ)]),
    "rwt_gen_rowsets": (C.c_int, [I32, I32, I32, P, P, P, P, P, P, P, SZ, P]),
    "rwt_env_ws": (C.c_int, [I32, I32, I32, I32, C.POINTER(SZ)]),
    "rwt_env_init": (C.c_int, [C.POINTER(Csr), P, P, P, P, I32, I32, I32, C.POINTER(EnvParams),
                               P, SZ, P]),
    "rwt_env_reset": (C.c_int, [I32, I32, I32, I32, P, P, SZ, P]),
    "rwt_env_step": (C.c_int, [I32, I32, I32, I32, P, P, P, P, P, P, SZ, P]),
    "rwt_env_step_observe": (C.c_int, [I32, I32, I32, I32, P, P, P, P, P, P, P, P, P, SZ, P]),
    "rwt_env_observe": (C.c_int, [I32, I32, I32, I32, P, P, P, P, SZ, P]),
    "rwt_env_levels": (C.c_int, [I32, I32, I32, I32, P, P, P, P, SZ, P]),
}

_lib = None


def load() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with paper_2609_40159_amd.build.build() "
            "(there is no fallback implementation)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    # a library built from other sources than the ones next to it (a stale
    # build shipped with the tree) is refused: rebuild it
    from ._srchash import source_hash
    from .build import FLAGS
    want = source_hash(FLAGS)
    have = lib.rwt_source_hash().decode()
    if want is not None and have != want:
        raise ImportError(
            f"{LIB_PATH} was built from other sources (library {have}, sources {want}): "
            "rebuild it with paper_2609_40159_amd.build.build()")
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != OK:
        msg = load().rwt_last_error_string().decode(errors="replace")
        raise RwtError(status, msg)
