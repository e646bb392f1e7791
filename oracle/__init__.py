"""Python access to the CPU FP64 oracle -- TEST INFRASTRUCTURE ONLY.

Loads ``liboracle.so`` (built from ``oracle.c`` with gcc) through ctypes.
Only the tests, the smoke check and the benchmark's CPU-baseline leg use
this package; the GPU library never imports it and shares no code with it.
See ``oracle.c`` for the definitions each function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, INVALID_ARG, NOT_LOWER, UNSORTED_OR_DUP, MISSING_DIAG, ZERO_DIAG, BAD_ROWSET, \
    BUFFER_TOO_SMALL = 0, -1, -2, -3, -4, -5, -6, -7

STATUS_NAMES = {OK: "OK", INVALID_ARG: "INVALID_ARG", NOT_LOWER: "NOT_LOWER",
                UNSORTED_OR_DUP: "UNSORTED_OR_DUP", MISSING_DIAG: "MISSING_DIAG",
                ZERO_DIAG: "ZERO_DIAG", BAD_ROWSET: "BAD_ROWSET",
                BUFFER_TOO_SMALL: "BUFFER_TOO_SMALL"}


def build(force: bool = False) -> str:
    """Compile liboracle.so (plain gcc, no fused multiply-add)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Stats(C.Structure):
    _fields_ = [("num_levels", C.c_int32), ("thin_count", C.c_int32),
                ("S1", C.c_uint64), ("S2_lo", C.c_uint64), ("S2_hi", C.c_uint64),
                ("cv", C.c_double), ("cv_rows", C.c_double), ("alc", C.c_double),
                ("arl", C.c_double), ("air", C.c_double), ("thin_threshold", C.c_double)]


class _GenParams(C.Structure):
    _fields_ = [("alpha", C.c_double), ("thin_stop", C.c_double), ("max_dist", C.c_int32),
                ("max_moves", C.c_int32), ("max_steps", C.c_int32), ("pad_", C.c_int32)]


class _GenResult(C.Structure):
    _fields_ = [("moves", C.c_int32), ("steps", C.c_int32), ("stop", C.c_int32),
                ("levels", C.c_int32), ("thin", C.c_int32), ("thin0", C.c_int32),
                ("rejected", C.c_int32), ("pad_", C.c_int32), ("threshold", C.c_double),
                ("S1", C.c_uint64), ("S2_lo", C.c_uint64), ("S2_hi", C.c_uint64),
                ("cv", C.c_double)]


GEN_NO_SOURCE, GEN_THIN, GEN_MOVES, GEN_STEPS = 0, 1, 2, 3


class _EnvParams(C.Structure):
    _fields_ = [("alpha", C.c_double), ("thin_stop", C.c_double), ("reward_alpha", C.c_double),
                ("eps", C.c_double), ("decay", C.c_double), ("max_dist", C.c_int32),
                ("search_window", C.c_int32), ("dist_threshold", C.c_int32),
                ("max_steps", C.c_int32), ("stall_steps", C.c_int32), ("keep_top", C.c_int32)]


class _EnvResult(C.Structure):
    _fields_ = [("outcome", C.c_int32), ("node", C.c_int32), ("src", C.c_int32),
                ("tgt", C.c_int32), ("collapsed", C.c_int32), ("done", C.c_int32),
                ("steps", C.c_int32), ("moves", C.c_int32), ("levels", C.c_int32),
                ("thin", C.c_int32), ("thin0", C.c_int32), ("pad_", C.c_int32),
                ("reward", C.c_double), ("r_cv", C.c_double), ("r_cp", C.c_double),
                ("r_rwdist", C.c_double), ("r_abandon", C.c_double), ("cv", C.c_double),
                ("cv_rows", C.c_double)]


ENV_MOVED, ENV_INVALID, ENV_REJECTED, ENV_IGNORED = 0, 1, 2, 3
ENV_DEFAULTS = dict(alpha=1.0, thin_stop=0.02, reward_alpha=1.0, eps=1e-6, decay=0.9, max_dist=8,
                    search_window=5, dist_threshold=2, max_steps=0, stall_steps=0, keep_top=8)


_lib = None


def _L():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.c_void_p
        _lib.orc_validate.argtypes = [C.c_int32, P, P, P, P]
        _lib.orc_validate.restype = C.c_int
        _lib.orc_analyze.argtypes = [C.c_int32, P, P, P, P, P, P, P, C.POINTER(_Stats)]
        _lib.orc_analyze.restype = C.c_int32
        _lib.orc_rewrite.argtypes = [C.c_int32, P, P, P, P, C.c_int32, P, P, C.c_int32, P,
                                     C.c_int64, P, P, P, C.c_int64, P, C.c_int64, P, P, P,
                                     C.c_int64, P]
        _lib.orc_rewrite.restype = C.c_int
        _lib.orc_solve.argtypes = [C.c_int32, P, P, P, C.c_int32, P, C.c_int64, P, C.c_int64]
        _lib.orc_solve.restype = None
        _lib.orc_solve_transpose.argtypes = _lib.orc_solve.argtypes
        _lib.orc_solve_transpose.restype = None
        _lib.orc_solve_upper.argtypes = _lib.orc_solve.argtypes
        _lib.orc_solve_upper.restype = None
        _lib.orc_grad_vals.argtypes = [C.c_int32, P, P, C.c_int32, P, C.c_int64, P,
                                       C.c_int64, P]
        _lib.orc_grad_vals.restype = None
        _lib.orc_generate.argtypes = [C.c_int32, P, P, C.c_int32, C.c_double, C.c_double,
                                      C.POINTER(_GenParams), C.c_int32, P, P, P,
                                      C.POINTER(_GenResult), P, P, P]
        _lib.orc_generate.restype = C.c_int
        _lib.orc_env_create.argtypes = [C.c_int32, P, P, C.c_int32, C.c_double, C.c_double,
                                        C.POINTER(_EnvParams), C.c_int32]
        _lib.orc_env_create.restype = C.c_void_p
        _lib.orc_env_destroy.argtypes = [P]
        _lib.orc_env_destroy.restype = None
        _lib.orc_env_reset.argtypes = [P]
        _lib.orc_env_reset.restype = None
        _lib.orc_env_step.argtypes = [P, C.c_int32, C.POINTER(_EnvResult)]
        _lib.orc_env_step.restype = None
        _lib.orc_env_observe.argtypes = [P, P, P, P]
        _lib.orc_env_observe.restype = None
        _lib.orc_env_state.argtypes = [P, P, P, P, P, P, P, P]
        _lib.orc_env_state.restype = None
    return _lib


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Analysis:
    level: np.ndarray      # int32 [n]
    rows: np.ndarray       # int32 [D]
    cost: np.ndarray       # int64 [D]
    perm: np.ndarray       # int32 [n]
    level_ptr: np.ndarray  # int32 [D+1]
    num_levels: int
    S1: int
    S2: int
    cv: float
    cv_rows: float
    alc: float
    arl: float
    air: float
    thin_threshold: float
    thin_count: int


def validate(n, rowptr, colidx, vals=None) -> tuple[int, int]:
    bad = np.zeros(1, dtype=np.int32)
    vals = None if vals is None else _f64(vals)
    st = _L().orc_validate(n, _p(_i32(rowptr)), _p(_i32(colidx)), _p(vals), _p(bad))
    return int(st), int(bad[0])


def analyze(n, rowptr, colidx) -> Analysis:
    rowptr = _i32(rowptr)
    colidx = _i32(colidx)
    level = np.zeros(max(n, 1), dtype=np.int32)
    rows = np.zeros(max(n, 1), dtype=np.int32)
    cost = np.zeros(max(n, 1), dtype=np.int64)
    perm = np.zeros(max(n, 1), dtype=np.int32)
    lptr = np.zeros(n + 1, dtype=np.int32)
    st = _Stats()
    D = _L().orc_analyze(n, _p(rowptr), _p(colidx), _p(level), _p(rows), _p(cost),
                         _p(perm), _p(lptr), C.byref(st))
    return Analysis(level[:n], rows[:D], cost[:D], perm[:n], lptr[:D + 1], int(D),
                    int(st.S1), int(st.S2_lo) | (int(st.S2_hi) << 64), st.cv, st.cv_rows,
                    st.alc, st.arl, st.air, st.thin_threshold, int(st.thin_count))


@dataclass
class Rewritten:
    rowptr: np.ndarray
    colidx: np.ndarray
    vals: np.ndarray
    Bp: np.ndarray          # (k, n)
    c_ptr: np.ndarray       # int32 [m+1]
    c_col: np.ndarray
    c_val: np.ndarray
    skipped: int


def rewrite(n, rowptr, colidx, vals, level, rows, targets=None, B=None) -> Rewritten:
    rowptr, colidx, vals, level = _i32(rowptr), _i32(colidx), _f64(vals), _i32(level)
    rows = _i32(rows)
    targets = None if targets is None else _i32(targets)
    m = rows.shape[0]
    if B is None:
        B = np.zeros((0, n))
    B = _f64(B)
    k = B.shape[0]
    sizes = np.zeros(3, dtype=np.int64)
    lib = _L()
    st = lib.orc_rewrite(n, _p(rowptr), _p(colidx), _p(vals), _p(level), m, _p(rows),
                         _p(targets), k, _p(B), n, None, None, None, 0, None, n, None,
                         None, None, 0, _p(sizes))
    if st not in (OK, BUFFER_TOO_SMALL):
        raise ValueError("oracle rewrite: " + STATUS_NAMES.get(st, str(st)))
    nnz, nc = int(sizes[0]), int(sizes[1])
    orp = np.zeros(n + 1, dtype=np.int32)
    oci = np.zeros(max(nnz, 1), dtype=np.int32)
    ov = np.zeros(max(nnz, 1), dtype=np.float64)
    Bp = np.zeros((k, n), dtype=np.float64)
    cp = np.zeros(m + 1, dtype=np.int32)
    cc = np.zeros(max(nc, 1), dtype=np.int32)
    cv = np.zeros(max(nc, 1), dtype=np.float64)
    st = lib.orc_rewrite(n, _p(rowptr), _p(colidx), _p(vals), _p(level), m, _p(rows),
                         _p(targets), k, _p(B), n, _p(orp), _p(oci), _p(ov), nnz, _p(Bp), n,
                         _p(cp), _p(cc), _p(cv), nc, _p(sizes))
    if st != OK:
        raise ValueError("oracle rewrite: " + STATUS_NAMES.get(st, str(st)))
    return Rewritten(orp, oci[:nnz], ov[:nnz], Bp, cp, cc[:nc], cv[:nc], int(sizes[2]))


def solve(n, rowptr, colidx, vals, B) -> np.ndarray:
    """X = L^{-1} B; B has shape (k, n) (column-major n x k)."""
    B = _f64(np.atleast_2d(B))
    X = np.zeros_like(B)
    _L().orc_solve(n, _p(_i32(rowptr)), _p(_i32(colidx)), _p(_f64(vals)), B.shape[0],
                   _p(B), n, _p(X), n)
    return X


def solve_upper(n, rowptr, colidx, vals, B) -> np.ndarray:
    """X = U^{-1} B for an upper-triangular CSR U (diagonal first in each row);
    B has shape (k, n)."""
    B = _f64(np.atleast_2d(B))
    X = np.zeros_like(B)
    _L().orc_solve_upper(n, _p(_i32(rowptr)), _p(_i32(colidx)), _p(_f64(vals)), B.shape[0],
                         _p(B), n, _p(X), n)
    return X


def solve_pair(n, l_rowptr, l_colidx, l_vals, u_rowptr, u_colidx, u_vals, B) -> np.ndarray:
    """X = U^{-1} (L^{-1} B): the preconditioner application of an incomplete
    LU factorization."""
    Y = solve(n, l_rowptr, l_colidx, l_vals, B)
    return solve_upper(n, u_rowptr, u_colidx, u_vals, Y)


def solve_transpose(n, rowptr, colidx, vals, G) -> np.ndarray:
    """Y = L^{-T} G; G has shape (k, n)."""
    G = _f64(np.atleast_2d(G))
    Y = np.zeros_like(G)
    _L().orc_solve_transpose(n, _p(_i32(rowptr)), _p(_i32(colidx)), _p(_f64(vals)),
                             G.shape[0], _p(G), n, _p(Y), n)
    return Y


def grad_vals(n, rowptr, colidx, Y, X) -> np.ndarray:
    Y = _f64(np.atleast_2d(Y))
    X = _f64(np.atleast_2d(X))
    out = np.zeros(int(rowptr[-1]), dtype=np.float64)
    _L().orc_grad_vals(n, _p(_i32(rowptr)), _p(_i32(colidx)), Y.shape[0], _p(Y), n, _p(X),
                       n, _p(out))
    return out


def adjoint(n, rowptr, colidx, vals, X, G) -> tuple[np.ndarray, np.ndarray]:
    """Gradients of sum(G * X) with X = L^{-1} B: (grad_B, grad_vals)."""
    Y = solve_transpose(n, rowptr, colidx, vals, G)
    return Y, grad_vals(n, rowptr, colidx, Y, X)


@dataclass
class Generated:
    rows: np.ndarray        # int32 [moves], move order
    src: np.ndarray         # source level of each move
    tgt: np.ndarray         # target level of each move
    moves: int
    steps: int
    stop: int               # GEN_NO_SOURCE / GEN_THIN / GEN_MOVES / GEN_STEPS
    levels: int             # non-empty levels at the end
    thin: int
    thin0: int
    rejected: int
    threshold: float
    S1: int
    S2: int
    cv: float
    level_cost: np.ndarray  # int64 [D]
    level_rows: np.ndarray  # int32 [D]
    level_deps: np.ndarray  # int64 [D]


def generate(n, rowptr, level, num_levels, alc, cv, *, alpha=1.0, thin_stop=0.02, max_dist=8,
             max_moves=0, max_steps=0, cap=None) -> Generated:
    """Rewriting list of the fixed-policy environment run (see orc_generate)."""
    rowptr, level = _i32(rowptr), _i32(level)
    cap = n if cap is None else int(cap)
    D = int(num_levels)
    prm = _GenParams(float(alpha), float(thin_stop), int(max_dist), int(max_moves),
                     int(max_steps), 0)
    res = _GenResult()
    mr = np.zeros(max(cap, 1), dtype=np.int32)
    ms = np.zeros(max(cap, 1), dtype=np.int32)
    mt = np.zeros(max(cap, 1), dtype=np.int32)
    oc = np.zeros(max(D, 1), dtype=np.int64)
    orr = np.zeros(max(D, 1), dtype=np.int32)
    od = np.zeros(max(D, 1), dtype=np.int64)
    st = _L().orc_generate(n, _p(rowptr), _p(level), D, float(alc), float(cv), C.byref(prm),
                           cap, _p(mr), _p(ms), _p(mt), C.byref(res), _p(oc), _p(orr), _p(od))
    if st != OK:
        raise ValueError("oracle generate: " + STATUS_NAMES.get(st, str(st)))
    m = int(res.moves)
    return Generated(mr[:m].copy(), ms[:m].copy(), mt[:m].copy(), m, int(res.steps),
                     int(res.stop), int(res.levels), int(res.thin), int(res.thin0),
                     int(res.rejected), float(res.threshold), int(res.S1),
                     int(res.S2_lo) | (int(res.S2_hi) << 64), float(res.cv), oc[:D].copy(),
                     orr[:D].copy(), od[:D].copy())


class Env:
    """One environment of Sections 4.1-4.5 driven from outside, with the
    reward of Algorithm 2 (see orc_env_step for every reading taken).
    ``level`` is the analysis' level of every row; ``alc`` and ``cv`` its
    average level cost and CV of level costs."""

    def __init__(self, n, rowptr, level, num_levels, alc, cv, cap=None, **params):
        unknown = set(params) - set(ENV_DEFAULTS)
        if unknown:
            raise TypeError("unknown environment parameters: %s" % sorted(unknown))
        prm = dict(ENV_DEFAULTS, **params)
        self.params = prm
        self.n, self.D = int(n), int(num_levels)
        self.cap = self.n if cap is None else int(cap)
        self._rowptr, self._level = _i32(rowptr), _i32(level)
        cp = _EnvParams(float(prm["alpha"]), float(prm["thin_stop"]), float(prm["reward_alpha"]),
                        float(prm["eps"]), float(prm["decay"]), int(prm["max_dist"]),
                        int(prm["search_window"]), int(prm["dist_threshold"]),
                        int(prm["max_steps"]), int(prm["stall_steps"]), int(prm["keep_top"]))
        self._h = _L().orc_env_create(self.n, _p(self._rowptr), _p(self._level), self.D,
                                      float(alc), float(cv), C.byref(cp), self.cap)
        if not self._h:
            raise ValueError("oracle environment: invalid arguments")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _L().orc_env_destroy(h)
            self._h = None

    def reset(self):
        _L().orc_env_reset(self._h)

    def step(self, action) -> dict:
        r = _EnvResult()
        _L().orc_env_step(self._h, int(action), C.byref(r))
        return {f: getattr(r, f) for f, _ in _EnvResult._fields_ if f != "pad_"}

    def observe(self):
        """(level features [6, D], global features [9], mask [D] bool)."""
        lv = np.zeros((6, max(self.D, 1)), dtype=np.float64)
        gl = np.zeros(9, dtype=np.float64)
        mk = np.zeros(max(self.D, 1), dtype=np.uint8)
        _L().orc_env_observe(self._h, _p(lv), _p(gl), _p(mk))
        return lv[:, :self.D], gl, mk[:self.D].astype(bool)

    def state(self):
        """(level of every row, per-level cost, rows, dependency sums, and
        the move list (rows, sources, targets))."""
        lev = np.zeros(self.n, dtype=np.int32)
        cost = np.zeros(self.D, dtype=np.int64)
        rows = np.zeros(self.D, dtype=np.int32)
        deps = np.zeros(self.D, dtype=np.int64)
        c = max(self.cap, 1)
        mr, ms, mt = (np.zeros(c, dtype=np.int32) for _ in range(3))
        _L().orc_env_state(self._h, _p(lev), _p(cost), _p(rows), _p(deps), _p(mr), _p(ms), _p(mt))
        return lev, cost, rows, deps, (mr, ms, mt)
