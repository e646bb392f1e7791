"""Python surface of the HIP library: analyze, rewrite, solve plans, adjoint.

PyTorch provides device memory and streams; every computation runs in
librwtrsv.so.  Dense blocks of k right-hand sides are torch tensors of shape
(k, n) (column q contiguous, i.e. column-major n x k with leading dimension
n) or of shape (n,) for a single right-hand side.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import RwtError, check

__all__ = ["CSRMatrix", "LevelInfo", "validate", "analyze", "rewrite", "Rewrite", "Rewriter", "Plan",
           "solve",
           "apply_MT", "grad_vals", "Batch", "RwtError", "Env", "tall_block_order"]


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dt(dtype: torch.dtype) -> int:
    if dtype == torch.float64:
        return _lib.F64
    if dtype == torch.float32:
        return _lib.F32
    raise TypeError(f"unsupported value type {dtype}")


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


@dataclass
class CSRMatrix:
    """Lower-triangular CSR on the GPU (diagonal last in each row)."""
    rowptr: torch.Tensor   # int32 [n+1]
    colidx: torch.Tensor   # int32 [nnz]
    vals: torch.Tensor | None   # float64/float32 [nnz]

    @property
    def n(self) -> int:
        return self.rowptr.numel() - 1

    @property
    def nnz(self) -> int:
        return self.colidx.numel()

    @property
    def device(self):
        return self.rowptr.device

    @property
    def dtype(self):
        return self.vals.dtype if self.vals is not None else torch.float64

    @classmethod
    def from_arrays(cls, rowptr, colidx, vals=None, device="cuda", dtype=torch.float64):
        rp = torch.as_tensor(rowptr, dtype=torch.int32).to(device).contiguous()
        ci = torch.as_tensor(colidx, dtype=torch.int32).to(device).contiguous()
        v = None if vals is None else torch.as_tensor(vals).to(device=device, dtype=dtype).contiguous()
        return cls(rp, ci, v)

    def view(self) -> _lib.Csr:
        # the library reads these pointers on the GPU: refuse host tensors,
        # mixed devices and wrong index or value types before any launch
        dev = self.rowptr.device
        if dev.type != "cuda":
            raise ValueError(f"the matrix is on {dev}; the library needs GPU tensors")
        if self.rowptr.dtype != torch.int32 or self.colidx.dtype != torch.int32:
            raise ValueError("rowptr and colidx must be int32")
        _on(self.colidx, dev, "colidx")
        if self.vals is not None:
            _on(self.vals, dev, "vals")
            if self.vals.dtype not in (torch.float64, torch.float32):
                raise ValueError(f"unsupported value type {self.vals.dtype}")
            if self.vals.numel() != self.colidx.numel():
                raise ValueError("vals and colidx differ in length")
        if not (self.rowptr.is_contiguous() and self.colidx.is_contiguous()
                and (self.vals is None or self.vals.is_contiguous())):
            raise ValueError("CSR arrays must be contiguous")
        c = _lib.Csr()
        c.n = self.n
        c.nnz = self.nnz
        c.rowptr = self.rowptr.data_ptr()
        c.colidx = self.colidx.data_ptr() if self.nnz else None
        c.vals = self.vals.data_ptr() if self.vals is not None and self.nnz else None
        c.dt = _dt(self.dtype)
        return c

    def with_vals(self, vals: torch.Tensor) -> "CSRMatrix":
        return CSRMatrix(self.rowptr, self.colidx, vals)


def validate(L: CSRMatrix) -> tuple[str, int]:
    """(status name, offending row or -1)."""
    lib = _lib.load()
    ws = _workspace(lib.rwt_validate_ws(), L.device)
    bad = C.c_int32(-1)
    st = lib.rwt_validate(C.byref(L.view()), _ptr(ws), ws.numel(), C.byref(bad), _stream())
    return _lib.STATUS.get(st, str(st)), int(bad.value)


@dataclass
class LevelInfo:
    level: torch.Tensor       # int32 [n]
    perm: torch.Tensor        # int32 [n]
    level_ptr: torch.Tensor   # int32 [D+1]
    rows: torch.Tensor        # int32 [D]
    cost: torch.Tensor        # int64 [D]
    stats: dict
    device_stats: torch.Tensor  # raw device copy of the statistics struct

    @property
    def num_levels(self) -> int:
        return int(self.stats["num_levels"])


def analyze(L: CSRMatrix) -> LevelInfo:
    """Level-set analysis (levels, (level,row) order, per-level rows/cost, CV...)."""
    lib = _lib.load()
    n = L.n
    dev = L.device
    sz = C.c_size_t(0)
    check(lib.rwt_analyze_ws(C.byref(L.view()), C.byref(sz)))
    ws = _workspace(sz.value, dev)
    level = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    lptr = torch.empty(n + 1, dtype=torch.int32, device=dev)
    rows = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    cost = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
    dstats = torch.empty(C.sizeof(_lib.LevelStats), dtype=torch.uint8, device=dev)
    hs = _lib.LevelStats()
    check(lib.rwt_analyze(C.byref(L.view()), _ptr(ws), ws.numel(), _ptr(level), _ptr(perm),
                          _ptr(lptr), _ptr(rows), _ptr(cost), _ptr(dstats), C.byref(hs),
                          _stream()))
    D = int(hs.num_levels)
    return LevelInfo(level[:n], perm[:n], lptr[:D + 1], rows[:D], cost[:D], hs.as_dict(), dstats)


@dataclass
class Rewrite:
    L: CSRMatrix              # rewritten matrix L'
    B: torch.Tensor | None    # B' (k, n)
    crow: torch.Tensor        # substitution e: row crow[e] -= cval[e] * row ccol[e]
    ccol: torch.Tensor
    cval: torch.Tensor
    cptr: torch.Tensor        # offsets of each set row's substitutions
    skipped: int
    # C^T ordering for apply_MT, built on first use (the pattern of C does
    # not change when the numeric rewrite is re-run)
    mt_ws: torch.Tensor | None = None


def _same_device(t: torch.Tensor, device) -> bool:
    d = torch.device(device)
    if t.device.type != d.type:
        return False
    if d.type == "cuda":
        want = d.index if d.index is not None else torch.cuda.current_device()
        have = t.device.index if t.device.index is not None else torch.cuda.current_device()
        return want == have
    return True


def _on(t: torch.Tensor | None, device, what: str, dtype=None) -> torch.Tensor | None:
    """Refuse, before any launch, a tensor that is not on the given device
    (a host pointer handed to a kernel faults the GPU) or not of dtype."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if not _same_device(t, device):
        raise ValueError(f"{what} is on {t.device}, expected {torch.device(device)}")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{what} has dtype {t.dtype}, expected {dtype}")
    return t


def _block(B: torch.Tensor | None, n: int, dtype, device,
           what: str = "dense block") -> tuple[torch.Tensor | None, int]:
    if B is None:
        return None, 0
    _on(B, device, what)
    if B.dim() == 1:
        B = B.reshape(1, -1)
    if B.dim() != 2 or B.shape[-1] != n or B.dtype != dtype or not B.is_contiguous():
        raise ValueError(f"{what} must be a contiguous (k, {n}) tensor of {dtype}")
    return B, B.shape[0]


def _out_like(out: torch.Tensor | None, B2: torch.Tensor, what: str = "output") -> torch.Tensor:
    """The output block: new, or the caller's, which must match B2 exactly
    (shape, dtype, device, contiguity) since the kernels write it as B2."""
    if out is None:
        return torch.empty_like(B2)
    _on(out, B2.device, what, B2.dtype)
    X = out.reshape(B2.shape) if out.numel() == B2.numel() and out.is_contiguous() else out
    if X.shape != B2.shape or not X.is_contiguous():
        raise ValueError(f"{what} must be a contiguous tensor of the right-hand side's shape")
    return X


class Rewriter:
    """Symbolic rewrite of a row set, kept so the numeric part can be re-run
    for new values or right-hand sides into the same L' buffers."""

    def __init__(self, L: CSRMatrix, level: torch.Tensor, rows, targets=None):
        lib = _lib.load()
        self._lib = lib
        n = L.n
        dev = L.device
        self.L = L
        self.level = _on(level, dev, "level", torch.int32).contiguous()
        if isinstance(rows, torch.Tensor):
            _on(rows, dev, "rows")
        if isinstance(targets, torch.Tensor):
            _on(targets, dev, "targets")
        self.rows = torch.as_tensor(rows, dtype=torch.int32).to(dev).contiguous()
        self.m = self.rows.numel()
        self.targets = (None if targets is None else
                        torch.as_tensor(targets, dtype=torch.int32).to(dev).contiguous())
        sz = C.c_size_t(0)
        check(lib.rwt_rewrite_ws(C.byref(L.view()), self.m, C.byref(sz)))
        self.ws = _workspace(sz.value, dev)
        rowptr = torch.empty(n + 1, dtype=torch.int32, device=dev)
        self.cptr = torch.empty(self.m + 1, dtype=torch.int32, device=dev)
        sizes = (C.c_int64 * 3)()
        check(lib.rwt_rewrite_symbolic(C.byref(L.view()), _ptr(level), _ptr(self.rows),
                                       _ptr(self.targets), self.m, _ptr(self.ws), self.ws.numel(),
                                       _ptr(rowptr), _ptr(self.cptr), sizes, _stream()))
        self.nnz, self.nc, self.skipped = int(sizes[0]), int(sizes[1]), int(sizes[2])
        colidx = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
        vals = torch.empty(max(self.nnz, 1), dtype=L.dtype, device=dev)
        self.Lp = CSRMatrix(rowptr, colidx[:self.nnz], vals[:self.nnz])
        self._colidx, self._vals = colidx, vals
        self.crow = torch.empty(max(self.nc, 1), dtype=torch.int32, device=dev)
        self.ccol = torch.empty(max(self.nc, 1), dtype=torch.int32, device=dev)
        self.cval = torch.empty(max(self.nc, 1), dtype=L.dtype, device=dev)

    def numeric(self, vals: torch.Tensor | None = None,
                B: torch.Tensor | None = None) -> torch.Tensor | None:
        """Fill L' values (in place) and the multipliers; return B' for B."""
        if vals is not None:
            _on(vals, self.L.device, "vals", self.L.dtype)
            if vals.numel() != self.L.nnz:
                raise ValueError(f"vals must hold {self.L.nnz} entries")
        L = self.L if vals is None else self.L.with_vals(vals.contiguous())
        n = L.n
        B2, k = _block(B, n, L.dtype, L.device)
        Bp = torch.empty((k, n), dtype=L.dtype, device=L.device) if B2 is not None else None
        lpv = _lib.Csr()
        lpv.n = n
        lpv.nnz = self.nnz
        lpv.rowptr = self.Lp.rowptr.data_ptr()
        lpv.colidx = self._colidx.data_ptr()
        lpv.vals = self._vals.data_ptr()
        lpv.dt = _dt(L.dtype)
        check(self._lib.rwt_rewrite_numeric(
            C.byref(L.view()), _ptr(self.level), _ptr(self.rows), _ptr(self.targets), self.m,
            _ptr(B2), k, n, C.byref(lpv), _ptr(Bp), n, _ptr(self.crow), _ptr(self.ccol),
            _ptr(self.cval), _ptr(self.ws), self.ws.numel(), _stream()))
        if Bp is None:
            return None
        return Bp.reshape(B.shape)

    def result(self, Bp=None) -> "Rewrite":
        nc = self.nc
        return Rewrite(self.Lp, Bp, self.crow[:nc], self.ccol[:nc], self.cval[:nc], self.cptr,
                       self.skipped)


def rewrite(L: CSRMatrix, level: torch.Tensor, rows, targets=None,
            B: torch.Tensor | None = None) -> Rewrite:
    """Equation rewriting of the given rows (targets default to level - 1)."""
    rw = Rewriter(L, level, rows, targets)
    Bp = rw.numeric(None, B)
    return rw.result(Bp)


# sync-free solves: whether helper waves prefetch the x values a row block
# reads from earlier blocks ("auto": the plan times both)
STAGE = {"auto": 0, "on": 1, "off": 2}
STAGE_NAME = {1: "on", 2: "off"}


def _option(table: dict, value, what: str) -> int:
    if value not in table:
        raise ValueError(f"{what} must be one of {sorted(table)}, not {value!r}")
    return table[value]


class Plan:
    """Analysis + schedule of one matrix; solves L X = B and L^T Y = G."""

    # the C entry points of this kind of plan (UpperPlan substitutes its own)
    _C = dict(ws="rwt_plan_ws", create="rwt_plan_create", info="rwt_plan_get_info",
              levels="rwt_plan_levels", destroy="rwt_plan_destroy", solve="rwt_solve",
              solve_t="rwt_solve_transpose", check="rwt_plan_check")

    def __init__(self, L: CSRMatrix, algo: str = "auto", kmax: int = 1, block_rows: int = 0,
                 lanes_per_row: int = 0, narrow_rows: int = -1, watchdog_ms: int = 0,
                 rhs_chunk: int = 0, stage_outside: str = "auto"):
        lib = _lib.load()
        self.L = L
        self._lib = lib
        self._fn = {k: getattr(lib, v) for k, v in self._C.items()}
        o = _lib.PlanOpts()
        o.algo = _option(_lib.ALGO, algo, "algo")
        o.block_rows = block_rows
        o.lanes_per_row = lanes_per_row
        o.narrow_rows = narrow_rows
        o.kmax = kmax
        o.watchdog_ms = watchdog_ms
        o.rhs_chunk = rhs_chunk
        o.stage_outside = _option(STAGE, stage_outside, "stage_outside")
        self.opts = o
        sz = C.c_size_t(0)
        view = L.view()
        check(self._fn["ws"](C.byref(view), C.byref(o), C.byref(sz)))
        self.ws = _workspace(sz.value, L.device)
        h = C.c_void_p()
        check(self._fn["create"](C.byref(view), C.byref(o), _ptr(self.ws), self.ws.numel(),
                                 C.byref(h), _stream()))
        self._h = h
        self.kmax = kmax

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._fn["destroy"](h)
            self._h = None

    @property
    def info(self) -> dict:
        inf = _lib.PlanInfo()
        check(self._fn["info"](self._h, C.byref(inf)))
        d = {f: getattr(inf, f) for f, _ in inf._fields_ if f not in ("stats", "pad_")}
        d["algo_fwd"] = _lib.ALGO_NAME[d["algo_fwd"]]
        d["algo_bwd"] = _lib.ALGO_NAME[d["algo_bwd"]]
        d["stage_outside"] = STAGE_NAME[d["stage_outside"]]
        d["stats"] = inf.stats.as_dict()
        return d

    def levels(self) -> tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
        """(level[n], perm[n], level_ptr[D+1]) views into the plan's workspace
        (for an UpperPlan: of the reversed matrix J U J, row i' = U's row
        n-1-i')."""
        a, b, c = C.c_void_p(), C.c_void_p(), C.c_void_p()
        check(self._fn["levels"](self._h, C.byref(a), C.byref(b), C.byref(c)))
        n = self.L.n
        D = self.info["stats"]["num_levels"]
        base = self.ws.data_ptr()

        def view(ptr, count):
            off = ptr.value - base
            return self.ws[off:off + 4 * count].view(torch.int32)
        return view(a, n), view(b, n), view(c, D + 1)

    def _run(self, fn, B: torch.Tensor, out: torch.Tensor | None):
        B2, k = _block(B, self.L.n, self.L.dtype, self.L.device)
        if k > self.kmax:
            raise ValueError(f"{k} right-hand sides, the plan was made for at most {self.kmax}")
        X = _out_like(out, B2)
        check(fn(self._h, _ptr(B2), k, self.L.n, _ptr(X), self.L.n, _stream()))
        return X.reshape(B.shape)

    def solve(self, B: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        return self._run(self._fn["solve"], B, out)

    def solve_transpose(self, G: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        return self._run(self._fn["solve_t"], G, out)

    def check(self) -> None:
        """Raise if a device wait expired in the last solve (synchronizes)."""
        check(self._fn["check"](self._h, _stream()))


def solve(L: CSRMatrix, B: torch.Tensor, plan: Plan | None = None,
          out: torch.Tensor | None = None) -> torch.Tensor:
    """X = L^{-1} B (B: (n,) or (k, n), one right-hand side per row of the
    block, column-major at the boundary).  Without a plan one is built for L
    (analysis, schedule and autotuning); keep a Plan to reuse them."""
    if plan is None:
        k = 1 if B.dim() == 1 else B.shape[0]
        plan = Plan(L, kmax=k)
    elif plan.L is not L:
        raise ValueError("the plan was built for another matrix")
    return plan.solve(B, out=out)


class UpperPlan(Plan):
    """Solves U X = B and U^T Y = G for an upper-triangular CSR U (diagonal
    first in each row), through the reversed lower matrix J U J; same
    options as Plan."""

    _C = dict(ws="rwt_upper_ws", create="rwt_upper_create", info="rwt_upper_get_info",
              levels="rwt_upper_levels", destroy="rwt_upper_destroy", solve="rwt_upper_solve",
              solve_t="rwt_upper_solve_transpose", check="rwt_upper_check")

    def refresh(self) -> None:
        """Take U's current values (after they were changed in place)."""
        check(self._lib.rwt_upper_refresh(self._h, _stream()))


def solve_pair(Lp: Plan, Up: UpperPlan, B: torch.Tensor,
               out: torch.Tensor | None = None) -> torch.Tensor:
    """X = U^{-1} (L^{-1} B): one application of the preconditioner M = L U."""
    lib = _lib.load()
    n = Lp.L.n
    if Up.L.n != n or Up.L.dtype != Lp.L.dtype or not _same_device(Up.L.rowptr, Lp.L.device):
        raise ValueError("the lower and upper plans differ in size, value type or device")
    B2, k = _block(B, n, Lp.L.dtype, Lp.L.device)
    if k > min(Lp.kmax, Up.kmax):
        raise ValueError(f"{k} right-hand sides, the plans allow {min(Lp.kmax, Up.kmax)}")
    X = _out_like(out, B2)
    check(lib.rwt_solve_pair(Lp._h, Up._h, _ptr(B2), k, n, _ptr(X), n, _stream()))
    return X.reshape(B.shape)


def apply_MT(rw: Rewrite, Y: torch.Tensor) -> torch.Tensor:
    """Y - C^T Y for the multipliers of a rewrite (grad_B of the rewritten system)."""
    lib = _lib.load()
    n = rw.L.n
    Y2, k = _block(Y, n, rw.L.dtype, rw.L.device)
    nc = rw.crow.numel()
    if rw.mt_ws is None:
        sz = C.c_size_t(0)
        check(lib.rwt_apply_MT_ws(n, nc, C.byref(sz)))
        ws = _workspace(sz.value, Y.device)
        check(lib.rwt_apply_MT_prepare(n, nc, _ptr(rw.ccol), _ptr(ws), ws.numel(), _stream()))
        rw.mt_ws = ws
    ws = rw.mt_ws
    out = torch.empty_like(Y2)
    check(lib.rwt_apply_MT_apply(n, nc, _ptr(rw.crow), _ptr(rw.cval), _dt(rw.L.dtype), _ptr(Y2), k,
                                 n, _ptr(out), n, _ptr(ws), ws.numel(), _stream()))
    return out.reshape(Y.shape)


def apply_M(rw: Rewrite, B: torch.Tensor) -> torch.Tensor:
    """M B = B - C B: the right-hand side of the rewritten system for a new B."""
    lib = _lib.load()
    n = rw.L.n
    B2, k = _block(B, n, rw.L.dtype, rw.L.device)
    sz = C.c_size_t(0)
    check(lib.rwt_apply_M_ws(n, C.byref(sz)))
    ws = _workspace(sz.value, B.device)
    out = torch.empty_like(B2)
    check(lib.rwt_apply_M(n, rw.crow.numel(), _ptr(rw.crow), _ptr(rw.ccol), _ptr(rw.cval),
                          _dt(rw.L.dtype), _ptr(B2), k, n, _ptr(out), n, _ptr(ws), ws.numel(),
                          _stream()))
    return out.reshape(B.shape)


def grad_vals(L: CSRMatrix, gB: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    """-sum_q gB[row_p, q] * X[col_p, q] on every stored entry of L."""
    lib = _lib.load()
    gB2, k = _block(gB, L.n, L.dtype, L.device, "gB")
    X2, k2 = _block(X, L.n, L.dtype, L.device, "X")
    if k != k2:
        raise ValueError("gB and X must have the same number of columns")
    out = torch.empty(L.nnz, dtype=L.dtype, device=L.device)
    check(lib.rwt_grad_vals(C.byref(L.view()), _ptr(gB2), L.n, _ptr(X2), L.n, k, _ptr(out),
                            _stream()))
    return out


def _check_info(info: "LevelInfo", device) -> None:
    for name in ("level", "level_ptr", "cost", "device_stats"):
        _on(getattr(info, name), device, f"analysis array {name}")


GEN_STOPS = {0: "no_source", 1: "thin", 2: "moves", 3: "steps"}


@dataclass
class Generated:
    """Rewriting lists of num_env environments over one matrix (move order)."""
    rows: torch.Tensor        # int32 (num_env, cap); environment e uses [:moves[e]]
    src: torch.Tensor
    tgt: torch.Tensor
    results: list             # per environment: moves, steps, stop, levels, thin, ...
    level_cost: torch.Tensor | None   # int64 (num_env, D) final per-level sums
    level_rows: torch.Tensor | None
    level_deps: torch.Tensor | None
    d_res: torch.Tensor       # device copy of the results (rwt_gen_result array)
    n: int
    cap: int


def _gen_params(params: dict) -> _lib.GenParams:
    return _lib.GenParams(float(params.get("alpha", 1.0)), float(params.get("thin_stop", 0.02)),
                          int(params.get("max_dist", 8)), int(params.get("max_moves", 0)),
                          int(params.get("max_steps", 0)), 0)


def generate(L: CSRMatrix, info: LevelInfo, params, cap: int, level_sums: bool = False,
             sync: bool = True) -> Generated:
    """Run one environment per parameter dict (keys alpha, thin_stop, max_dist,
    max_moves, max_steps) on L; each keeps at most cap moves."""
    lib = _lib.load()
    if isinstance(params, dict):
        params = [params]
    ne = len(params)
    n, D = L.n, info.num_levels
    dev = L.device
    _check_info(info, dev)
    sz = C.c_size_t(0)
    check(lib.rwt_generate_ws(n, D, ne, C.byref(sz)))
    ws = _workspace(sz.value, dev)
    hp = (_lib.GenParams * max(ne, 1))(*[_gen_params(q) for q in params])
    mr = torch.empty((ne, max(cap, 1)), dtype=torch.int32, device=dev)
    ms = torch.empty_like(mr)
    mt = torch.empty_like(mr)
    d_res = torch.empty(max(ne, 1) * C.sizeof(_lib.GenResult), dtype=torch.uint8, device=dev)
    lc = lr = ld = None
    if level_sums:
        lc = torch.empty((ne, max(D, 1)), dtype=torch.int64, device=dev)
        lr = torch.empty((ne, max(D, 1)), dtype=torch.int32, device=dev)
        ld = torch.empty((ne, max(D, 1)), dtype=torch.int64, device=dev)
    check(lib.rwt_generate(C.byref(L.view()), _ptr(info.level), _ptr(info.level_ptr),
                           _ptr(info.cost), _ptr(info.device_stats), D, ne, hp, cap, _ptr(mr),
                           _ptr(ms), _ptr(mt), _ptr(d_res), _ptr(lc), _ptr(lr), _ptr(ld),
                           _ptr(ws), ws.numel(), _stream()))
    results = []
    if sync and ne > 0:
        raw = d_res.cpu().numpy().tobytes()
        for e in range(ne):
            r = _lib.GenResult.from_buffer_copy(raw, e * C.sizeof(_lib.GenResult))
            d = r.as_dict()
            d["stop_name"] = GEN_STOPS.get(d["stop"], "?")
            results.append(d)
    return Generated(mr[:, :cap], ms[:, :cap], mt[:, :cap], results,
                     None if lc is None else lc[:, :D], None if lr is None else lr[:, :D],
                     None if ld is None else ld[:, :D], d_res, n, cap)


ENV_DEFAULTS = dict(alpha=1.0, thin_stop=0.02, reward_alpha=1.0, eps=1e-6, decay=0.9, max_dist=8,
                    search_window=5, dist_threshold=2, max_steps=0, stall_steps=0, keep_top=8)
ENV_OUTCOMES = {0: "moved", 1: "invalid", 2: "rejected", 3: "ignored", 4: "error"}


class EnvStep:
    """Results of one rwt_env_step call, as views of the environment's
    result buffer (the next step overwrites them; clone to keep)."""

    def __init__(self, raw: torch.Tensor, num_env: int):
        self.raw = raw
        self.num_env = num_env
        ints = raw.view(torch.int32).view(num_env, -1)
        dbl = raw.view(torch.float64).view(num_env, -1)
        self.outcome, self.node, self.src, self.tgt = ints[:, 0], ints[:, 1], ints[:, 2], ints[:, 3]
        self.collapsed, self.done = ints[:, 4], ints[:, 5]
        self.reward = dbl[:, 6]
        self.terms = dbl[:, 7:11]          # r_cv, r_cp, r_rwdist, r_abandon
        self.cv = dbl[:, 11]

    def results(self) -> list[dict]:
        buf = self.raw.cpu().numpy().tobytes()
        sz = C.sizeof(_lib.EnvResult)
        return [_lib.EnvResult.from_buffer_copy(buf, e * sz).as_dict()
                for e in range(self.num_env)]


class Env:
    """num_env environments of Sections 4.1-4.5 over one analysed matrix,
    stepped together by the caller's policy (rwt_env_*): step(actions)
    returns the Algorithm 2 rewards, observe() the Table 1 features and the
    action mask.  Move lists grow in mv_row / mv_src / mv_tgt (num_env, cap);
    cap defaults to the step limit (no episode makes more moves), which
    keeps the per-environment memory at 45 bytes per level plus 24 per move
    of capacity."""

    def __init__(self, L: CSRMatrix, info: LevelInfo, num_env: int, cap: int | None = None,
                 **params):
        unknown = set(params) - set(ENV_DEFAULTS)
        if unknown:
            raise TypeError("unknown environment parameters: %s" % sorted(unknown))
        self.lib = _lib.load()
        p = dict(ENV_DEFAULTS, **params)
        self.params = p
        self.n, self.D, self.E = L.n, info.num_levels, int(num_env)
        if cap is None:
            # moves never outnumber steps: the step limit bounds the list
            steps = int(p["max_steps"]) or max(2 * self.D, 6144)
            cap = min(self.n, steps)
        self.cap = int(cap)
        self.device = L.device
        _check_info(info, self.device)
        sz = C.c_size_t(0)
        check(self.lib.rwt_env_ws(self.n, self.D, self.E, self.cap, C.byref(sz)))
        self.ws = _workspace(sz.value, self.device)
        hp = _lib.EnvParams(float(p["alpha"]), float(p["thin_stop"]), float(p["reward_alpha"]),
                            float(p["eps"]), float(p["decay"]), int(p["max_dist"]),
                            int(p["search_window"]), int(p["dist_threshold"]),
                            int(p["max_steps"]), int(p["stall_steps"]), int(p["keep_top"]))
        dev = self.device
        self.mv_row = torch.full((self.E, self.cap), -1, dtype=torch.int32, device=dev)
        self.mv_src = torch.full_like(self.mv_row, -1)
        self.mv_tgt = torch.full_like(self.mv_row, -1)
        self._res = torch.zeros(self.E * C.sizeof(_lib.EnvResult), dtype=torch.uint8, device=dev)
        self.obs_level = torch.empty((self.E, 6, self.D), dtype=torch.float32, device=dev)
        self.obs_global = torch.empty((self.E, 9), dtype=torch.float32, device=dev)
        self.mask = torch.empty((self.E, self.D), dtype=torch.uint8, device=dev)
        check(self.lib.rwt_env_init(C.byref(L.view()), _ptr(info.level), _ptr(info.level_ptr),
                                    _ptr(info.cost), _ptr(info.device_stats), self.D, self.E,
                                    self.cap, C.byref(hp), _ptr(self.ws), self.ws.numel(),
                                    _stream()))

    def _dims(self):
        return self.n, self.D, self.E, self.cap

    def reset(self, which: torch.Tensor | None = None):
        """Reset every environment, or those with which[e] != 0 (bool/uint8)."""
        w = None if which is None else which.to(device=self.device, dtype=torch.uint8).contiguous()
        check(self.lib.rwt_env_reset(*self._dims(), _ptr(w), _ptr(self.ws), self.ws.numel(),
                                     _stream()))

    def step(self, actions, observe: bool = False) -> EnvStep:
        """Apply one action per environment; with observe=True the
        observation and mask of the new state are written in the same
        launch (obs_level / obs_global / mask)."""
        a = torch.as_tensor(actions, dtype=torch.int32).to(self.device).contiguous()
        if a.numel() != self.E:
            raise ValueError("one action per environment")
        if observe:
            check(self.lib.rwt_env_step_observe(
                *self._dims(), _ptr(a), _ptr(self._res), _ptr(self.mv_row), _ptr(self.mv_src),
                _ptr(self.mv_tgt), _ptr(self.obs_level), _ptr(self.obs_global), _ptr(self.mask),
                _ptr(self.ws), self.ws.numel(), _stream()))
        else:
            check(self.lib.rwt_env_step(*self._dims(), _ptr(a), _ptr(self._res),
                                        _ptr(self.mv_row), _ptr(self.mv_src), _ptr(self.mv_tgt),
                                        _ptr(self.ws), self.ws.numel(), _stream()))
        self._last_actions = a            # keep alive until the launch ran
        return EnvStep(self._res, self.E)

    def observe(self, level: bool = True, glob: bool = True, mask: bool = True):
        """(level features (E, 6, D) f32, global features (E, 9) f32, mask
        (E, D) uint8); the buffers are reused by the next call."""
        check(self.lib.rwt_env_observe(*self._dims(), _ptr(self.obs_level if level else None),
                                       _ptr(self.obs_global if glob else None),
                                       _ptr(self.mask if mask else None), _ptr(self.ws),
                                       self.ws.numel(), _stream()))
        return self.obs_level, self.obs_global, self.mask

    def levels(self):
        """Per-level (cost, rows, dependency sums), each (E, D)."""
        c = torch.empty((self.E, self.D), dtype=torch.int64, device=self.device)
        r = torch.empty((self.E, self.D), dtype=torch.int32, device=self.device)
        d = torch.empty_like(c)
        check(self.lib.rwt_env_levels(*self._dims(), _ptr(c), _ptr(r), _ptr(d), _ptr(self.ws),
                                      self.ws.numel(), _stream()))
        return c, r, d


def gen_rowsets(g: Generated) -> tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
    """(cand_ptr, cand_rows, cand_targets): each environment's moved rows in
    ascending order with their targets, concatenated (batch candidate form)."""
    lib = _lib.load()
    ne = g.rows.shape[0]
    dev = g.rows.device
    sz = C.c_size_t(0)
    check(lib.rwt_gen_rowsets_ws(ne, g.cap, C.byref(sz)))
    ws = _workspace(sz.value, dev)
    ptr = torch.empty(ne + 1, dtype=torch.int32, device=dev)
    rows = torch.empty(max(ne * g.cap, 1), dtype=torch.int32, device=dev)
    tg = torch.empty_like(rows)
    # the move arrays are (ne, cap) with row stride cap: contiguous only when
    # cap >= 1 (the allocation keeps one column for cap == 0)
    mr = g.rows.contiguous()
    mt = g.tgt.contiguous()
    check(lib.rwt_gen_rowsets(g.n, ne, g.cap, _ptr(g.d_res), _ptr(mr), _ptr(mt), _ptr(ptr),
                              _ptr(rows), _ptr(tg), _ptr(ws), ws.numel(), _stream()))
    return ptr, rows, tg


class Batch:
    """Many matrices (each with k right-hand sides) and many candidate rewrite
    sets, run as one persistent launch (optionally a captured graph).

    mats: list of (CSRMatrix FP64, B (k, n) or None, X (k, n) or None).
    cand_mat: matrix index of each candidate; cand_ptr (C+1) and cand_rows
    are device int32 tensors whose contents may change between launches
    (within cand_rows_cap rows).  block_rows: per-matrix solve block sizes
    (default: autotuned).  All work runs on the batch's own stream,
    ordered after the caller's current stream and before it again.
    """

    def __init__(self, mats, cand_mat, cand_ptr, cand_rows, cand_targets=None,
                 cand_rows_cap: int | None = None, pattern_cap: int = 0, watchdog_ms: int = 0,
                 block_rows=None, cand_mode: str = "auto"):
        lib = _lib.load()
        self._lib = lib
        self.mats = list(mats)
        dev = self.mats[0][0].device if self.mats else torch.device("cuda")
        self.stream = torch.cuda.Stream(device=dev)
        arr = (_lib.BatchMatrix * max(1, len(self.mats)))()
        self._keep = []
        for i, (L, B, X) in enumerate(self.mats):
            if L.dtype != torch.float64:
                raise TypeError("batched matrices must be float64")
            arr[i].L = L.view()
            k = 0
            if B is not None:
                if not _same_device(L.rowptr, dev):
                    raise ValueError(f"matrix {i} is on {L.device}, the batch on {dev}")
                B2, k = _block(B, L.n, L.dtype, dev, f"B of matrix {i}")
                X2, k2 = _block(X, L.n, L.dtype, dev, f"X of matrix {i}")
                if k != k2:
                    raise ValueError("B and X must have the same number of columns")
                arr[i].B = B2.data_ptr()
                arr[i].X = X2.data_ptr()
                self._keep += [B2, X2]
            arr[i].k = k
            arr[i].block_rows = 0 if block_rows is None else int(block_rows[i])
            arr[i].ldb = L.n
            arr[i].ldx = L.n
        self._arr = arr
        self.cand_mat = (C.c_int32 * max(1, len(cand_mat)))(*cand_mat)
        self.cand_ptr = cand_ptr
        self.cand_rows = cand_rows
        self.cand_targets = cand_targets
        self.num_cand = len(cand_mat)
        d = _lib.BatchDesc()
        d.count = len(self.mats)
        d.num_cand = self.num_cand
        d.mats = C.cast(arr, C.c_void_p)
        d.h_cand_mat = C.cast(self.cand_mat, C.c_void_p)
        d.d_cand_ptr = cand_ptr.data_ptr() if self.num_cand else None
        d.d_cand_rows = cand_rows.data_ptr() if self.num_cand else None
        d.d_cand_targets = None if cand_targets is None else cand_targets.data_ptr()
        d.cand_rows_cap = int(cand_rows_cap if cand_rows_cap is not None
                              else (cand_rows.numel() if cand_rows is not None else 0))
        if not 0 <= int(pattern_cap) < 2 ** 31:
            raise ValueError(f"pattern_cap must be in [0, 2^31), got {pattern_cap}")
        d.pattern_cap = int(pattern_cap)
        d.watchdog_ms = watchdog_ms
        d.cand_mode = {"auto": 0, "blocks": 1, "sweep": 2, "walk": 3}[cand_mode]
        self.desc = d
        sz = C.c_size_t(0)
        check(lib.rwt_batch_ws(C.byref(d), C.byref(sz)))
        self.ws = _workspace(sz.value, dev)
        h = C.c_void_p()
        self._enter()
        try:
            check(lib.rwt_batch_create(C.byref(d), _ptr(self.ws), self.ws.numel(), C.byref(h),
                                       self.stream.cuda_stream))
        finally:
            self._leave()
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.rwt_batch_destroy(h)
            self._h = None

    def _enter(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.stream.device))

    def _leave(self):
        torch.cuda.current_stream(self.stream.device).wait_stream(self.stream)

    def run(self) -> None:
        """Enqueue one batched launch (no graph)."""
        self._enter()
        check(self._lib.rwt_batch_run(self._h, self.stream.cuda_stream))
        self._leave()

    def run_timed(self) -> tuple:
        """Enqueue one batched launch with events around its persistent
        kernel, recorded on the batch's stream: (start, end) events of
        the persistent kernel alone (the setup kernels run before)."""
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        self._enter()
        check(self._lib.rwt_batch_run_setup(self._h, self.stream.cuda_stream))
        a.record(self.stream)
        check(self._lib.rwt_batch_run_main(self._h, self.stream.cuda_stream))
        b.record(self.stream)
        self._leave()
        return a, b

    def capture(self) -> None:
        """Capture the launch sequence into a graph (replayed by launch())."""
        self._enter()
        check(self._lib.rwt_batch_capture(self._h, self.stream.cuda_stream))
        self._leave()

    def launch(self) -> None:
        self._enter()
        check(self._lib.rwt_batch_launch(self._h, self.stream.cuda_stream))
        self._leave()

    def stats(self) -> list[dict]:
        out = (_lib.CandStats * max(1, self.num_cand))()
        st = self._lib.rwt_batch_stats(self._h, C.cast(out, C.c_void_p), self.stream.cuda_stream)
        res = []
        for c in range(self.num_cand):
            s = out[c]
            res.append({"num_levels": s.num_levels, "valid": bool(s.valid), "S1": int(s.S1),
                        "S2": int(s.S2_lo) | (int(s.S2_hi) << 64), "cv": s.cv})
        self.last_status = _lib.STATUS.get(st, str(st))
        if st not in (_lib.OK, -6):        # rejected candidates are reported per entry
            check(st)
        return res

    @property
    def info(self) -> dict:
        i = _lib.BatchInfo()
        check(self._lib.rwt_batch_get_info(self._h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in i._fields_ if f != "pad_"}

    def solve_plain(self, which=None) -> None:
        """Solve the given matrices (default: all) one launch each with their
        batch plans (same schedules): the one-launch-per-matrix baseline."""
        which = range(len(self.mats)) if which is None else which
        self._enter()
        for m in which:
            L, B, X = self.mats[m]
            if B is None:
                continue
            p = C.c_void_p()
            check(self._lib.rwt_batch_plan(self._h, m, C.byref(p)))
            B2, k = _block(B, L.n, L.dtype, L.device)
            X2, _ = _block(X, L.n, L.dtype, L.device)
            check(self._lib.rwt_solve(p, _ptr(B2), k, L.n, _ptr(X2), L.n, self.stream.cuda_stream))
        self._leave()

    def plan_info(self, m: int) -> dict:
        p = C.c_void_p()
        check(self._lib.rwt_batch_plan(self._h, m, C.byref(p)))
        inf = _lib.PlanInfo()
        check(self._lib.rwt_plan_get_info(p, C.byref(inf)))
        algo = ("walk" if inf.algo_fwd == _lib.ALGO["walk"] else
                "one workgroup" if inf.num_blocks == 1 else "sync-free blocks")
        return {"algo": algo, "chunk_rounds": inf.chunk_rounds,
                "block_rows": inf.block_rows, "lanes_per_row": inf.lanes_per_row,
                "rhs_chunk": inf.rhs_chunk, "num_blocks": inf.num_blocks,
                "tuned_ms": inf.tuned_ms_syncfree}


def tall_block_order(rowptr, colidx, a: int = 0, b: int = 0) -> np.ndarray:
    """Topological row order (new -> old) whose consecutive rows form tiles
    of whole dependency chains, for the sync-free solve (host code; tile of
    a positions along a chain of chains by b chains of chains, 0: 4 and 8).
    rowptr and colidx are L's pattern as host arrays."""
    lib = _lib.load()
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(colidx, dtype=np.int32)
    n = rp.shape[0] - 1
    if n < 0:
        raise ValueError("rowptr needs n + 1 entries")
    if n > 0 and (rp[0] != 0 or np.any(np.diff(rp) < 0)):
        raise ValueError("rowptr must start at 0 and be non-decreasing")
    if ci.shape[0] < (int(rp[-1]) if n > 0 else 0):
        raise ValueError(f"colidx has {ci.shape[0]} entries, rowptr[n] = {int(rp[-1])}")
    perm = np.empty(n, dtype=np.int32)
    check(lib.rwt_tall_block_order(n, rp.ctypes.data, ci.ctypes.data, a, b, perm.ctypes.data))
    return perm


def probe_handoff(rounds: int = 2000) -> float:
    """One-way cross-workgroup hand-off latency on the current device, in ns."""
    lib = _lib.load()
    ws = _workspace(lib.rwt_probe_handoff_ws(rounds), "cuda")
    out = C.c_double(0.0)
    check(lib.rwt_probe_handoff(rounds, _ptr(ws), ws.numel(), C.byref(out), _stream()))
    return float(out.value)
