"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module only *draws* inputs: sparse lower-triangular matrices in CSR
form, right-hand sides built from a known solution, and the row sets that
say which rows get rewritten.  It contains none of the method's arithmetic
(no level computation, no rewriting, no triangular solve); functions that
choose rows from a level array receive that array as an argument.

Matrix families (the paper's SuiteSparse inputs are not available; these
stand in for the two regimes it covers -- wide PDE levels and deep, thin
levels, Section 5, Table 2):

* ``laplacian_2d`` / ``laplacian_3d``: lower triangle (diagonal included) of
  the 5-point / 7-point Laplacian in natural order, x fastest.
* ``power_law``: off-diagonal row counts Pareto(alpha=2, x_m=4) capped at
  2000, dependency distances geometric (mean 200) truncated at min(1e4, i),
  values N(0,1)/k_i off the diagonal and U[1,2] on it.

CSR convention everywhere: int32 ``rowptr[n+1]``, int32 ``colidx[nnz]``
strictly ascending within a row with the diagonal stored last, float64
``vals[nnz]``.  Dense blocks of k right-hand sides are column-major n x k,
held in NumPy as an array of shape (k, n) (column q contiguous).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSR", "laplacian_2d", "laplacian_3d", "power_law", "random_lower",
    "rhs", "longest_path_rows", "thin_first_rows", "random_rowset",
    "batch_manifest", "build_matrix", "WORKLOADS",
]


@dataclass
class CSR:
    n: int
    rowptr: np.ndarray  # int32 [n+1]
    colidx: np.ndarray  # int32 [nnz]
    vals: np.ndarray    # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def row_of_entry(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int32), np.diff(self.rowptr))

    def to_dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n))
        a[self.row_of_entry(), self.colidx] = self.vals
        return a

    def astype(self, dtype) -> "CSR":
        return CSR(self.n, self.rowptr, self.colidx, self.vals.astype(dtype))


def _assemble(n: int, cols_per_row: list[np.ndarray] | None, rowptr: np.ndarray,
              colidx: np.ndarray, vals: np.ndarray) -> CSR:
    return CSR(n, rowptr.astype(np.int32), colidx.astype(np.int32),
               vals.astype(np.float64))


def _stencil_lower(dims: tuple[int, ...], diag: float, off: float) -> CSR:
    """Lower triangle of the (2*len(dims)+1)-point Laplacian, natural order."""
    n = int(np.prod(dims))
    strides = [1]
    for d in dims[:-1]:
        strides.append(strides[-1] * d)
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx.copy()
    for d in dims:
        coords.append(rem % d)
        rem //= d
    # candidate dependencies: one per axis with coordinate > 0, ordered by
    # ascending column, i.e. descending stride
    has = [coords[a] > 0 for a in range(len(dims))]
    cnt = np.ones(n, dtype=np.int64)
    for h in has:
        cnt += h
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt, out=rowptr[1:])
    nnz = int(rowptr[-1])
    colidx = np.empty(nnz, dtype=np.int64)
    vals = np.empty(nnz, dtype=np.float64)
    pos = rowptr[:-1].copy()
    for a in reversed(range(len(dims))):
        sel = has[a]
        colidx[pos[sel]] = idx[sel] - strides[a]
        vals[pos[sel]] = off
        pos[sel] += 1
    colidx[pos] = idx
    vals[pos] = diag
    return _assemble(n, None, rowptr, colidx, vals)


def laplacian_2d(nx: int, ny: int, diag: float = 4.0, off: float = -1.0) -> CSR:
    return _stencil_lower((nx, ny), diag, off)


def laplacian_3d(nx: int, ny: int, nz: int, diag: float = 6.0, off: float = -1.0) -> CSR:
    return _stencil_lower((nx, ny, nz), diag, off)


def _trunc_geometric(rng: np.random.Generator, p: float, m: np.ndarray) -> np.ndarray:
    """Geometric(p) on {1,2,...} conditioned on d <= m (inverse CDF)."""
    u = rng.random(m.shape[0])
    q = np.log1p(-p)
    top = -np.expm1(m * q)            # P(d <= m)
    d = np.ceil(np.log1p(-u * top) / q)
    return np.clip(d, 1, m).astype(np.int64)


def power_law(n: int, seed: int, *, alpha: float = 2.0, x_m: float = 4.0,
              cap: int = 2000, dist_mean: float = 200.0, dist_cut: int = 10_000) -> CSR:
    """Random power-law lower-triangular CSR (see module docstring).

    k_i = min(cap, round(x_m * U^(-1/alpha))), then k_i = min(k_i, i); the k_i
    distances are distinct draws of a geometric variable with mean
    ``dist_mean`` restricted to [1, min(dist_cut, i)].
    """
    rng = np.random.default_rng(seed)
    p = 1.0 / dist_mean
    u = 1.0 - rng.random(n)                                   # (0, 1]
    k = np.minimum(cap, np.rint(x_m * u ** (-1.0 / alpha))).astype(np.int64)
    i_all = np.arange(n, dtype=np.int64)
    k = np.minimum(k, i_all)
    mmax = np.minimum(dist_cut, i_all)

    # Rows with many dependencies or a short support: exact successive
    # weighted sampling without replacement (exponential keys, the k smallest
    # of E_d / w_d), which is the law of "redraw until distinct".
    special = np.nonzero((k > 0) & ((k > 64) | (mmax < 4 * k)))[0]
    bulk = (k > 0)
    bulk[special] = False

    chosen_rows = []
    chosen_d = []
    # bulk rows: draw k_i, drop repeats, redraw only the shortfall
    rows0 = np.nonzero(bulk)[0]
    rr = np.repeat(rows0, k[rows0])
    dd = _trunc_geometric(rng, p, mmax[rr])
    for _ in range(1000):
        key = rr * (dist_cut + 1) + dd
        _, first = np.unique(key, return_index=True)
        first.sort()
        rr, dd = rr[first], dd[first]
        got = np.bincount(rr, minlength=n)
        short = np.where(bulk, k - got, 0)
        need_rows = np.nonzero(short > 0)[0]
        if need_rows.size == 0:
            break
        nr = np.repeat(need_rows, short[need_rows])
        nd = _trunc_geometric(rng, p, mmax[nr])
        rr = np.concatenate([rr, nr])
        dd = np.concatenate([dd, nd])
    else:  # pragma: no cover
        raise RuntimeError("power_law: distance sampling did not converge")
    chosen_rows.append(rr)
    chosen_d.append(dd)
    for i in special:
        m = int(mmax[i])
        dist = np.arange(1, m + 1)
        logw = (dist - 1) * np.log1p(-p)
        keys = np.log(rng.exponential(size=m)) - logw
        d = dist[np.argpartition(keys, int(k[i]) - 1)[: int(k[i])]]
        chosen_rows.append(np.full(d.shape[0], i, dtype=np.int64))
        chosen_d.append(d.astype(np.int64))
    rows = np.concatenate(chosen_rows)
    cols = rows - np.concatenate(chosen_d)
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order]

    offcnt = np.bincount(rows, minlength=n)
    assert np.array_equal(offcnt, k)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(offcnt + 1, out=rowptr[1:])
    nnz = int(rowptr[-1])
    colidx = np.empty(nnz, dtype=np.int64)
    vals = np.empty(nnz, dtype=np.float64)
    off_pos = np.arange(rows.size) + rows          # shift by one diagonal per earlier row
    offvals = rng.standard_normal(rows.size) / k[rows]
    colidx[off_pos] = cols
    vals[off_pos] = offvals
    diag_pos = rowptr[1:] - 1
    colidx[diag_pos] = i_all
    vals[diag_pos] = rng.uniform(1.0, 2.0, n)
    return _assemble(n, None, rowptr, colidx, vals)


def random_lower(n: int, density: float, seed: int, *, diag_lo: float = 1.0,
                 diag_hi: float = 2.0) -> CSR:
    """Small dense-ish random lower-triangular matrix for brute-force tests."""
    rng = np.random.default_rng(seed)
    mask = np.tril(rng.random((n, n)) < density, k=-1)
    rows, cols = np.nonzero(mask)
    offcnt = np.bincount(rows, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(offcnt + 1, out=rowptr[1:])
    colidx = np.empty(int(rowptr[-1]), dtype=np.int64)
    vals = np.empty(int(rowptr[-1]), dtype=np.float64)
    off_pos = np.arange(rows.size) + rows
    colidx[off_pos] = cols
    vals[off_pos] = rng.standard_normal(rows.size) / np.maximum(1, offcnt[rows])
    colidx[rowptr[1:] - 1] = np.arange(n)
    vals[rowptr[1:] - 1] = rng.uniform(diag_lo, diag_hi, n)
    return _assemble(n, None, rowptr, colidx, vals)


def transpose_upper(L: CSR, seed: int | None = None) -> CSR:
    """U = L^T as an upper-triangular CSR (rows hold the diagonal first, then
    ascending columns).  With a seed, the values are redrawn: off-diagonal
    N(0,1)/(entries in the row), diagonal U[1,2] -- the second factor of an
    incomplete-LU-like pair with the pattern of L^T."""
    n = L.n
    rows = L.row_of_entry()
    order = np.argsort(L.colidx, kind="stable")     # by U row, then by U column
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(L.colidx, minlength=n), out=rowptr[1:])
    colidx = rows[order].astype(np.int32)
    vals = L.vals[order].copy()
    if seed is not None:
        rng = np.random.default_rng([seed, 11])
        cnt = np.diff(rowptr)
        vals = rng.standard_normal(colidx.size) / np.maximum(1, np.repeat(cnt - 1, cnt))
        vals[rowptr[:-1]] = rng.uniform(1.0, 2.0, n)
    return CSR(n, rowptr.astype(np.int32), colidx, vals)


def rhs(L: CSR, k: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """x* ~ U[-1,1] (shape (k, n), column q contiguous) and B = L x* in FP64.

    B is formed row by row with ascending columns: it is an input of the
    solve, not a step of it.
    """
    rng = np.random.default_rng([seed, 7])
    xs = rng.uniform(-1.0, 1.0, (k, L.n))
    rowidx = L.row_of_entry()
    B = np.empty_like(xs)
    for q in range(k):
        prod = L.vals * xs[q, L.colidx]
        B[q] = np.bincount(rowidx, weights=prod, minlength=L.n)
    return xs, B


# ---------------------------------------------------------------------------
# Row-set rules.  Each takes an already computed level array (one int per
# row); none of them computes levels itself.
# ---------------------------------------------------------------------------

def longest_path_rows(L: CSR, level: np.ndarray, frac: float = 0.01) -> np.ndarray:
    """Rows on one longest dependency path, lowest index first.

    Start at the lowest-index row on the deepest level; repeatedly step to
    the lowest-index dependency that sits exactly one level lower.  Level-0
    rows are dropped; the first floor(frac*n) rows in ascending order are
    returned.
    """
    level = np.asarray(level)
    D = int(level.max()) + 1
    r = int(np.nonzero(level == D - 1)[0][0])
    path = [r]
    while level[r] > 0:
        cols = L.colidx[L.rowptr[r]:L.rowptr[r + 1] - 1]
        cand = cols[level[cols] == level[r] - 1]
        r = int(cand.min())
        path.append(r)
    path = np.array(sorted(p for p in path if level[p] > 0), dtype=np.int32)
    return path[: int(np.floor(frac * L.n))]


def thin_first_rows(level: np.ndarray, frac: float) -> tuple[np.ndarray, np.ndarray]:
    """Whole thin levels, thinnest first, up to floor(frac*n) rows.

    Levels 1..D-1 are ordered by (row count, level index) and taken while the
    running total stays <= floor(frac*n) (stop at the first that does not
    fit).  Returns (rows ascending, targets = level - 1).
    """
    level = np.asarray(level)
    n = level.shape[0]
    D = int(level.max()) + 1
    cnt = np.bincount(level, minlength=D)
    cap = int(np.floor(frac * n))
    order = sorted(range(1, D), key=lambda l: (int(cnt[l]), l))
    take = []
    tot = 0
    for l in order:
        if tot + int(cnt[l]) > cap:
            break
        tot += int(cnt[l])
        take.append(l)
    sel = np.isin(level, np.array(take, dtype=level.dtype))
    rows = np.nonzero(sel)[0].astype(np.int32)
    return rows, (level[rows] - 1).astype(np.int32)


def random_rowset(level: np.ndarray, frac: float, seed) -> tuple[np.ndarray, np.ndarray]:
    """Uniform sample (no replacement) of floor(frac*n) rows with level >= 1."""
    level = np.asarray(level)
    rng = np.random.default_rng(seed)
    elig = np.nonzero(level >= 1)[0]
    m = min(int(np.floor(frac * level.shape[0])), elig.size)
    rows = np.sort(rng.choice(elig, size=m, replace=False)).astype(np.int32)
    return rows, (level[rows] - 1).astype(np.int32)


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def batch_manifest(count: int = 256, seed_base: int = 1000, n_lo: int = 2000,
                   n_hi: int = 200_000, k_lo: int = 1, k_hi: int = 16,
                   candidates: int = 32) -> list[dict]:
    """Uneven batch: first quarter 2D, second quarter 3D, second half power-law."""
    out = []
    for m in range(count):
        rng = np.random.default_rng(seed_base + m)
        n_target = int(rng.integers(n_lo, n_hi + 1))
        k = int(rng.integers(k_lo, k_hi + 1))
        if m < count // 4:
            side = max(2, int(round(np.sqrt(n_target))))
            spec = {"kind": "lap2d", "dims": (side, side)}
        elif m < count // 2:
            side = max(2, int(round(np.cbrt(n_target))))
            spec = {"kind": "lap3d", "dims": (side, side, side)}
        else:
            spec = {"kind": "powerlaw", "n": n_target, "seed": seed_base + m}
        phis = rng.uniform(0.005, 0.015, candidates)
        spec.update({"index": m, "k": k, "phis": phis.tolist(),
                     "cand_seeds": [(seed_base + m, c) for c in range(candidates)]})
        out.append(spec)
    return out


def build_matrix(spec: dict) -> CSR:
    kind = spec["kind"]
    if kind == "lap2d":
        return laplacian_2d(*spec["dims"])
    if kind == "lap3d":
        return laplacian_3d(*spec["dims"])
    if kind == "powerlaw":
        return power_law(spec["n"], spec["seed"])
    raise ValueError(kind)


def _batch_member(spec: dict):
    L = build_matrix(spec)
    k = spec["k"]
    xs, B = rhs(L, k, spec["index"] + 1) if k > 0 else (None, None)
    return L, xs, B


def build_batch(manifest: list[dict], workers: int = 1) -> list[tuple]:
    """(L, x*, B) of every manifest entry, optionally in forked worker
    processes (call before any GPU use in the parent)."""
    if workers <= 1:
        return [_batch_member(s) for s in manifest]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_batch_member, manifest, chunksize=1)


def candidate_rows(spec: dict, level: np.ndarray, c: int) -> np.ndarray:
    """Candidate c of a batched matrix: a uniform sample of floor(phi_c * n)
    rows with level >= 1 (seed (matrix seed, c)); targets are level - 1."""
    rows, _ = random_rowset(level, spec["phis"][c], list(spec["cand_seeds"][c]))
    return rows


#: The named workloads (the paper's scale classes, synthetic stand-ins).
WORKLOADS = {
    "lap2d_64": {"kind": "lap2d", "dims": (64, 64), "k": 1, "seed": 1,
                 "rule": "longest_path", "frac": 0.01},
    "lap3d_128": {"kind": "lap3d", "dims": (128, 128, 128), "k": 1, "seed": 2,
                  "rule": "thin_first", "frac": 0.01},
    "powerlaw_1m": {"kind": "powerlaw", "n": 1_000_000, "seed": 3, "k": 64,
                    "rule": "thin_first", "frac": 0.008},
    "lap3d_64": {"kind": "lap3d", "dims": (64, 64, 64), "k": 32, "seed": 5,
                 "rule": "thin_first", "frac": 0.01},
    "powerlaw_262k": {"kind": "powerlaw", "n": 262_144, "seed": 5, "k": 32,
                      "rule": "thin_first", "frac": 0.01},
}
