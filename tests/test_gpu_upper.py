"""GPU parity of the upper-triangular solves and the L-then-U pair against
the oracle's backward substitution: every schedule, FP64 and FP32, several
right-hand sides, in place, after a value refresh, at full size (128^3 and
power-law 1M), and the validation of U reported on U's rows."""
import numpy as np
import pytest
import scipy.sparse
import torch

import synth
from gpu_helpers import DEV, block, host, relerr, to_gpu

pytestmark = pytest.mark.gpu


def uppers():
    n = 500
    chain = synth.CSR(n, np.concatenate([np.arange(0, 2 * n - 1, 2), [2 * n - 1]]).astype(np.int32),
                      np.concatenate([[i, i + 1] for i in range(n - 1)] + [[n - 1]]).astype(np.int32),
                      np.concatenate([[2.0, -0.7] for _ in range(n - 1)] + [[2.0]]))
    return {
        "lap2d_60x50": synth.transpose_upper(synth.laplacian_2d(60, 50)),
        "lap3d_14x12x10": synth.transpose_upper(synth.laplacian_3d(14, 12, 10), seed=1),
        "powerlaw_20k": synth.transpose_upper(synth.power_law(20000, 3), seed=2),
        "random_400": synth.transpose_upper(synth.random_lower(400, 0.05, 4), seed=3),
        "chain_500": chain,
        "diag_300": synth.CSR(300, np.arange(301, dtype=np.int32), np.arange(300, dtype=np.int32),
                              np.linspace(1, 2, 300)),
        "single": synth.CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([3.0])),
    }


def lower_of_transpose(U):
    """CSR of U^T (lower triangular), for the oracle's forward solve."""
    A = scipy.sparse.csr_matrix((U.vals, U.colidx, U.rowptr), shape=(U.n, U.n)).T.tocsr()
    A.sort_indices()
    return synth.CSR(U.n, A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data)


@pytest.mark.parametrize("name", sorted(uppers()))
@pytest.mark.parametrize("algo", ["auto", "level", "syncfree"])
def test_upper_solve_matches_oracle(orc, name, algo):
    from paper_2609_40159_amd.api import UpperPlan
    U = uppers()[name]
    xs, B = synth.rhs(U, 3, 5)
    ref = orc.solve_upper(U.n, U.rowptr, U.colidx, U.vals, B)
    assert relerr(ref, xs) <= 1e-12
    up = UpperPlan(to_gpu(U), algo=algo, kmax=3)
    X = up.solve(block(B))
    up.check()
    assert relerr(host(X), ref) <= 1e-12, name
    # the transposed solve: U^T y = g is a forward solve with U^T
    G = np.random.default_rng(7).standard_normal((2, U.n))
    Lt = lower_of_transpose(U)
    refT = orc.solve(U.n, Lt.rowptr, Lt.colidx, Lt.vals, G)
    Y = up.solve_transpose(block(G))
    assert relerr(host(Y), refT) <= 1e-12, name


@pytest.mark.parametrize("name", ["lap3d_14x12x10", "powerlaw_20k"])
def test_upper_outside_staging_agrees(orc, name):
    """Upper solves with the helper waves' staging of outside values on and
    off: bit-identical, and equal to the oracle's backward substitution."""
    from paper_2609_40159_amd.api import UpperPlan
    U = uppers()[name]
    xs, B = synth.rhs(U, 3, 6)
    ref = orc.solve_upper(U.n, U.rowptr, U.colidx, U.vals, B)
    G = to_gpu(U)
    out = {}
    for st in ("on", "off"):
        up = UpperPlan(G, algo="syncfree", kmax=3, block_rows=128, stage_outside=st)
        assert up.info["stage_outside"] == st and up.info["num_blocks"] > 1
        X = up.solve(block(B))
        Y = up.solve_transpose(block(B))
        up.check()
        assert relerr(host(X), ref) <= 1e-12, st
        out[st] = (X, Y)
    assert torch.equal(out["on"][0], out["off"][0]) and torch.equal(out["on"][1], out["off"][1])


def test_upper_solve_fp32_and_in_place(orc):
    from paper_2609_40159_amd.api import UpperPlan
    U = synth.transpose_upper(synth.power_law(30000, 9), seed=4)
    xs, B = synth.rhs(U, 2, 6)
    ref = orc.solve_upper(U.n, U.rowptr, U.colidx, U.vals, B)
    up = UpperPlan(to_gpu(U, torch.float32), kmax=2)
    X = up.solve(block(B, torch.float32))
    assert relerr(host(X).astype(np.float64), ref) <= 1e-5
    up64 = UpperPlan(to_gpu(U), kmax=2)
    Bd = block(B)
    up64.solve(Bd, out=Bd)                        # in place
    assert relerr(host(Bd), ref) <= 1e-12


def test_solve_pair_matches_oracle(orc):
    from paper_2609_40159_amd.api import Plan, UpperPlan, solve_pair
    for seed, Lh in enumerate([synth.laplacian_2d(80, 70), synth.power_law(40000, 12),
                               synth.random_lower(600, 0.03, 13)]):
        Uh = synth.transpose_upper(synth.power_law(Lh.n, 20 + seed) if Lh.n > 1000
                                   else synth.random_lower(Lh.n, 0.03, 30), seed=40 + seed)
        B = np.random.default_rng(seed).standard_normal((4, Lh.n))
        ref = orc.solve_pair(Lh.n, Lh.rowptr, Lh.colidx, Lh.vals, Uh.rowptr, Uh.colidx, Uh.vals, B)
        Lp = Plan(to_gpu(Lh), kmax=4)
        Up = UpperPlan(to_gpu(Uh), kmax=4)
        X = solve_pair(Lp, Up, block(B))
        Lp.check()
        Up.check()
        assert relerr(host(X), ref) <= 1e-12, seed
        Bd = block(B)
        solve_pair(Lp, Up, Bd, out=Bd)
        assert relerr(host(Bd), ref) <= 1e-12, seed


def test_upper_refresh_takes_new_values(orc):
    from paper_2609_40159_amd.api import UpperPlan
    U = synth.transpose_upper(synth.laplacian_2d(50, 40), seed=8)
    G = to_gpu(U)
    up = UpperPlan(G, kmax=1)
    B = np.random.default_rng(2).standard_normal((1, U.n))
    new_vals = U.vals * np.where(np.isin(np.arange(U.vals.size), U.rowptr[:-1]), 1.5, -0.5)
    G.vals.copy_(torch.as_tensor(new_vals, device=DEV))
    stale = host(up.solve(block(B)))
    ref_old = orc.solve_upper(U.n, U.rowptr, U.colidx, U.vals, B)
    assert relerr(stale, ref_old) <= 1e-12          # the plan's copy until refreshed
    up.refresh()
    ref_new = orc.solve_upper(U.n, U.rowptr, U.colidx, new_vals, B)
    assert relerr(host(up.solve(block(B))), ref_new) <= 1e-12


def test_upper_full_size(orc):
    from paper_2609_40159_amd.api import Plan, UpperPlan, solve_pair
    print("upper parity: lap3d_128 pair", flush=True)
    Lh = synth.laplacian_3d(128, 128, 128)
    Uh = synth.transpose_upper(Lh)
    B = np.random.default_rng(3).standard_normal((1, Lh.n))
    ref = orc.solve_pair(Lh.n, Lh.rowptr, Lh.colidx, Lh.vals, Uh.rowptr, Uh.colidx, Uh.vals, B)
    Lp = Plan(to_gpu(Lh), kmax=1)
    Up = UpperPlan(to_gpu(Uh), kmax=1)
    X = solve_pair(Lp, Up, block(B))
    Up.check()
    assert relerr(host(X), ref) <= 1e-12
    print("upper parity: powerlaw_1m, 16 right-hand sides", flush=True)
    Uh = synth.transpose_upper(synth.power_law(1 << 20, 7), seed=9)
    xs, B = synth.rhs(Uh, 16, 4)
    ref = orc.solve_upper(Uh.n, Uh.rowptr, Uh.colidx, Uh.vals, B)
    Up = UpperPlan(to_gpu(Uh), kmax=16)
    X = Up.solve(block(B))
    Up.check()
    assert relerr(host(X), ref) <= 1e-12


def test_upper_validation_reports_rows():
    from paper_2609_40159_amd import _lib
    from paper_2609_40159_amd.api import CSRMatrix, UpperPlan

    def make(rows, vals=None):
        n = len(rows)
        rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
        ci = np.concatenate([np.asarray(r, np.int32) for r in rows])
        va = np.ones(ci.size) if vals is None else np.asarray(vals, np.float64)
        return CSRMatrix.from_arrays(rp, ci, va, device=DEV)

    good = [[0, 2], [1, 3], [2], [3]]
    UpperPlan(make(good))
    cases = [([[0, 2], [0, 1], [2], [3]], "NOT_LOWER", 1),      # entry below the diagonal
             ([[0, 2], [1, 3], [2, 3, 3], [3]], "UNSORTED_OR_DUP", 2),
             ([[0, 2], [3], [2], [3]], "MISSING_DIAG", 1),        # no diagonal first
             ([[0, 2], [1, 3], [2], [3]], "ZERO_DIAG", 1)]
    for rows, code, row in cases:
        vals = None
        if code == "ZERO_DIAG":
            vals = [1, 1, 0, 1, 1, 1]
        with pytest.raises(_lib.RwtError) as ei:
            UpperPlan(make(rows, vals))
        assert ei.value.name == code, (rows, ei.value)
        assert f"U row {row}" in str(ei.value), (rows, ei.value)


@pytest.mark.parametrize("which", ["lap3d_20x18x16", "powerlaw_30k", "lap3d_128"])
def test_apply_M_and_pair_with_rewritten_factor(orc, which):
    """M B equals the rewrite's B' bit for bit, and the pair with the
    rewritten factor, U^{-1} L'^{-1} (M B), equals U^{-1} L^{-1} B."""
    from paper_2609_40159_amd.api import Plan, UpperPlan, analyze, apply_M, rewrite, solve_pair
    Lh = {"lap3d_20x18x16": lambda: synth.laplacian_3d(20, 18, 16),
          "powerlaw_30k": lambda: synth.power_law(30000, 17),
          "lap3d_128": lambda: synth.laplacian_3d(128, 128, 128)}[which]()
    Uh = synth.transpose_upper(Lh, seed=5)
    print(f"rewritten pair: {which}", flush=True)
    k = 1 if which == "lap3d_128" else 3
    G = to_gpu(Lh)
    info = analyze(G)
    lv = host(info.level)
    rows, targets = synth.thin_first_rows(lv, 0.01 if which != "powerlaw_30k" else 0.008)
    B = np.random.default_rng(11).standard_normal((k, Lh.n))
    rw = rewrite(G, info.level, torch.as_tensor(rows, device=DEV),
                 torch.as_tensor(targets, device=DEV), block(B))
    MB = apply_M(rw, block(B))
    assert torch.equal(MB, rw.B.reshape(MB.shape))
    Lp = Plan(rw.L, kmax=k)
    Up = UpperPlan(to_gpu(Uh), kmax=k)
    X = solve_pair(Lp, Up, MB)
    Lp.check()
    ref = orc.solve_pair(Lh.n, Lh.rowptr, Lh.colidx, Lh.vals, Uh.rowptr, Uh.colidx, Uh.vals, B)
    assert relerr(host(X), ref) <= 1e-12
