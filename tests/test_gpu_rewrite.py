"""GPU parity: equation rewriting, patterns and (FP64) values bit-exact."""
import numpy as np
import pytest
import torch

import synth
from gpu_helpers import block, host, relerr, to_gpu

pytestmark = pytest.mark.gpu


def run_both(orc, L, rows, targets, B):
    from paper_2609_40159_amd.api import analyze, rewrite
    G = to_gpu(L)
    info = analyze(G)
    a = orc.analyze(L.n, L.rowptr, L.colidx)
    rw = rewrite(G, info.level, rows, targets, block(B))
    ref = orc.rewrite(L.n, L.rowptr, L.colidx, L.vals, a.level, rows, targets, B)
    return rw, ref


def check_same(rw, ref):
    assert np.array_equal(host(rw.L.rowptr), ref.rowptr)
    assert np.array_equal(host(rw.L.colidx), ref.colidx)
    assert np.array_equal(host(rw.L.vals), ref.vals)          # bit for bit
    assert np.array_equal(host(rw.B), ref.Bp)
    assert np.array_equal(host(rw.cptr), ref.c_ptr)
    assert np.array_equal(host(rw.ccol), ref.c_col)
    assert np.array_equal(host(rw.cval), ref.c_val)
    assert rw.skipped == ref.skipped
    rowsC = np.repeat(np.arange(len(ref.c_ptr) - 1), np.diff(ref.c_ptr))
    return rowsC


def test_rewrite_2d_longest_path(orc):
    L = synth.laplacian_2d(64, 64)
    a = orc.analyze(L.n, L.rowptr, L.colidx)
    rows = synth.longest_path_rows(L, a.level, 0.01)
    xs, B = synth.rhs(L, 1, 1)
    rw, ref = run_both(orc, L, rows, None, B)
    check_same(rw, ref)
    from paper_2609_40159_amd.api import analyze
    b = analyze(rw.L)
    assert b.num_levels == 127 and round(b.stats["cv"], 6) == 0.568720


@pytest.mark.parametrize("seed", range(6))
def test_rewrite_random_sets_and_targets(orc, seed):
    rng = np.random.default_rng(seed)
    L = synth.power_law(4000, 100 + seed) if seed % 2 else synth.random_lower(500, 0.05, seed)
    a = orc.analyze(L.n, L.rowptr, L.colidx)
    rows, _ = synth.random_rowset(a.level, 0.2, seed)
    targets = np.array([int(rng.integers(0, l + 2)) for l in a.level[rows]], np.int32)
    B = rng.standard_normal((3, L.n))
    rw, ref = run_both(orc, L, rows, targets, B)
    check_same(rw, ref)


def test_rewrite_long_rows_use_the_fallback(orc):
    """Rows longer than the LDS accumulator (hub rows, deep targets)."""
    from gpu_helpers import matrices_small
    L = matrices_small()["hub_2500"]
    a = orc.analyze(L.n, L.rowptr, L.colidx)
    rows = np.array([2000, 2001, 2100, 2499], np.int32)
    targets = np.array([0, 0, 0, 0], np.int32)
    B = np.random.default_rng(3).standard_normal((2, L.n))
    rw, ref = run_both(orc, L, rows, targets, B)
    check_same(rw, ref)
    D = synth.random_lower(900, 0.8, 5)     # dense: closures far beyond the LDS capacity
    a = orc.analyze(D.n, D.rowptr, D.colidx)
    rows = np.array([600, 700, 899], np.int32)
    rw, ref = run_both(orc, D, rows, np.zeros(3, np.int32), B[:, :900].copy())
    check_same(rw, ref)


def test_rewrite_thin_first_3d_64(orc):
    from paper_2609_40159_amd.api import Plan, analyze
    L = synth.laplacian_3d(64, 64, 64)
    a = orc.analyze(L.n, L.rowptr, L.colidx)
    rows, tg = synth.thin_first_rows(a.level, 0.01)
    xs, B = synth.rhs(L, 2, 5)
    rw, ref = run_both(orc, L, rows, tg, B)
    check_same(rw, ref)
    assert analyze(rw.L).num_levels == 172
    X = Plan(rw.L, kmax=2).solve(rw.B)
    assert relerr(host(X), xs) <= 1e-12


def test_rewrite_errors(orc):
    from paper_2609_40159_amd.api import RwtError, analyze, rewrite
    L = synth.laplacian_2d(8, 8)
    G = to_gpu(L)
    info = analyze(G)
    for rows, tg in [([5, 3], None), ([4, 4], None), ([-1], None), ([64], None), ([9], [-2])]:
        with pytest.raises(RwtError) as e:
            rewrite(G, info.level, rows, tg)
        assert e.value.name == "BAD_ROWSET"
    rw = rewrite(G, info.level, [0, 9, 10], [0, 5, 9])      # all no-ops
    assert rw.skipped == 3
    assert torch.equal(rw.L.colidx, G.colidx) and torch.equal(rw.L.vals, G.vals)
    rw = rewrite(G, info.level, [])
    assert torch.equal(rw.L.rowptr, G.rowptr)
