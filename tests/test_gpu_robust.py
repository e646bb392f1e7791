"""Sync-free robustness on the GPU: the bounded waits (Section 7 names the
spinning of sync-free solvers as their risk) and run-to-run determinism.

The watchdog case is forced from the host: rwt_solve_withhold never
publishes one row, so its readers in other blocks wait until the plan's
watchdog expires; every wait is bounded, the kernel exits, the plan reports
DEADLOCK, and the next solve on the same plan is correct."""
import ctypes as C
import time

import numpy as np
import pytest
import torch

import synth
from gpu_helpers import block, host, relerr, to_gpu

pytestmark = pytest.mark.gpu


def _withhold(plan, row, B):
    from paper_2609_40159_amd import _lib
    lib = _lib.load()
    X = torch.empty_like(B)
    n = plan.L.n
    _lib.check(lib.rwt_solve_withhold(plan._h, row, B.data_ptr(), B.shape[0], n, X.data_ptr(), n,
                                      torch.cuda.current_stream().cuda_stream))
    return X


@pytest.mark.parametrize("algo", ["syncfree", "level"])
def test_watchdog_withheld_row_then_recovers(orc, algo):
    from paper_2609_40159_amd._lib import RwtError
    from paper_2609_40159_amd.api import Plan
    # 64 x 64 grid in natural order, 64-row blocks: row 63's only reader,
    # row 127, sits in the next block
    L = synth.laplacian_2d(64, 64)
    xs, B = synth.rhs(L, 1, 3)
    ref = orc.solve(L.n, L.rowptr, L.colidx, L.vals, B)
    plan = Plan(to_gpu(L), algo=algo, block_rows=64, narrow_rows=0, watchdog_ms=50)
    assert plan.info["algo_fwd"] == algo
    Bd = block(B)
    print(f"watchdog: {algo}, withheld row 63", flush=True)
    t0 = time.perf_counter()
    X = _withhold(plan, 63, Bd)
    with pytest.raises(RwtError) as ei:
        plan.check()                       # synchronizes: the launch has ended
    elapsed = time.perf_counter() - t0
    assert ei.value.name == "DEADLOCK"
    assert elapsed < 30.0, elapsed          # bounded waits, not a hang
    assert not np.array_equal(host(X), ref)   # the withheld value never arrived
    # the same plan solves correctly afterwards
    X2 = plan.solve(Bd)
    plan.check()
    assert relerr(host(X2), ref) <= 1e-12
    assert relerr(host(X2), xs) <= 1e-12


def test_withhold_rejects_rows_out_of_range():
    from paper_2609_40159_amd import _lib
    from paper_2609_40159_amd.api import Plan
    L = synth.laplacian_2d(8, 8)
    plan = Plan(to_gpu(L), algo="syncfree", block_rows=16)
    lib = _lib.load()
    st = lib.rwt_solve_withhold(plan._h, L.n, C.c_void_p(256), 1, L.n, C.c_void_p(512), L.n, None)
    assert _lib.STATUS[st] == "INVALID_ARG"


@pytest.mark.parametrize("name", ["powerlaw_20k", "lap3d_24", "rewritten_lap3d_32"])
def test_repeated_solves_bit_identical(orc, name):
    """Randomized row-block sizes and staging: every repeat of the forward
    and the transposed solve is bit-identical to the first solve (the
    per-row sums run in a fixed order whatever the schedule), and the
    oracle agrees within 1e-12."""
    from paper_2609_40159_amd.api import Plan, analyze, rewrite
    if name == "powerlaw_20k":
        L = synth.power_law(20000, 31)
    elif name == "lap3d_24":
        L = synth.laplacian_3d(24, 24, 24)
    else:
        L0 = synth.laplacian_3d(32, 32, 32)
        a = orc.analyze(L0.n, L0.rowptr, L0.colidx)
        rows, tg = synth.thin_first_rows(a.level, 0.01)
        rw = orc.rewrite(L0.n, L0.rowptr, L0.colidx, L0.vals, a.level, rows, tg)
        L = synth.CSR(L0.n, rw.rowptr, rw.colidx, rw.vals)
    k = 2
    B = np.random.default_rng(9).standard_normal((k, L.n))
    ref = orc.solve(L.n, L.rowptr, L.colidx, L.vals, B)
    refT = orc.solve_transpose(L.n, L.rowptr, L.colidx, L.vals, B)
    G = to_gpu(L)
    Bd = block(B)
    rng = np.random.default_rng(sum(map(ord, name)))
    sizes = sorted(set([int(x) for x in rng.integers(1, 4097, 4)] + [64]))
    first = None
    for R in sizes:
        stage = ["on", "off"][int(rng.integers(2))]
        print(f"determinism: {name} block_rows={R} stage={stage}", flush=True)
        plan = Plan(G, algo="syncfree", kmax=k, block_rows=R, lanes_per_row=4,
                    stage_outside=stage)
        for rep in range(6):
            X = plan.solve(Bd)
            Y = plan.solve_transpose(Bd)
            plan.check()
            if first is None:
                first = (X.clone(), Y.clone())
                assert relerr(host(X), ref) <= 1e-12
                assert relerr(host(Y), refT) <= 1e-12
            assert torch.equal(X, first[0]), (R, rep)
            assert torch.equal(Y, first[1]), (R, rep)
