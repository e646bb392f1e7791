"""GPU parity of the row-order walk (one wavefront per right-hand-side
column walking the rows in order, 64 at a time): forward and transposed
solves against the FP64 oracle on every structure -- including a chain (a
chunk spans 64 levels), a hub row longer than the chunk stage, a dense
block and n = 1 -- its choice by the autotuner, run-to-run bit identity,
and the batched walks (solves and candidate levels) against the oracle and
against the single-matrix plan with the same schedule."""
import numpy as np
import pytest
import torch

import synth
from gpu_helpers import DEV, block, host, matrices_small, relerr, to_gpu

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


@pytest.mark.parametrize("name", list(matrices_small()))
def test_walk_solves_match_oracle(orc, name):
    from paper_2609_40159_amd.api import Plan
    L = matrices_small()[name]
    rng = np.random.default_rng(2)
    for k in (1, 5):
        B = rng.standard_normal((k, L.n))
        ref = orc.solve(L.n, L.rowptr, L.colidx, L.vals, B)
        refT = orc.solve_transpose(L.n, L.rowptr, L.colidx, L.vals, B)
        for dt in (torch.float64, torch.float32):
            print(f"walk: {name} k={k} {dt}", flush=True)
            plan = Plan(to_gpu(L, dt), algo="walk", kmax=k)
            assert plan.info["algo_fwd"] == "walk"
            X = plan.solve(block(B, dt))
            Y = plan.solve_transpose(block(B, dt))
            plan.check()
            assert relerr(host(X).astype(np.float64), ref) <= TOL[dt], (k, dt)
            assert relerr(host(Y).astype(np.float64), refT) <= TOL[dt], (k, dt)


def test_walk_in_place_repeat_and_powerlaw(orc):
    from paper_2609_40159_amd.api import Plan
    L = synth.power_law(200_000, 41)
    xs, B = synth.rhs(L, 3, 9)
    ref = orc.solve(L.n, L.rowptr, L.colidx, L.vals, B)
    refT = orc.solve_transpose(L.n, L.rowptr, L.colidx, L.vals, B)
    G = to_gpu(L)
    plan = Plan(G, algo="walk", kmax=3)
    Bt = block(B)
    X1 = plan.solve(Bt)
    Y1 = plan.solve_transpose(Bt)
    for _ in range(4):
        assert torch.equal(plan.solve(Bt), X1)
        assert torch.equal(plan.solve_transpose(Bt), Y1)
    B2 = Bt.clone()
    plan.solve(B2, out=B2)
    assert torch.equal(B2, X1)
    plan.check()
    assert relerr(host(X1), ref) <= 1e-12 and relerr(host(X1), xs) <= 1e-12
    assert relerr(host(Y1), refT) <= 1e-12
    info = plan.info
    assert info["chunk_rounds"] <= 12.0


def test_autotuner_considers_the_walk_where_it_fits():
    from paper_2609_40159_amd.api import Plan
    pl = Plan(to_gpu(synth.power_law(50_000, 43)), algo="auto", kmax=2)
    assert pl.info["chunk_rounds"] <= 12.0 and pl.info["tuned_ms_walk"] > 0
    grid = Plan(to_gpu(synth.laplacian_3d(30, 30, 30)), algo="auto")
    assert grid.info["chunk_rounds"] > 12.0 and grid.info["tuned_ms_walk"] == 0
    assert grid.info["algo_fwd"] != "walk"


def test_batched_walks_match_oracle_and_plan(orc):
    """Mixed batch: power-law matrices take the walk (solves and candidate
    levels), grids the sync-free blocks; solves equal the single-matrix
    plan with the same schedule bit for bit and the oracle within 1e-12,
    candidate statistics equal the oracle's, over graph replays."""
    from paper_2609_40159_amd.api import Batch, Plan
    mats = [("powerlaw_30k", synth.power_law(30_000, 51), 3),
            ("lap2d_100", synth.laplacian_2d(100, 100), 2),
            ("powerlaw_8k", synth.power_law(8_000, 52), 1),
            ("lap3d_20", synth.laplacian_3d(20, 20, 20), 4)]
    gm, refs, cand_mat, rows_l, cref = [], [], [], [], []
    for m, (name, L, k) in enumerate(mats):
        xs, B = synth.rhs(L, k, 60 + m)
        Bd = block(B)
        gm.append((to_gpu(L), Bd, torch.empty_like(Bd)))
        refs.append(orc.solve(L.n, L.rowptr, L.colidx, L.vals, B))
        a = orc.analyze(L.n, L.rowptr, L.colidx)
        for c in range(6):
            rows, _ = synth.random_rowset(a.level, 0.005 + 0.002 * c, [70 + m, c])
            rw = orc.rewrite(L.n, L.rowptr, L.colidx, L.vals, a.level, rows, None)
            b = orc.analyze(L.n, rw.rowptr, rw.colidx)
            cand_mat.append(m)
            rows_l.append(rows)
            cref.append((b.num_levels, b.S1, b.S2, b.cv))
    ptr = np.concatenate([[0], np.cumsum([len(r) for r in rows_l])]).astype(np.int32)
    rows = np.concatenate(rows_l).astype(np.int32)
    bt = Batch(gm, cand_mat, torch.as_tensor(ptr, device=DEV), torch.as_tensor(rows, device=DEV),
               None, pattern_cap=256 * rows.size)
    kinds = [bt.plan_info(m)["algo"] for m in range(len(mats))]
    assert kinds[0] == "walk" and kinds[2] == "walk"
    assert kinds[1] != "walk" and kinds[3] != "walk"
    bt.capture()
    for rep in range(3):
        bt.launch()
        torch.cuda.synchronize()
        st = bt.stats()
        assert bt.last_status == "OK"
        for m, ((G, Bd, Xd), ref) in enumerate(zip(gm, refs)):
            assert relerr(host(Xd), ref) <= 1e-12, (mats[m][0], rep)
        for c, want in enumerate(cref):
            g = st[c]
            assert (g["num_levels"], g["S1"], g["S2"], g["cv"]) == want, (c, rep)
    # the single-matrix plan with the same schedule gives the same bits
    for m in (0, 2):
        G, Bd, Xd = gm[m]
        pl = Plan(G, algo="walk", kmax=Bd.shape[0])
        assert torch.equal(pl.solve(Bd), Xd)
    # the walk forced for every matrix's candidates gives the same statistics
    bt2 = Batch(gm, cand_mat, torch.as_tensor(ptr, device=DEV), torch.as_tensor(rows, device=DEV),
                None, pattern_cap=256 * rows.size, cand_mode="walk")
    bt2.run()
    torch.cuda.synchronize()
    st2 = bt2.stats()
    for c, want in enumerate(cref):
        g = st2[c]
        assert (g["num_levels"], g["S1"], g["S2"], g["cv"]) == want, ("forced walk", c)
