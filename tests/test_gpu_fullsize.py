"""GPU parity at the benchmark's full sizes, in the launch configurations it
times, element by element against the FP64 oracle.

- The batched workload's members across its whole size range (the largest
  2D, 3D and power-law factors of the 256-matrix batch, whose deepest
  member has 13,246 levels, and small ones), each with its right-hand
  sides and its 32 candidate rewrite sets, in one captured launch replayed
  twice: solves within 1e-12, candidate statistics (levels, S1, exact S2,
  CV) bit-exact against the oracle's rewrite + analysis (Sections 2.1, 2.2).
- The 128^3 factor with 1% of its rows rewritten, one right-hand side, the
  autotuned plan: forward and transposed solves in FP64 (1e-12) and FP32
  (1e-5) against the oracle's solves of the oracle's rewritten matrix, and
  the forward result against the original system's solution."""
import numpy as np
import pytest
import torch

import synth
from gpu_helpers import DEV, block, host, relerr, to_gpu

pytestmark = pytest.mark.gpu

# batch members (index in the 256-matrix manifest): the three largest of
# each kind, the deepest power-law factor (193: n = 197,595, 13,246 levels)
# among them, and the smallest of each kind
MEMBERS = [58, 17, 61, 66, 92, 105, 193, 172, 203, 46, 115, 153]


def test_batch_members_full_size_vs_oracle(orc):
    from paper_2609_40159_amd.api import Batch
    man = synth.batch_manifest(256)
    specs = [man[i] for i in MEMBERS]
    mats, refs, cand_mat, rows_l, cand_ref = [], [], [], [], []
    for spec in specs:
        L = synth.build_matrix(spec)
        xs, B = synth.rhs(L, spec["k"], spec["index"] + 1)
        G = to_gpu(L)
        Bd = block(B)
        mats.append((G, Bd, torch.empty_like(Bd)))
        refs.append((orc.solve(L.n, L.rowptr, L.colidx, L.vals, B), xs))
        a = orc.analyze(L.n, L.rowptr, L.colidx)
        for c in range(len(spec["phis"])):
            r = synth.candidate_rows(spec, a.level, c)
            rw = orc.rewrite(L.n, L.rowptr, L.colidx, L.vals, a.level, r, None)
            b = orc.analyze(L.n, rw.rowptr, rw.colidx)
            cand_mat.append(len(mats) - 1)
            rows_l.append(r)
            cand_ref.append((b.num_levels, b.S1, b.S2, b.cv))
        print(f"full-size batch member {spec['index']} ({spec['kind']}, n={L.n}, "
              f"levels={a.num_levels}, k={spec['k']}) prepared", flush=True)
    ptr = np.concatenate([[0], np.cumsum([len(r) for r in rows_l])]).astype(np.int32)
    rows = np.concatenate(rows_l).astype(np.int32)
    d_rows = torch.as_tensor(rows, device=DEV)
    d_ptr = torch.as_tensor(ptr, device=DEV)
    bt = Batch(mats, cand_mat, d_ptr, d_rows, None, pattern_cap=256 * max(1, rows.size))
    bt.capture()
    for rep in range(2):
        for _, _, Xd in mats:
            Xd.fill_(0.0)
        print(f"full-size batch: launch {rep}", flush=True)
        bt.launch()
        torch.cuda.synchronize()
        st = bt.stats()
        assert bt.last_status == "OK"
        for m, ((_, _, Xd), (ref, xs)) in enumerate(zip(mats, refs)):
            assert relerr(host(Xd), ref) <= 1e-12, (MEMBERS[m], rep)
            assert relerr(host(Xd), xs) <= 1e-12, (MEMBERS[m], rep)
        for c, (D, S1, S2, cv) in enumerate(cand_ref):
            g = st[c]
            assert g["valid"]
            assert (g["num_levels"], g["S1"], g["S2"], g["cv"]) == (D, S1, S2, cv), \
                (MEMBERS[cand_mat[c]], c, rep)


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_rewritten_128_tuned_forward_and_transposed(orc, dt):
    from paper_2609_40159_amd.api import Plan, Rewriter, analyze
    tol = 1e-12 if dt == torch.float64 else 1e-5
    L = synth.laplacian_3d(128, 128, 128)
    xs, B = synth.rhs(L, 1, 2)
    Gh = np.random.default_rng(102).standard_normal((1, L.n))
    a = orc.analyze(L.n, L.rowptr, L.colidx)
    rows, tg = synth.thin_first_rows(a.level, 0.01)
    rw = orc.rewrite(L.n, L.rowptr, L.colidx, L.vals, a.level, rows, tg, B)
    refX = orc.solve(L.n, rw.rowptr, rw.colidx, rw.vals, rw.Bp)
    refY = orc.solve_transpose(L.n, rw.rowptr, rw.colidx, rw.vals, Gh)
    print(f"rewritten 128^3 ({dt}): oracle done", flush=True)
    G = to_gpu(L, dt)
    info = analyze(G)
    r = Rewriter(G, info.level, torch.as_tensor(rows, device=DEV), torch.as_tensor(tg, device=DEV))
    Bp = r.numeric(None, block(B, dt))
    assert np.array_equal(host(r.Lp.rowptr), rw.rowptr)
    assert np.array_equal(host(r.Lp.colidx), rw.colidx)
    plan = Plan(r.Lp, algo="auto", kmax=1)
    print(f"rewritten 128^3 ({dt}): plan {plan.info['algo_fwd']} "
          f"block_rows={plan.info['block_rows']} stage={plan.info['stage_outside']}", flush=True)
    X = plan.solve(Bp)
    Y = plan.solve_transpose(block(Gh, dt))
    plan.check()
    assert relerr(host(X).astype(np.float64), refX) <= tol
    assert relerr(host(X).astype(np.float64), xs) <= tol
    assert relerr(host(Y).astype(np.float64), refY) <= tol
