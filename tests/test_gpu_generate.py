"""GPU parity of the rewrite-list generator (one wave per environment)
against the oracle: the triplets, the run summaries and the final per-level
sums bit for bit, on the hand-worked cases, on small matrices of every
structure with a grid of parameters, at full size (128^3 Laplacian; the
power-law 1M matrix on step-limited runs plus invariants of a full run), and
the candidate row sets it hands to the rewrite and to the batch."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from gpu_helpers import DEV, host, matrices_small, to_gpu
from test_oracle_generate import csr_of, parse_cases

pytestmark = pytest.mark.gpu

PARAMS = [dict(max_dist=1), dict(max_dist=2), dict(max_dist=3), dict(max_dist=8, alpha=0.5),
          dict(max_dist=40, alpha=2.0), dict(max_dist=4, thin_stop=0.5),
          dict(max_dist=6, max_moves=7), dict(max_dist=6, max_steps=11), dict(max_dist=0),
          dict(max_dist=5, thin_stop=1.5), dict(max_dist=3, alpha=0.0),
          dict(max_dist=16, alpha=1e6)]


def run_gpu(L, params, cap):
    from paper_2609_40159_amd import api
    G = to_gpu(L)
    info = api.analyze(G)
    return G, info, api.generate(G, info, params, cap, level_sums=True)


def run_oracle(orc, L, params, cap):
    a = orc.analyze(L.n, L.rowptr, L.colidx)
    return a, [orc.generate(L.n, L.rowptr, a.level, a.num_levels, a.alc, a.cv, cap=cap, **q)
               for q in params]


def check_same(out, refs, tag=""):
    rows, src, tgt = host(out.rows), host(out.src), host(out.tgt)
    lc, lr, ld = host(out.level_cost), host(out.level_rows), host(out.level_deps)
    for e, ref in enumerate(refs):
        r = out.results[e]
        m = ref.moves
        where = f"{tag} env {e}"
        assert r["moves"] == m, where
        assert np.array_equal(rows[e, :m], ref.rows), where
        assert np.array_equal(src[e, :m], ref.src), where
        assert np.array_equal(tgt[e, :m], ref.tgt), where
        for key in ("steps", "stop", "levels", "thin", "thin0", "rejected", "S1", "S2"):
            assert r[key] == getattr(ref, key), (where, key)
        assert r["threshold"] == ref.threshold, where
        assert r["cv"] == ref.cv, where
        assert np.array_equal(lc[e], ref.level_cost), where
        assert np.array_equal(lr[e], ref.level_rows), where
        assert np.array_equal(ld[e], ref.level_deps), where


@pytest.mark.parametrize("case", parse_cases(), ids=lambda c: c["name"])
def test_generate_hand_worked(case):
    rp, ci = csr_of(case["n"], case["deps"])
    L = synth.CSR(case["n"], rp, ci, np.where(np.isin(np.arange(rp[-1]), rp[1:] - 1), 2.0, -0.5))
    _, _, out = run_gpu(L, [case["params"]], case["n"])
    r = out.results[0]
    m = r["moves"]
    got = list(zip(host(out.rows)[0, :m].tolist(), host(out.src)[0, :m].tolist(),
                   host(out.tgt)[0, :m].tolist()))
    assert got == case["moves"]
    exp = case["result"]
    for key in ("steps", "stop", "levels", "thin", "thin0", "rejected", "S1", "S2"):
        assert r[key] == exp[key], key
    assert host(out.level_rows)[0].tolist() == case["level_rows"]
    assert host(out.level_cost)[0].tolist() == case["level_cost"]
    assert host(out.level_deps)[0].tolist() == case["level_deps"]


def small_matrices():
    out = dict(matrices_small())
    out["lap3d_20"] = synth.laplacian_3d(20, 20, 20)
    out["powerlaw_60k"] = synth.power_law(60000, 41)
    return out


@pytest.mark.parametrize("name", sorted(small_matrices()))
def test_generate_matches_oracle(orc, name):
    L = small_matrices()[name]
    print(f"generator parity: {name} n={L.n} envs={len(PARAMS)}", flush=True)
    _, _, out = run_gpu(L, PARAMS, L.n)
    _, refs = run_oracle(orc, L, PARAMS, L.n)
    check_same(out, refs, name)


def test_generate_capacity_limits(orc):
    L = synth.laplacian_2d(30, 30)
    for cap in (0, 1, 3, 17):
        _, _, out = run_gpu(L, PARAMS[:4], cap)
        _, refs = run_oracle(orc, L, PARAMS[:4], cap)
        check_same(out, refs, f"cap {cap}")
        assert all(r["moves"] <= cap for r in out.results)


def test_generate_full_size_lap3d_128(orc):
    L = synth.laplacian_3d(128, 128, 128)
    params = [dict(max_dist=2), dict(max_dist=8), dict(max_dist=32), dict(max_dist=8, alpha=0.5),
              dict(max_dist=8, alpha=2.0), dict(max_dist=4, thin_stop=0.9),
              dict(max_dist=8, max_steps=20000), dict(max_dist=1)]
    print("generator parity: lap3d_128", flush=True)
    _, _, out = run_gpu(L, params, 8192)
    _, refs = run_oracle(orc, L, params, 8192)
    check_same(out, refs, "lap3d_128")


def test_generate_powerlaw_1m(orc):
    """Step-limited runs against the oracle; a full-length run (140k steps)
    against invariants that hold for any length."""
    L = synth.power_law(1 << 20, 7)
    params = [dict(max_dist=2, max_steps=1500), dict(max_dist=8, max_steps=2500),
              dict(max_dist=32, alpha=0.5, max_steps=2000)]
    print("generator parity: powerlaw_1m (step-limited)", flush=True)
    _, info, out = run_gpu(L, params + [dict(max_dist=8)], 1 << 18)
    a, refs = run_oracle(orc, L, params, 1 << 18)
    check_same(out, refs, "powerlaw_1m")
    # the full run: moves are legal and the per-level sums equal a recount
    r = out.results[3]
    m = r["moves"]
    D = a.num_levels
    rows, src, tgt = host(out.rows)[3, :m], host(out.src)[3, :m], host(out.tgt)[3, :m]
    assert r["stop"] == 3 and r["steps"] == 2 * D and r["steps"] == m + r["rejected"]
    assert np.unique(rows).size == m
    assert np.array_equal(src, a.level[rows])
    assert np.all(tgt < src) and np.all(src - tgt <= 8)
    deps = np.diff(L.rowptr) - 1
    lev = a.level.copy()
    lev[rows] = tgt
    assert np.array_equal(host(out.level_rows)[3], np.bincount(lev, minlength=D))
    assert np.array_equal(host(out.level_cost)[3],
                          np.bincount(lev, weights=2 * deps + 1, minlength=D).astype(np.int64))
    assert np.array_equal(host(out.level_deps)[3],
                          np.bincount(lev, weights=deps, minlength=D).astype(np.int64))


def test_gen_rowsets_feed_rewrite_and_batch(orc):
    from paper_2609_40159_amd import api
    mats = [synth.laplacian_2d(48, 40), synth.power_law(8000, 43)]
    params = [dict(max_dist=1), dict(max_dist=2), dict(max_dist=3, alpha=0.5),
              dict(max_dist=2, max_moves=5), dict(max_dist=0)]
    for L in mats:
        G, info, out = run_gpu(L, params, 2000)
        ptr, rows, tg = api.gen_rowsets(out)
        ptr, rows, tg = host(ptr), host(rows), host(tg)
        a = orc.analyze(L.n, L.rowptr, L.colidx)
        cands = []
        for e in range(len(params)):
            m = out.results[e]["moves"]
            mr, mt = host(out.rows)[e, :m], host(out.tgt)[e, :m]
            order = np.argsort(mr, kind="stable")
            assert ptr[e + 1] - ptr[e] == m
            assert np.array_equal(rows[ptr[e]:ptr[e + 1]], mr[order])
            assert np.array_equal(tg[ptr[e]:ptr[e + 1]], mt[order])
            cands.append((rows[ptr[e]:ptr[e + 1]], tg[ptr[e]:ptr[e + 1]]))
        # one list through the single-matrix rewrite: identical pattern
        r1, t1 = cands[1]
        rw = api.rewrite(G, info.level, torch.as_tensor(r1, device=DEV),
                         torch.as_tensor(t1, device=DEV))
        ref = orc.rewrite(L.n, L.rowptr, L.colidx, L.vals, a.level, r1, t1)
        assert np.array_equal(host(rw.L.rowptr), ref.rowptr)
        assert np.array_equal(host(rw.L.colidx), ref.colidx)
        # all lists as batch candidates, straight from the device arrays
        need = 0
        refs = []
        for r, t in cands:
            rw2 = orc.rewrite(L.n, L.rowptr, L.colidx, L.vals, a.level, r, t)
            need += int(np.sum(rw2.rowptr[r + 1] - rw2.rowptr[r]))
            a2 = orc.analyze(L.n, rw2.rowptr, rw2.colidx)
            refs.append(a2)
        d_ptr = torch.as_tensor(ptr, device=DEV)
        d_rows = torch.as_tensor(rows, device=DEV)
        d_tg = torch.as_tensor(tg, device=DEV)
        bt = api.Batch([(G, None, None)], [0] * len(params), d_ptr, d_rows, d_tg,
                       cand_rows_cap=rows.size, pattern_cap=max(need, 1))
        bt.run()
        got = bt.stats()
        for c, a2 in enumerate(refs):
            assert got[c]["valid"]
            assert got[c]["num_levels"] == a2.num_levels
            assert got[c]["S1"] == a2.S1 and got[c]["S2"] == a2.S2 and got[c]["cv"] == a2.cv


def test_generate_repeated_calls_and_argument_errors(orc):
    from paper_2609_40159_amd import _lib, api
    L = synth.power_law(5000, 44)
    G, info, out1 = run_gpu(L, PARAMS, L.n)
    out2 = api.generate(G, info, PARAMS, L.n, level_sums=True)
    for e in range(len(PARAMS)):
        assert out1.results[e] == out2.results[e]
        m = out1.results[e]["moves"]
        assert torch.equal(out1.rows[e, :m], out2.rows[e, :m])
    with pytest.raises(_lib.RwtError):
        api.generate(G, info, [dict(max_dist=-1)], 10)
    with pytest.raises(_lib.RwtError):
        api.generate(G, info, [dict(alpha=float("nan"))], 10)
    with pytest.raises(_lib.RwtError):
        api.generate(G, info, [dict(max_steps=-3)], 10)
    lib = _lib.load()
    sz = C.c_size_t(0)
    assert lib.rwt_generate_ws(10, 11, 1, C.byref(sz)) == -1      # D > n: invalid
    assert lib.rwt_gen_rowsets_ws(1 << 16, 1 << 16, C.byref(sz)) == -8  # too large
    empty = api.generate(G, info, [], 10)
    assert empty.results == []
