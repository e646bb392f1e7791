"""GPU parity of the environment step (Sections 4.1-4.5, Algorithms 1 and
2) against the oracle's environment, step by step: every environment of a
batch is mirrored by an oracle environment fed the same actions; node,
target, outcome, episode end and level table bit-exact, the CV bit-exact
(exact integer sums on both sides), the reward terms within 1e-12
(logarithms of two libraries), the float32 observation within float32
rounding of the oracle's FP64 values, and the mask bit-exact.  Actions are
drawn from the GPU mask (checked first) with some invalid ones mixed in;
some environments are reset part-way."""
import numpy as np
import pytest
import torch

import synth
from gpu_helpers import DEV, host, matrices_small, to_gpu

pytestmark = pytest.mark.gpu

KEYS_EXACT = ("outcome", "node", "src", "tgt", "collapsed", "done", "steps", "moves", "levels",
              "thin", "thin0")
TERMS = ("reward", "r_cv", "r_cp", "r_rwdist", "r_abandon")


def compare_step(g: dict, o: dict, where):
    for k in KEYS_EXACT:
        assert g[k] == o[k], (where, k, g[k], o[k])
    for k in TERMS:
        assert g[k] == pytest.approx(o[k], rel=1e-12, abs=1e-14), (where, k, g[k], o[k])
    assert g["cv"] == o["cv"] and g["cv_rows"] == o["cv_rows"], where


def compare_obs(env, oenvs, sample, where):
    lv, gl, mk = env.observe()
    idx = torch.as_tensor(sample, device=DEV)
    lv, gl, mkh = host(lv[idx]), host(gl[idx]), host(mk)
    for q, e in enumerate(sample):
        f, g, m = oenvs[e].observe()
        np.testing.assert_allclose(lv[q], f, rtol=2e-7, atol=1e-30, err_msg=str((where, e)))
        np.testing.assert_allclose(gl[q], g, rtol=2e-7, atol=1e-30, err_msg=str((where, e)))
        assert np.array_equal(mkh[e].astype(bool), m), (where, e)
    return mkh


def run(L, E, steps, params, seed, sample=None, cap=None, reset_every=0):
    import oracle
    from paper_2609_40159_amd.api import Env, analyze
    G = to_gpu(L)
    info = analyze(G)
    a = oracle.analyze(L.n, L.rowptr, L.colidx)
    assert a.num_levels == info.num_levels
    env = Env(G, info, E, cap=cap, **params)
    sample = list(range(E)) if sample is None else sample
    oenvs = {e: oracle.Env(L.n, L.rowptr, a.level, a.num_levels, a.alc, a.cv, cap=env.cap,
                           **params) for e in sample}
    rng = np.random.default_rng(seed)
    D = a.num_levels
    for k in range(steps):
        mk = compare_obs(env, oenvs, sample, (k, "obs"))
        acts = np.empty(E, np.int32)
        for e in range(E):
            valid = np.flatnonzero(mk[e])
            if valid.size and rng.random() < 0.85:
                acts[e] = rng.choice(valid)
            else:
                acts[e] = rng.integers(-2, D + 2)
        st = env.step(torch.as_tensor(acts))
        res = st.results()
        for e in sample:
            compare_step(res[e], oenvs[e].step(int(acts[e])), (k, e, int(acts[e])))
        if reset_every and k % reset_every == reset_every - 1:
            which = np.zeros(E, np.uint8)
            which[rng.choice(E, size=max(1, E // 3), replace=False)] = 1
            env.reset(torch.as_tensor(which))
            for e in sample:
                if which[e]:
                    oenvs[e].reset()
        if all(r["done"] >= 0 for r in res):
            break
    # the level table and the move lists
    cost, rows, deps = (host(t) for t in env.levels())
    mvr, mvs, mvt = host(env.mv_row), host(env.mv_src), host(env.mv_tgt)
    for e in sample:
        _, oc, orr, od, (omr, oms, omt) = oenvs[e].state()
        assert np.array_equal(cost[e], oc) and np.array_equal(rows[e], orr)
        assert np.array_equal(deps[e], od)
        if not reset_every:
            m = res[e]["moves"]
            assert np.array_equal(mvr[e, :m], omr[:m]) and np.array_equal(mvs[e, :m], oms[:m])
            assert np.array_equal(mvt[e, :m], omt[:m])
    return res


PARAMS = [dict(), dict(search_window=1, max_dist=3),
          dict(alpha=0.0, stall_steps=3, keep_top=2, dist_threshold=0, decay=0.7),
          dict(max_dist=40, search_window=8, thin_stop=0.3, reward_alpha=2.0, max_steps=90)]


@pytest.mark.parametrize("name", sorted(matrices_small()))
@pytest.mark.parametrize("pi", range(len(PARAMS)))
def test_env_matches_oracle(name, pi):
    L = matrices_small()[name]
    print(f"env parity: {name} params {pi}", flush=True)
    run(L, 6, 150, PARAMS[pi], seed=10 * pi + 1)


def test_env_partial_resets_and_small_cap():
    L = synth.power_law(20000, 21)
    print("env parity: partial resets, cap 40", flush=True)
    run(L, 12, 200, dict(max_dist=20), seed=5, cap=40, reset_every=25)


def test_env_full_size_sampled():
    """The 128^3 factor with 256 environments stepped 120 times; four of them
    checked against the oracle at every step."""
    L = synth.laplacian_3d(128, 128, 128)
    print("env parity: lap3d_128, 256 environments, sampled", flush=True)
    run(L, 256, 120, dict(), seed=9, sample=[0, 77, 154, 255])


def test_env_deep_powerlaw_sampled():
    """Power-law 1M (about 67k levels, mostly thin): long searches for the
    nearest non-empty level and the window; 32 environments stepped 60
    times, two checked against the oracle at every step."""
    L = synth.power_law(1 << 20, 7)
    print("env parity: powerlaw_1m, 32 environments, sampled", flush=True)
    run(L, 32, 60, dict(max_dist=64, search_window=5, stall_steps=4, keep_top=6), seed=4,
        sample=[0, 31])


def test_env_workspace_mismatch_is_refused():
    from paper_2609_40159_amd import _lib
    from paper_2609_40159_amd.api import Env, analyze
    L = synth.laplacian_2d(20, 20)
    G = to_gpu(L)
    env = Env(G, analyze(G), 4)
    lib = _lib.load()
    import ctypes as C
    res = torch.zeros(4 * C.sizeof(_lib.EnvResult), dtype=torch.uint8, device=DEV)
    acts = torch.ones(4, dtype=torch.int32, device=DEV)
    mv = torch.zeros(4 * env.cap, dtype=torch.int32, device=DEV)
    # the same workspace described with another level count: the kernel
    # refuses it
    st = lib.rwt_env_step(env.n, env.D - 1, 4, env.cap, C.c_void_p(acts.data_ptr()),
                          C.c_void_p(res.data_ptr()), C.c_void_p(mv.data_ptr()),
                          C.c_void_p(mv.data_ptr()), C.c_void_p(mv.data_ptr()),
                          C.c_void_p(env.ws.data_ptr()), env.ws.numel(),
                          C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0
    torch.cuda.synchronize()
    out = [_lib.EnvResult.from_buffer_copy(res.cpu().numpy().tobytes(), e * C.sizeof(_lib.EnvResult))
           for e in range(4)]
    assert all(r.outcome == 4 for r in out)


def test_env_graph_replay_matches_eager():
    """One rollout step (observe, a deterministic masked policy, step)
    captured in a graph and replayed, with eager work and synchronizations
    between replays, equals the same steps run eagerly on a twin."""
    from paper_2609_40159_amd.api import Env, analyze
    L = synth.power_law(30000, 23)
    G = to_gpu(L)
    info = analyze(G)
    E = 64
    A = Env(G, info, E, cap=400, max_dist=30, stall_steps=5, keep_top=3)
    B = Env(G, info, E, cap=400, max_dist=30, stall_steps=5, keep_top=3)
    w = torch.rand((E, info.num_levels), generator=torch.Generator().manual_seed(3)).to(DEV)

    def one(env):
        _, _, mask = env.observe()
        act = (w * mask).argmax(dim=1).to(torch.int32)
        return env.step(act)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        one(B)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        outB = one(B)
    A.reset()
    B.reset()
    torch.cuda.synchronize()
    print("env graph replay: 150 replays", flush=True)
    for k in range(150):
        outA = one(A)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(outA.raw, outB.raw), k
        if k % 10 == 0:
            ca, ra, da = A.levels()
            cb, rb, db = B.levels()
            assert torch.equal(ca, cb) and torch.equal(ra, rb) and torch.equal(da, db), k
            assert torch.equal(A.obs_level, B.obs_level) and torch.equal(A.mask, B.mask), k
            torch.cuda.synchronize()
    assert torch.equal(A.mv_row, B.mv_row) and torch.equal(A.mv_tgt, B.mv_tgt)
    assert int(outA.raw.view(torch.int32).view(E, -1)[:, 7].sum()) > 0   # moves were made


def test_env_capacity_one_and_single_environment():
    """A move capacity of one ends every episode after its first move (the
    MOVES end); a single environment; both against the oracle."""
    L = synth.laplacian_2d(30, 20)
    print("env parity: cap 1, 8 environments", flush=True)
    res = run(L, 8, 12, dict(), seed=21, cap=1)
    assert all(r["done"] in (-1, 2) for r in res)
    assert any(r["done"] == 2 for r in res)
    print("env parity: one environment", flush=True)
    run(synth.power_law(3000, 5), 1, 80, dict(search_window=3), seed=22)


def test_env_step_observe_equals_separate_calls():
    """The fused step-and-observe launch gives bit for bit the results, moves,
    level table, observation and mask of a step followed by an observe."""
    from paper_2609_40159_amd.api import Env, analyze
    L = synth.power_law(20000, 27)
    G = to_gpu(L)
    info = analyze(G)
    E = 48
    kw = dict(max_dist=25, stall_steps=3, keep_top=4, search_window=4)
    A = Env(G, info, E, cap=300, **kw)
    B = Env(G, info, E, cap=300, **kw)
    w = torch.rand((E, info.num_levels), generator=torch.Generator().manual_seed(5)).to(DEV)
    _, _, mask = A.observe()
    B.observe()
    print("env fused step+observe: 120 steps", flush=True)
    for k in range(120):
        act = (w * A.mask).argmax(dim=1).to(torch.int32)
        if k % 7 == 3:
            act[::5] = -1                      # some invalid actions
        ra = A.step(act)
        A.observe()
        rb = B.step(act, observe=True)
        torch.cuda.synchronize()
        assert torch.equal(ra.raw, rb.raw), k
        assert torch.equal(A.obs_level, B.obs_level) and torch.equal(A.obs_global, B.obs_global), k
        assert torch.equal(A.mask, B.mask), k
    ca, rwa, da = A.levels()
    cb, rwb, db = B.levels()
    assert torch.equal(ca, cb) and torch.equal(rwa, rwb) and torch.equal(da, db)
    assert torch.equal(A.mv_row, B.mv_row) and torch.equal(A.mv_tgt, B.mv_tgt)
