"""Maskable PPO (Section 4.5) over the batched environment step, on the
GPU: masked sampling never picks a masked level; the environment state
reached under the policy's actions equals the oracle's environment fed the
same actions (node, target, outcome, rewards, level table); a short
training run updates the policy with finite losses; and the policy's
rewrite list, applied with the rewrite and scored by the analysis, gives
the levels the environment tracked or fewer."""
import numpy as np
import pytest
import torch

import synth
from gpu_helpers import DEV, host, to_gpu

pytestmark = pytest.mark.gpu

KEYS = ("outcome", "node", "src", "tgt", "collapsed", "done", "steps", "moves", "levels", "thin")


def test_policy_actions_respect_the_mask_and_match_the_oracle():
    import oracle
    from paper_2609_40159_amd import ppo
    from paper_2609_40159_amd.api import Env, analyze
    L = synth.power_law(4000, 61)
    G = to_gpu(L)
    info = analyze(G)
    a = oracle.analyze(L.n, L.rowptr, L.colidx)
    E = 6
    env = Env(G, info, E, cap=400, max_steps=300)
    oenv = [oracle.Env(L.n, L.rowptr, a.level, a.num_levels, a.alc, a.cv, cap=400, max_steps=300)
            for _ in range(E)]
    torch.manual_seed(3)
    pol = ppo.LevelPolicy(hidden=32).to(DEV)
    lv, gl, mk = env.observe()
    ended = np.zeros(E, bool)
    for k in range(120):
        with torch.no_grad():
            logits, _ = pol(lv, gl)
            act = torch.distributions.Categorical(logits=ppo.masked_logits(logits, mk)).sample()
        mh, ah = host(mk), host(act)
        for e in range(E):
            if not ended[e]:
                assert mh[e, ah[e]] == 1, (k, e, ah[e])      # never a masked level
        st = env.step(act.to(torch.int32), observe=True)
        res = st.results()
        for e in range(E):
            o = oenv[e].step(int(ah[e]))
            for key in KEYS:
                assert res[e][key] == o[key], (k, e, key, res[e][key], o[key])
            assert res[e]["reward"] == pytest.approx(o["reward"], rel=1e-12, abs=1e-14)
            ended[e] = res[e]["done"] >= 0
        if ended.all():
            break
    c, r, d = env.levels()
    mr, mt = host(env.mv_row), host(env.mv_tgt)
    for e in range(E):
        st_o = oenv[e].state()
        oc, orr, od = st_o[1], st_o[2], st_o[3]
        assert np.array_equal(host(c)[e], oc) and np.array_equal(host(r)[e], orr)
        assert np.array_equal(host(d)[e], od)
        m = res[e]["moves"]
        orows, _, otg = st_o[4]
        assert np.array_equal(mr[e, :m], orows[:m]) and np.array_equal(mt[e, :m], otg[:m])


def test_short_training_and_scored_rewrite_list():
    from paper_2609_40159_amd import ppo
    from paper_2609_40159_amd.api import Env, Rewriter, analyze
    L = synth.power_law(6000, 62)
    G = to_gpu(L)
    info = analyze(G)
    env = Env(G, info, 4, max_steps=256)
    pol = ppo.LevelPolicy(hidden=32).to(DEV)
    before = [p.detach().clone() for p in pol.parameters()]
    cfg = ppo.PPOConfig(n_steps=128, updates=2, epochs=2, batch_size=64, seed=5)
    out = ppo.train(env, pol, cfg)
    assert out["updates"] == 2 and out["env_steps"] == 2 * 128 * 4
    for rec in cfg.stats:
        for key in ("policy_loss", "value_loss", "approx_kl"):
            assert np.isfinite(rec[key]), (key, rec)
    assert any(not torch.equal(p0, p1) for p0, p1 in zip(before, pol.parameters()))
    lists = ppo.rollout_lists(env, pol, greedy=False, seed=1)
    D0 = info.num_levels
    for e, li in enumerate(lists):
        if li["rows"].size == 0:
            continue
        rw = Rewriter(G, info.level, li["rows"], li["targets"])
        rw.numeric()
        a2 = analyze(rw.Lp)
        # recomputed levels of L' are at most the levels the environment
        # tracked (rewriting moves every rewritten row to its target or lower)
        assert a2.num_levels <= li["env_levels"] <= D0, (e, a2.num_levels, li["env_levels"], D0)
