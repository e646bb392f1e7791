"""Host-side checks of the Maskable PPO pieces (no GPU): generalized
advantage estimation against its definition summed out by hand, masked
sampling never picking a masked level, the clipped surrogate on a worked
example, and the final rewrite list of a move list."""
import numpy as np
import torch

from paper_2609_40159_amd import ppo


def test_gae_matches_the_discounted_sum_of_td_errors():
    rng = np.random.default_rng(0)
    T, E, g, lam = 7, 3, 0.9, 0.8
    r = rng.standard_normal((T, E))
    v = rng.standard_normal((T, E))
    d = (rng.random((T, E)) < 0.3).astype(float)
    lastv = rng.standard_normal(E)
    adv, ret = ppo.gae(torch.tensor(r), torch.tensor(v), torch.tensor(d), torch.tensor(lastv), g, lam)
    for e in range(E):
        for t in range(T):
            # A_t = sum_k (g lam)^k delta_{t+k}, stopping after an episode end
            a, w = 0.0, 1.0
            for k in range(t, T):
                nv = lastv[e] if k == T - 1 else v[k + 1, e]
                delta = r[k, e] + g * nv * (1 - d[k, e]) - v[k, e]
                a += w * delta
                if d[k, e]:
                    break
                w *= g * lam
            assert abs(adv[t, e].item() - a) < 1e-12
            assert abs(ret[t, e].item() - (a + v[t, e])) < 1e-12


def test_masked_levels_are_never_sampled():
    torch.manual_seed(1)
    E, D = 64, 37
    logits = torch.randn(E, D) * 5
    mask = (torch.rand(E, D) < 0.2).to(torch.uint8)
    mask[3] = 0                      # an ended episode: no valid level
    ml = ppo.masked_logits(logits, mask)
    dist = torch.distributions.Categorical(logits=ml)
    for _ in range(200):
        a = dist.sample()
        ok = mask[torch.arange(E), a].bool()
        ok[3] = True
        assert bool(ok.all())
    p = dist.probs
    assert float(p[mask == 0][~(torch.arange(E)[:, None].expand(E, D)[mask == 0] == 3)].max()) == 0.0
    assert int(dist.sample()[3]) == 0


def test_clipped_surrogate_worked_example():
    # ratio 1.5 with a positive advantage is clipped to 1.2; ratio 0.5 with a
    # negative advantage to 0.8 (the pessimistic bound of each pair)
    new = torch.log(torch.tensor([1.5, 0.5, 1.1]))
    old = torch.zeros(3)
    adv = torch.tensor([2.0, -1.0, 3.0])
    v = torch.tensor([1.0, 0.0, 2.0])
    ret = torch.tensor([2.0, 1.0, 2.0])
    loss, d = ppo.ppo_loss(new, old, adv, v, ret, torch.zeros(3), 0.2, 0.5, 0.0)
    want_pg = -(1.2 * 2.0 + 0.8 * -1.0 + 1.1 * 3.0) / 3
    assert abs(d["policy_loss"] - want_pg) < 1e-6
    assert abs(d["value_loss"] - (1.0 + 1.0 + 0.0) / 3) < 1e-6
    assert abs(float(loss) - (want_pg + 0.5 * 2.0 / 3)) < 1e-6
    assert abs(d["clip_fraction"] - 2.0 / 3) < 1e-6


def test_final_rewrite_list_keeps_each_rows_last_target():
    rows, tg = ppo.final_rewrite_list(np.array([9, 4, 9, 7]), np.array([5, 2, 3, 6]))
    assert rows.tolist() == [4, 7, 9] and tg.tolist() == [2, 6, 3]


def test_policy_shapes_and_independence_of_level_count():
    pol = ppo.LevelPolicy(hidden=16)
    for D in (5, 300):
        lg, v = pol(torch.randn(4, 6, D), torch.randn(4, 9))
        assert lg.shape == (4, D) and v.shape == (4,)
