"""Maskable PPO over the batched environment step (paper Section 4.5).

The policy picks a source level per environment from the observation of
Table 1 (six features per level, nine global ones); invalid levels are
removed from the categorical distribution by the action mask of Section
4.3 before sampling (Maskable PPO).  Rewards come from Algorithm 2 inside
the environment step; the clipped surrogate objective, generalized
advantage estimation and the value loss are the usual PPO ones.  Every
environment step, observation and mask runs in librwtrsv (rwt_env_*); this
module holds the network and the optimizer (plain PyTorch).

Differences from the paper's setup (Stable-Baselines3 MlpPolicy) and why:
the policy network is one small MLP applied to every level (its six
features and the nine globals) giving that level's logit, and the value
network an MLP over the globals and the levels' mean and maximum features,
so that the same weights run on a matrix of any level count (a flat MLP
over 6 D + 9 inputs ties the weights to D).  Hyperparameters default to
the paper's (learning rate 1e-4, 1024-step rollouts per environment, four
environments) and Stable-Baselines3's PPO defaults otherwise (10 epochs,
minibatch 64, gamma 0.99, GAE lambda 0.95, clip 0.2, value coefficient
0.5, gradient norm 0.5, no entropy bonus).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch
from torch import nn

__all__ = ["LevelPolicy", "PPOConfig", "masked_logits", "gae", "ppo_loss", "train", "rollout_lists",
           "final_rewrite_list"]

NEG = -1.0e30   # logit of a masked level (exp underflows to exactly 0)


class LevelPolicy(nn.Module):
    """Actor: one MLP per level (shared weights) over [6 level features, 9
    globals] -> logit.  Critic: MLP over [mean and max of the level
    features, 9 globals] -> value."""

    def __init__(self, hidden: int = 64):
        super().__init__()
        self.actor = nn.Sequential(nn.Linear(15, hidden), nn.Tanh(), nn.Linear(hidden, hidden),
                                   nn.Tanh(), nn.Linear(hidden, 1))
        self.critic = nn.Sequential(nn.Linear(21, hidden), nn.Tanh(), nn.Linear(hidden, hidden),
                                    nn.Tanh(), nn.Linear(hidden, 1))
        # small last layers: a near-uniform initial policy over the mask
        nn.init.orthogonal_(self.actor[-1].weight, gain=0.01)
        nn.init.zeros_(self.actor[-1].bias)
        nn.init.orthogonal_(self.critic[-1].weight, gain=1.0)
        nn.init.zeros_(self.critic[-1].bias)

    def forward(self, obs_level: torch.Tensor, obs_global: torch.Tensor):
        """obs_level (E, 6, D), obs_global (E, 9) -> logits (E, D), value (E,)."""
        x = obs_level.transpose(1, 2)                         # (E, D, 6)
        g = obs_global.unsqueeze(1).expand(-1, x.shape[1], -1)
        logits = self.actor(torch.cat([x, g], dim=-1)).squeeze(-1)
        pooled = torch.cat([x.mean(dim=1), x.amax(dim=1), obs_global], dim=-1)
        value = self.critic(pooled).squeeze(-1)
        return logits, value


def masked_logits(logits: torch.Tensor, mask: torch.Tensor) -> torch.Tensor:
    """Masked levels get a logit of -1e30 (probability exactly 0).  A row
    with no valid level (its episode ended; the environment ignores the
    action) keeps level 0 so that the distribution stays defined."""
    m = mask.bool()
    empty = ~m.any(dim=1)
    if bool(empty.any()):
        m = m.clone()
        m[empty, 0] = True
    return torch.where(m, logits, torch.full_like(logits, NEG))


def gae(rewards: torch.Tensor, values: torch.Tensor, dones: torch.Tensor, last_value: torch.Tensor,
        gamma: float, lam: float):
    """Generalized advantage estimation over a (T, E) rollout: dones[t] marks
    that the episode ended with step t (no bootstrap past it).  Returns
    (advantages, returns)."""
    T = rewards.shape[0]
    adv = torch.zeros_like(rewards)
    last = torch.zeros_like(last_value)
    for t in range(T - 1, -1, -1):
        nxt = last_value if t == T - 1 else values[t + 1]
        keep = 1.0 - dones[t]
        delta = rewards[t] + gamma * nxt * keep - values[t]
        last = delta + gamma * lam * keep * last
        adv[t] = last
    return adv, adv + values


def ppo_loss(new_logp, old_logp, adv, values, returns, entropy, clip: float, vf_coef: float,
             ent_coef: float):
    """Clipped surrogate (to minimize), value loss, and the diagnostics."""
    ratio = torch.exp(new_logp - old_logp)
    s1 = ratio * adv
    s2 = torch.clamp(ratio, 1.0 - clip, 1.0 + clip) * adv
    pg = -torch.min(s1, s2).mean()
    vf = ((returns - values) ** 2).mean()
    ent = entropy.mean()
    loss = pg + vf_coef * vf - ent_coef * ent
    with torch.no_grad():
        approx_kl = ((ratio - 1.0) - (new_logp - old_logp)).mean()
        clip_frac = ((ratio - 1.0).abs() > clip).float().mean()
    return loss, {"policy_loss": float(pg), "value_loss": float(vf), "entropy": float(ent),
                  "approx_kl": float(approx_kl), "clip_fraction": float(clip_frac)}


@dataclass
class PPOConfig:
    lr: float = 1e-4
    n_steps: int = 1024          # rollout steps per environment per update
    epochs: int = 10
    batch_size: int = 64
    gamma: float = 0.99
    gae_lambda: float = 0.95
    clip: float = 0.2
    vf_coef: float = 0.5
    ent_coef: float = 0.0
    max_grad_norm: float = 0.5
    updates: int = 30            # PPO rollout iterations (the paper: 30)
    seed: int = 0
    time_limit_s: float = 0.0    # stop after this many seconds (0: no limit)
    stats: list = field(default_factory=list)


def _step_done(st) -> torch.Tensor:
    return st.done >= 0


def train(env, policy: LevelPolicy, cfg: PPOConfig, log=None) -> dict:
    """Train policy on env (an api.Env of E environments) with masked PPO.
    Environments whose episode ended are reset before the next step."""
    dev = env.device
    torch.manual_seed(cfg.seed)
    opt = torch.optim.Adam(policy.parameters(), lr=cfg.lr, eps=1e-5)
    E, D, T = env.E, env.D, cfg.n_steps
    env.reset()
    lv, gl, mk = env.observe()
    buf_lv = torch.empty((T, E, 6, D), dtype=torch.float32, device=dev)
    buf_gl = torch.empty((T, E, 9), dtype=torch.float32, device=dev)
    buf_mk = torch.empty((T, E, D), dtype=torch.uint8, device=dev)
    buf_a = torch.empty((T, E), dtype=torch.int64, device=dev)
    buf_lp = torch.empty((T, E), dtype=torch.float32, device=dev)
    buf_v = torch.empty((T, E), dtype=torch.float32, device=dev)
    buf_r = torch.empty((T, E), dtype=torch.float32, device=dev)
    buf_d = torch.empty((T, E), dtype=torch.float32, device=dev)
    ep_ret = torch.zeros(E, dtype=torch.float64, device=dev)
    finished = []
    t_start = time.perf_counter()
    env_steps = 0
    for upd in range(cfg.updates):
        policy.eval()
        with torch.no_grad():
            for t in range(T):
                logits, value = policy(lv, gl)
                dist = torch.distributions.Categorical(logits=masked_logits(logits, mk))
                a = dist.sample()
                buf_lv[t].copy_(lv)
                buf_gl[t].copy_(gl)
                buf_mk[t].copy_(mk)
                buf_a[t] = a
                buf_lp[t] = dist.log_prob(a)
                buf_v[t] = value
                st = env.step(a.to(torch.int32), observe=True)
                r = st.reward
                done = _step_done(st)
                buf_r[t] = r.float()
                buf_d[t] = done.float()
                ep_ret += r
                if bool(done.any()):
                    finished.extend(ep_ret[done].tolist())
                    ep_ret[done] = 0.0
                    env.reset(done)
                    env.observe()
                env_steps += E
            _, last_v = policy(lv, gl)
        adv, ret = gae(buf_r, buf_v, buf_d, last_v, cfg.gamma, cfg.gae_lambda)
        N = T * E
        f_lv, f_gl = buf_lv.reshape(N, 6, D), buf_gl.reshape(N, 9)
        f_mk, f_a = buf_mk.reshape(N, D), buf_a.reshape(N)
        f_lp, f_adv, f_ret = buf_lp.reshape(N), adv.reshape(N), ret.reshape(N)
        f_v = buf_v.reshape(N)
        policy.train()
        g = torch.Generator(device="cpu").manual_seed(cfg.seed + upd)
        last = {}
        for _ in range(cfg.epochs):
            perm = torch.randperm(N, generator=g).to(dev)
            for s in range(0, N, cfg.batch_size):
                idx = perm[s:s + cfg.batch_size]
                logits, value = policy(f_lv[idx], f_gl[idx])
                dist = torch.distributions.Categorical(logits=masked_logits(logits, f_mk[idx]))
                nlp = dist.log_prob(f_a[idx])
                a_n = f_adv[idx]
                a_n = (a_n - a_n.mean()) / (a_n.std() + 1e-8) if a_n.numel() > 1 else a_n
                loss, last = ppo_loss(nlp, f_lp[idx], a_n, value, f_ret[idx], dist.entropy(),
                                      cfg.clip, cfg.vf_coef, cfg.ent_coef)
                opt.zero_grad(set_to_none=True)
                loss.backward()
                nn.utils.clip_grad_norm_(policy.parameters(), cfg.max_grad_norm)
                opt.step()
        var = float(f_ret.var())
        expl = float(1.0 - (f_ret - f_v).var() / var) if var > 0 else 0.0
        rec = dict(last, update=upd, explained_variance=expl, env_steps=env_steps,
                   mean_reward=float(buf_r.mean()),
                   mean_episode_return=(float(np.mean(finished[-16:])) if finished else None),
                   episodes=len(finished), elapsed_s=time.perf_counter() - t_start)
        cfg.stats.append(rec)
        if log:
            log(rec)
        if cfg.time_limit_s and time.perf_counter() - t_start > cfg.time_limit_s:
            break
    return {"updates": len(cfg.stats), "env_steps": env_steps, "episodes": len(finished),
            "elapsed_s": time.perf_counter() - t_start, "last": cfg.stats[-1] if cfg.stats else None}


def final_rewrite_list(rows: np.ndarray, tgts: np.ndarray):
    """(rows ascending, targets) of a move list: a row moved more than once
    (Section 4.2) ends on its last move's target level."""
    last = {}
    for r, t in zip(rows.tolist(), tgts.tolist()):
        last[int(r)] = int(t)
    rr = np.array(sorted(last), dtype=np.int32)
    return rr, np.array([last[r] for r in rr.tolist()], dtype=np.int32)


def rollout_lists(env, policy: LevelPolicy, greedy: bool = False, max_steps: int | None = None,
                  seed: int = 0):
    """Run every environment from its reset to the end of its episode under
    the policy; returns per environment (rows, targets) of its final
    rewrite list and the episode's step count."""
    torch.manual_seed(seed)
    env.reset()
    lv, gl, mk = env.observe()
    E = env.E
    steps = torch.zeros(E, dtype=torch.int64, device=env.device)
    ended = torch.zeros(E, dtype=torch.bool, device=env.device)
    limit = max_steps if max_steps is not None else 10 * env.cap + 10
    policy.eval()
    with torch.no_grad():
        for _ in range(limit):
            logits, _ = policy(lv, gl)
            ml = masked_logits(logits, mk)
            a = ml.argmax(dim=1) if greedy else torch.distributions.Categorical(logits=ml).sample()
            st = env.step(a.to(torch.int32), observe=True)
            steps += (~ended).long()
            ended |= _step_done(st)
            if bool(ended.all()):
                break
    res = st.results()
    out = []
    mr, mt = env.mv_row.cpu().numpy(), env.mv_tgt.cpu().numpy()
    for e in range(E):
        m = res[e]["moves"]
        rows, tg = final_rewrite_list(mr[e, :m], mt[e, :m])
        out.append({"rows": rows, "targets": tg, "moves": m, "steps": int(steps[e]),
                    "env_levels": res[e]["levels"], "env_cv": res[e]["cv"]})
    return out
