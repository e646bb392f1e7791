"""Pins of the oracle's environment step and reward (Sections 4.1-4.5,
Algorithms 1 and 2) against things other than itself:

- a second, independent implementation in plain Python written from the
  same readings (brute force over rows and levels at every step), run on
  small matrices under random actions, step by step: node, target,
  outcome, the four reward terms, state, observation and mask;
- the fixed-policy generator of the oracle (pinned by its own hand-worked
  cases): driving the environment with that policy and a search window of
  one gives the same move list and the same final level table;
- hand-worked cases (tests/golden/env_cases.txt);
- invariants: conservation of rows and cost, CV equal to numpy's
  population CV of the non-empty levels, reward terms by branch."""
import math
import os

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- brute force
class Brute:
    """The environment of the readings, in plain Python."""

    def __init__(self, rowptr, level, D, alc, cv, cap, p):
        self.p = p
        self.n = len(rowptr) - 1
        self.D = D
        self.cap = cap
        self.dr = [int(rowptr[i + 1] - rowptr[i] - 1) for i in range(self.n)]
        self.level0 = [int(x) for x in level]
        self.thr = alc * (1.0 + p["alpha"] * max(0.0, 1.0 - cv))
        self.alc, self.arl = alc, self.n / D
        self.max_steps = p["max_steps"] or max(2 * D, 6144)
        self.reset()

    def reset(self):
        self.lev = list(self.level0)
        self.init = self.rows()
        self.first = [0] * self.D
        self.ss = [0] * self.D
        self.ts = [0] * self.D
        self.tgt_ever = [False] * self.D
        self.steps = self.moves = 0
        self.last = -1
        self.last_collapse = 0
        self.T0 = self.thin_count()
        self.D0 = sum(1 for r in self.rows() if r)
        self.moves_list = []
        self.done = self.stop()

    def rows(self):
        r = [0] * self.D
        for l in self.lev:
            r[l] += 1
        return r

    def cost(self):
        c = [0] * self.D
        for i, l in enumerate(self.lev):
            c[l] += 2 * self.dr[i] + 1
        return c

    def thin(self, l):
        return self.rows()[l] > 0 and self.cost()[l] < self.thr

    def thin_count(self):
        return sum(1 for l in range(self.D) if self.thin(l))

    def cvs(self):
        r, c = self.rows(), self.cost()
        ne = [l for l in range(self.D) if r[l]]

        def cv(v):
            m = len(v)
            s1 = sum(v)
            if m <= 1 or s1 == 0:
                return 0.0
            num = m * sum(x * x for x in v) - s1 * s1
            return math.sqrt(float(num)) / float(s1)
        return cv([c[l] for l in ne]), cv([r[l] for l in ne])

    def stop(self):
        if self.T0 > 0 and self.thin_count() / self.T0 < self.p["thin_stop"]:
            return oracle.GEN_THIN
        if self.moves >= self.cap:
            return oracle.GEN_MOVES
        if self.steps >= self.max_steps:
            return oracle.GEN_STEPS
        if not any(self.rows()[1:]):
            return oracle.GEN_NO_SOURCE
        return -1

    def step(self, a):
        p, ra = self.p, self.p["reward_alpha"]
        out = dict(outcome=0, node=-1, src=-1, tgt=-1, collapsed=0, reward=0.0, r_cv=0.0,
                   r_cp=0.0, r_rwdist=0.0, r_abandon=0.0)
        if self.done >= 0:
            out["outcome"] = oracle.ENV_IGNORED
            return out
        rows = self.rows()
        step = self.steps + 1
        if not (1 <= a < self.D and rows[a] > 0):
            self.steps = step
            out.update(outcome=oracle.ENV_INVALID, reward=-ra)
            self.done = self.stop()
            return out
        node = min((i for i in range(self.n) if self.lev[i] == a), key=lambda i: (self.dr[i], i))
        above = [l for l in range(a) if rows[l] > 0]
        pl = max(above)
        if pl == 0:
            t = 0 if self.thin(0) else -1
        else:
            window = [l for l in range(pl, -1, -1) if self.thin(l)][:p["search_window"]]
            if window:
                # highest stamp; the first (nearest) among equals
                t = max(window, key=lambda l: (self.ts[l], l))
            else:
                t = pl if self.thin(a) else -1
        if t >= 0 and a - t > p["max_dist"]:
            t = -1
        if t < 0:
            self.steps = step
            out.update(outcome=oracle.ENV_REJECTED, node=node, src=a, reward=-ra)
            self.done = self.stop()
            return out
        cv0, _ = self.cvs()
        size = rows[a]
        src_thin = self.thin(a)
        rab = 0.0
        A = self.last
        if A >= 1 and A != a:
            if self.tgt_ever[A]:
                self.init[A] = rows[A]
                self.first[A] = 0
            elif rows[A] > 0:
                ones = any(rows[l] == 1 for l in range(1, self.D))
                if not (ones and self.thin(A)):
                    c = 1.0 - rows[A] / (self.init[A] + 1.0)
                    rab = -((1.0 - c) * math.log1p(step - self.first[A]))
        self.lev[node] = t
        self.tgt_ever[t] = True
        self.ts[t] = step
        self.ss[a] = step
        if self.first[a] == 0:
            self.first[a] = step
        self.last = a
        self.moves += 1
        self.steps = step
        self.moves_list.append((node, a, t))
        rows = self.rows()
        collapsed = rows[a] == 0
        if collapsed:
            self.last_collapse = step
        cv1, _ = self.cvs()
        levels = sum(1 for r in rows if r)
        dcv = cv0 - cv1
        rcv = -ra if dcv < -p["eps"] else (self.D0 * dcv if dcv > p["eps"] else 0.0)
        s = math.log(1.0 + size + 1.0)
        if collapsed:
            rcp = ra * (self.D0 / levels) * (1.0 + 1.0 / s)
        elif src_thin:
            rcp = ra / s
        else:
            rcp = -1.0 * ra * (1.0 + s)
        d, th = a - t, p["dist_threshold"]
        rrw = math.log1p(th - d) / self.D0 if d < th else -math.log1p(d - th) / self.D0
        out.update(outcome=oracle.ENV_MOVED, node=node, src=a, tgt=t, collapsed=int(collapsed),
                   r_cv=rcv, r_cp=rcp, r_rwdist=rrw, r_abandon=rab,
                   reward=0.8 * rcv + 0.8 * rcp + 0.05 * rrw + 0.5 * rab)
        self.done = self.stop()
        return out

    def mask(self):
        rows = self.rows()
        m = [self.done < 0 and l >= 1 and rows[l] > 0 for l in range(self.D)]
        if self.done >= 0:
            return m
        if self.last >= 1 and rows[self.last] == 1:
            return [l == self.last for l in range(self.D)]
        if self.p["stall_steps"] and self.steps - self.last_collapse >= self.p["stall_steps"]:
            valid = [l for l in range(self.D) if m[l]]
            key = {l: (-1 if self.tgt_ever[l] else self.ss[l]) for l in valid}
            keep = sorted(valid, key=lambda l: (-key[l], l))[:self.p["keep_top"]]
            return [l in keep for l in range(self.D)]
        return m

    def features(self):
        rows, cost = self.rows(), self.cost()
        f = np.zeros((6, self.D))
        for l in range(self.D):
            empty = rows[l] == 0
            f[0, l] = cost[l] / self.alc
            f[1, l] = rows[l] / self.arl
            f[2, l] = -1.0 if (empty or self.tgt_ever[l]) else (
                0.0 if self.ss[l] == 0 else self.p["decay"] ** (self.steps - self.ss[l]))
            f[3, l] = -1.0 if not self.thin(l) else (
                0.0 if self.ts[l] == 0 else self.p["decay"] ** (self.steps - self.ts[l]))
            f[4, l] = 1.0 - rows[l] / (self.init[l] + 1.0)
            f[5, l] = 1.0 if self.thin(l) else 0.0
        levels = sum(1 for r in rows if r)
        thin = self.thin_count()
        cvc, cvr = self.cvs()
        g = np.array([cvc, 1.0, cvr, 1.0, levels / self.n, self.moves / self.n,
                      thin / self.T0 if self.T0 else 0.0, levels / self.D0,
                      thin / levels if levels else 0.0])
        return f, g


def small_matrices():
    rng_lower = [synth.random_lower(n, 0.12, s) for n, s in [(30, 1), (45, 2), (60, 3)]]
    return {"lap2d_9x7": synth.laplacian_2d(9, 7), "lap3d_4x4x3": synth.laplacian_3d(4, 4, 3),
            "powerlaw_300": synth.power_law(300, 4), "rand_30": rng_lower[0],
            "rand_45": rng_lower[1], "rand_60": rng_lower[2]}


def make(L, cap=None, **kw):
    a = oracle.analyze(L.n, L.rowptr, L.colidx)
    prm = dict(oracle.ENV_DEFAULTS, **kw)
    env = oracle.Env(L.n, L.rowptr, a.level, a.num_levels, a.alc, a.cv, cap=cap, **kw)
    br = Brute(L.rowptr, a.level, a.num_levels, a.alc, a.cv, L.n if cap is None else cap, prm)
    return a, env, br


PARAMS = [dict(), dict(search_window=1), dict(search_window=3, max_dist=2, alpha=0.0),
          dict(alpha=3.0, dist_threshold=0, stall_steps=4, keep_top=2, eps=0.0),
          dict(max_dist=30, search_window=8, thin_stop=0.5, decay=0.5, reward_alpha=2.5)]


@pytest.mark.parametrize("name", sorted(small_matrices()))
@pytest.mark.parametrize("pi", range(len(PARAMS)))
def test_env_matches_brute_force(name, pi):
    L = small_matrices()[name]
    a, env, br = make(L, **PARAMS[pi])
    rng = np.random.default_rng(100 + pi)
    for k in range(120):
        f, g, mask = env.observe()
        bf, bg = br.features()
        np.testing.assert_allclose(f, bf, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(g, bg, rtol=1e-13, atol=1e-15)
        assert list(mask) == br.mask(), (name, k)
        # mostly masked-in actions, sometimes anything (invalid ones too)
        valid = np.flatnonzero(mask)
        if valid.size and rng.random() < 0.8:
            act = int(rng.choice(valid))
        else:
            act = int(rng.integers(-1, a.num_levels + 1))
        r = env.step(act)
        b = br.step(act)
        for key in ("outcome", "node", "src", "tgt", "collapsed"):
            assert r[key] == b[key], (name, k, act, key, r, b)
        for key in ("reward", "r_cv", "r_cp", "r_rwdist", "r_abandon"):
            assert r[key] == pytest.approx(b[key], rel=1e-13, abs=1e-15), (name, k, key)
        assert r["done"] == br.done and r["steps"] == br.steps and r["moves"] == br.moves
        lev, cost, rows, _, _ = env.state()
        assert list(lev) == br.lev
        if r["done"] >= 0:
            break


def test_env_window_one_reproduces_generator():
    """The fixed policy of the generator (fewest-rows thin source that never
    received rows and was never rejected) driving the environment with a
    window of one gives the generator's list and level table."""
    for L in [synth.laplacian_2d(30, 20), synth.laplacian_3d(9, 8, 7), synth.power_law(4000, 5),
              synth.random_lower(500, 0.02, 9)]:
        for md, alpha in [(8, 1.0), (2, 0.0), (30, 2.0)]:
            a = oracle.analyze(L.n, L.rowptr, L.colidx)
            D = a.num_levels
            g = oracle.generate(L.n, L.rowptr, a.level, D, a.alc, a.cv, alpha=alpha, max_dist=md)
            env = oracle.Env(L.n, L.rowptr, a.level, D, a.alc, a.cv, alpha=alpha, max_dist=md,
                             search_window=1, thin_stop=0.02)
            rejected = np.zeros(D, bool)
            target = np.zeros(D, bool)
            src = -1
            moves = 0
            while True:
                f, _, _ = env.observe()
                _, cost, rows, _, _ = env.state()
                thin = f[5] > 0
                if src < 0 or rows[src] == 0:
                    cand = [l for l in range(1, D) if thin[l] and not target[l] and not rejected[l]]
                    if not cand:
                        break
                    src = min(cand, key=lambda l: (rows[l], l))
                r = env.step(src)
                if r["outcome"] == oracle.ENV_REJECTED:
                    rejected[src] = True
                    src = -1
                elif r["outcome"] == oracle.ENV_MOVED:
                    target[r["tgt"]] = True
                    moves += 1
                if r["done"] >= 0:
                    break
            _, cost, rows, deps, (mr, ms, mt) = env.state()
            assert moves == g.moves, (L.n, md, alpha)
            assert np.array_equal(mr[:moves], g.rows)
            assert np.array_equal(ms[:moves], g.src)
            assert np.array_equal(mt[:moves], g.tgt)
            assert np.array_equal(cost, g.level_cost) and np.array_equal(rows, g.level_rows)
            assert np.array_equal(deps, g.level_deps)


def test_env_invariants_under_random_actions():
    L = synth.power_law(3000, 6)
    a = oracle.analyze(L.n, L.rowptr, L.colidx)
    D = a.num_levels
    env = oracle.Env(L.n, L.rowptr, a.level, D, a.alc, a.cv, search_window=5, max_dist=40)
    rng = np.random.default_rng(3)
    _, cost0, _, _, _ = env.state()
    for k in range(400):
        _, _, mask = env.observe()
        valid = np.flatnonzero(mask)
        if not valid.size:
            break
        r = env.step(int(rng.choice(valid)))
        lev, cost, rows, deps, _ = env.state()
        assert rows.sum() == L.n and cost.sum() == cost0.sum()
        assert np.array_equal(rows, np.bincount(lev, minlength=D))
        ne = cost[rows > 0].astype(np.float64)
        assert r["cv"] == pytest.approx(ne.std() / ne.mean(), rel=1e-12)
        assert r["levels"] == int((rows > 0).sum())
        if r["outcome"] == oracle.ENV_MOVED:
            assert r["tgt"] < r["src"] and r["src"] - r["tgt"] <= 40
            # the three branches of r_cp occupy disjoint ranges: a collapse
            # earns more than 1; a thin source that did not empty had at
            # least 2 rows, so 0 < 1/s <= 1/log(4); a thick source less
            # than -(1 + log 4)
            if r["collapsed"]:
                assert r["r_cp"] > 1.0
            else:
                assert 0.0 < r["r_cp"] <= 1.0 / math.log(4.0) or r["r_cp"] < -(1.0 + math.log(4.0))
            assert r["r_abandon"] <= 0.0
        else:
            assert r["reward"] == -1.0
        if r["done"] >= 0:
            break


def test_env_argument_checks():
    L = synth.laplacian_2d(5, 4)
    a = oracle.analyze(L.n, L.rowptr, L.colidx)
    for bad in [dict(decay=1.0), dict(decay=0.0), dict(search_window=0), dict(keep_top=0),
                dict(max_dist=-1), dict(eps=-1.0)]:
        with pytest.raises(ValueError):
            oracle.Env(L.n, L.rowptr, a.level, a.num_levels, a.alc, a.cv, **bad)
    with pytest.raises(TypeError):
        oracle.Env(L.n, L.rowptr, a.level, a.num_levels, a.alc, a.cv, window=3)


def _expr(s):
    return float(eval(s, {"__builtins__": {}}, {"ln": math.log, "sqrt": math.sqrt}))


def parse_env_cases():
    cases, cur = [], None
    for raw in open(os.path.join(HERE, "golden", "env_cases.txt")):
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "case":
            kv = dict(t.split("=") for t in tok[2:])
            cur = {"name": tok[1], "n": int(kv["n"]), "cap": int(kv["cap"]), "deps": {},
                   "params": {}, "steps": []}
            cases.append(cur)
        elif tok[0] == "deps":
            for t in tok[1:]:
                r, cs = t.split(":")
                cur["deps"][int(r)] = [int(c) for c in cs.split(",")]
        elif tok[0] == "params":
            for t in tok[1:]:
                k, v = t.split("=")
                cur["params"][k] = float(v) if "." in v or "e" in v else int(v)
        elif tok[0] == "step":
            cur["steps"].append({"action": int(tok[1]),
                                 "kv": dict(t.split("=", 1) for t in tok[2:]), "state": {}})
        else:
            cur["steps"][-1]["state"][tok[0]] = tok[1:]
    return cases


def case_matrix(c):
    n = c["n"]
    rp, ci, va = [0], [], []
    for i in range(n):
        for j in c["deps"].get(i, []):
            ci.append(j)
            va.append(-1.0)
        ci.append(i)
        va.append(4.0)
        rp.append(len(ci))
    return synth.CSR(n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(va))


@pytest.mark.parametrize("case", parse_env_cases(), ids=lambda c: c["name"])
def test_env_golden(case):
    L = case_matrix(case)
    a = oracle.analyze(L.n, L.rowptr, L.colidx)
    env = oracle.Env(L.n, L.rowptr, a.level, a.num_levels, a.alc, a.cv, cap=case["cap"],
                     **case["params"])
    for k, st in enumerate(case["steps"]):
        r = env.step(st["action"])
        where = (case["name"], k + 1)
        for key in ("outcome", "node", "src", "tgt", "collapsed", "done", "thin", "levels"):
            assert r[key] == int(st["kv"][key]), (where, key, r[key])
        terms = ("r_cv", "r_cp", "r_rwdist", "r_abandon")
        if "reward" in st["kv"]:
            assert r["reward"] == pytest.approx(_expr(st["kv"]["reward"]), rel=1e-12, abs=1e-15)
            for t in terms:
                assert r[t] == 0.0, (where, t)
        else:
            want = {t: _expr(st["kv"][t]) for t in terms}
            for t in terms:
                assert r[t] == pytest.approx(want[t], rel=1e-12, abs=1e-15), (where, t)
            total = 0.80 * want["r_cv"] + 0.80 * want["r_cp"] + 0.05 * want["r_rwdist"] + \
                0.50 * want["r_abandon"]
            assert r["reward"] == pytest.approx(total, rel=1e-12, abs=1e-15), where
        f, g, mask = env.observe()
        _, _, rows, _, _ = env.state()
        s = st["state"]
        assert list(rows) == [int(x) for x in s["rows"]], where
        assert list(np.flatnonzero(mask)) == [int(x) for x in s["mask"]], where
        for key, fi in (("src_aff", 2), ("tgt_aff", 3), ("completion", 4)):
            if key in s:
                np.testing.assert_allclose(f[fi], [_expr(x) for x in s[key]], rtol=1e-15)
        if "global" in s:
            np.testing.assert_allclose(g, [_expr(x) for x in s["global"]], rtol=1e-14)
