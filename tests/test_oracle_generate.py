"""Pins for the oracle's rewrite-list generator (Section 4.1 thin levels and
state, Section 4.3 node choice, Algorithm 1 target selection).  CPU only.

The hand-worked cases in golden/generator_cases.txt fix every branch of the
target selection, the node order and each stop rule; the invariants below
check the incremental bookkeeping against a recount from scratch, the
constraints every move must satisfy, and what the rewritten matrix must
look like when the list is applied (levels of L' never above the targets).
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "generator_cases.txt")


def parse_cases():
    cases, cur = [], None
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, _, rest = line.partition(" ")
        if key == "case":
            name, nfield = rest.split()
            cur = {"name": name, "n": int(nfield.split("=")[1]), "deps": {}, "moves": []}
            cases.append(cur)
        elif key == "deps":
            for tok in rest.split():
                r, cols = tok.split(":")
                cur["deps"][int(r)] = [int(c) for c in cols.split(",")]
        elif key in ("params", "result"):
            cur[key] = {k: float(v) if "." in v else int(v)
                        for k, v in (t.split("=") for t in rest.split())}
        elif key == "moves":
            cur["moves"] = [tuple(int(x) for x in t.split("/")) for t in rest.split()]
        elif key.startswith("level_"):
            cur[key] = [int(x) for x in rest.split()]
    return cases


def csr_of(n, deps):
    rp, ci = [0], []
    for i in range(n):
        ci += sorted(deps.get(i, [])) + [i]
        rp.append(len(ci))
    return np.array(rp, np.int32), np.array(ci, np.int32)


def run(n, rowptr, colidx, **kw):
    a = oracle.analyze(n, rowptr, colidx)
    return a, oracle.generate(n, rowptr, a.level, a.num_levels, a.alc, a.cv, **kw)


@pytest.mark.parametrize("case", parse_cases(), ids=lambda c: c["name"])
def test_generator_hand_worked(case):
    n = case["n"]
    rp, ci = csr_of(n, case["deps"])
    prm = case["params"]
    a, g = run(n, rp, ci, alpha=prm["alpha"], thin_stop=prm["thin_stop"],
               max_dist=prm["max_dist"], max_moves=prm["max_moves"],
               max_steps=prm["max_steps"])
    assert list(zip(g.rows.tolist(), g.src.tolist(), g.tgt.tolist())) == case["moves"]
    r = case["result"]
    assert (g.steps, g.stop, g.levels, g.thin, g.thin0, g.rejected, g.S1, g.S2) == \
        (r["steps"], r["stop"], r["levels"], r["thin"], r["thin0"], r["rejected"], r["S1"], r["S2"])
    assert g.level_rows.tolist() == case["level_rows"]
    assert g.level_cost.tolist() == case["level_cost"]
    assert g.level_deps.tolist() == case["level_deps"]
    # CV of the non-empty levels: population standard deviation over mean
    assert g.cv == pytest.approx(math.sqrt(g.levels * g.S2 - g.S1 ** 2) / g.S1, rel=1e-15)


MATRICES = {
    "chain40": None,
    "rand60": lambda: synth.random_lower(60, 0.08, 2),
    "grid2d": lambda: synth.laplacian_2d(12, 9),
    "grid3d": lambda: synth.laplacian_3d(6, 5, 4),
    "powerlaw": lambda: synth.power_law(3000, 5),
}
PARAMS = [dict(max_dist=1), dict(max_dist=3), dict(max_dist=8, alpha=0.5),
          dict(max_dist=40, alpha=2.0), dict(max_dist=4, thin_stop=0.5),
          dict(max_dist=6, max_moves=7), dict(max_dist=6, max_steps=11)]


def chain(n):
    rp = np.concatenate([[0], 1 + 2 * np.arange(n)]).astype(np.int32)
    ci = np.concatenate([[0], np.repeat(np.arange(1, n), 2) - np.tile([1, 0], n - 1)])
    return rp, ci.astype(np.int32)


def matrix(name):
    if name == "chain40":
        rp, ci = chain(40)
        return 40, rp, ci
    L = MATRICES[name]()
    return L.n, L.rowptr, L.colidx


@pytest.mark.parametrize("name", list(MATRICES))
@pytest.mark.parametrize("pi", range(len(PARAMS)))
def test_generator_invariants(name, pi):
    n, rp, ci = matrix(name)
    prm = PARAMS[pi]
    a, g = run(n, rp, ci, **prm)
    deps = np.diff(rp) - 1
    lev0 = a.level
    D = a.num_levels
    # every move: original level as source, a target above within max_dist,
    # each row at most once
    assert len(set(g.rows.tolist())) == g.moves
    assert np.array_equal(g.src, lev0[g.rows])
    assert np.all(g.tgt < g.src) and np.all(g.src - g.tgt <= prm["max_dist"])
    # a level that received a row is never a source afterwards
    targets_so_far = set()
    for s, t in zip(g.src.tolist(), g.tgt.tolist()):
        assert s not in targets_so_far
        targets_so_far.add(t)
    # rows leave each source in (dependencies, row) order
    for lv in set(g.src.tolist()):
        members = np.nonzero(lev0 == lv)[0]
        order = members[np.lexsort((members, deps[members]))]
        moved = g.rows[g.src == lv]
        assert np.array_equal(moved, order[:moved.size])
    # the incremental per-level sums equal a recount from the final levels
    lev = lev0.copy()
    lev[g.rows] = g.tgt
    assert np.array_equal(g.level_rows, np.bincount(lev, minlength=D))
    assert np.array_equal(g.level_cost, np.bincount(lev, weights=2 * deps + 1, minlength=D).astype(np.int64))
    assert np.array_equal(g.level_deps, np.bincount(lev, weights=deps, minlength=D).astype(np.int64))
    nonempty = g.level_cost[g.level_rows > 0]
    assert g.levels == nonempty.size
    assert g.S1 == int(rp[-1]) * 2 - n == int(nonempty.sum())
    assert g.S2 == sum(int(c) * int(c) for c in nonempty)
    thr = a.alc * (1.0 + prm.get("alpha", 1.0) * max(0.0, 1.0 - a.cv))
    assert g.threshold == thr
    thin = int(np.sum((g.level_rows > 0) & (g.level_cost < thr)))
    assert g.thin == thin and g.thin0 == int(np.sum(a.cost < thr))
    assert g.steps == g.moves + g.rejected
    # the stop rule that ended the run holds
    if g.stop == oracle.GEN_THIN:
        assert g.thin / g.thin0 < prm.get("thin_stop", 0.02)
    elif g.stop == oracle.GEN_MOVES:
        assert g.moves == prm["max_moves"]
    elif g.stop == oracle.GEN_STEPS:
        assert g.steps == prm["max_steps"]
    else:
        # no source: every thin level >= 1 received rows or was rejected
        cand = [l for l in range(1, D) if g.level_rows[l] > 0 and g.level_cost[l] < thr]
        assert len([l for l in cand if l not in targets_so_far]) <= g.rejected
    # applied by the rewrite, every moved row lands at or above its target
    # and no row moves down
    if g.moves:
        order = np.argsort(g.rows)
        vals = np.where(np.arange(rp[-1]) == np.repeat(rp[1:] - 1, np.diff(rp)), 2.0, -0.1)
        rw = oracle.rewrite(n, rp, ci, vals, lev0, g.rows[order], g.tgt[order])
        a2 = oracle.analyze(n, rw.rowptr, rw.colidx)
        assert np.all(a2.level[g.rows] <= g.tgt)
        assert np.all(a2.level <= lev)
        assert a2.num_levels <= int(lev.max()) + 1


def test_generator_capacity_and_arguments():
    n, rp, ci = matrix("chain40")
    a, g = run(n, rp, ci, max_dist=2, cap=3)
    assert g.moves == 3 and g.stop == oracle.GEN_MOVES
    a, g0 = run(n, rp, ci, max_dist=2, cap=0)
    assert g0.moves == 0 and g0.stop == oracle.GEN_MOVES and g0.steps == 0
    a, gz = run(n, rp, ci, max_dist=0)
    # distance 0 rejects every source
    assert gz.moves == 0 and gz.rejected == gz.steps > 0
    with pytest.raises(ValueError):
        run(n, rp, ci, max_dist=-1)
    with pytest.raises(ValueError):
        run(n, rp, ci, alpha=-1.0)
    e = oracle.generate(0, np.zeros(1, np.int32), np.zeros(0, np.int32), 0, 0.0, 0.0)
    assert e.moves == 0 and e.levels == 0
