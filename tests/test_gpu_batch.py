"""GPU parity of the batched persistent launch: per-matrix solves and the
level statistics of many candidate rewrite sets, eager and graph-replayed."""
import numpy as np
import pytest
import torch

import synth
from gpu_helpers import DEV, block, host, relerr, to_gpu

pytestmark = pytest.mark.gpu


def oracle_cand(orc, L, level, rows, targets):
    """Level statistics of the rewritten matrix, from the oracle."""
    rw = orc.rewrite(L.n, L.rowptr, L.colidx, L.vals, level, rows, targets)
    a = orc.analyze(L.n, rw.rowptr, rw.colidx)
    return {"num_levels": a.num_levels, "S1": a.S1, "S2": a.S2, "cv": a.cv}


def same_stats(got, ref):
    assert got["valid"]
    assert got["num_levels"] == ref["num_levels"]
    assert got["S1"] == ref["S1"] and got["S2"] == ref["S2"]
    assert got["cv"] == ref["cv"]          # exact radicand, one rounding per operation


def mixed_matrices():
    return [
        ("lap2d_40", synth.laplacian_2d(40, 40), 1),
        ("powerlaw_3k", synth.power_law(3000, 21), 3),
        ("lap3d_12x10x9", synth.laplacian_3d(12, 10, 9), 16),
        ("random_400", synth.random_lower(400, 0.04, 22), 0),     # analysis only
        ("powerlaw_20k", synth.power_law(20000, 23), 5),
        ("lap2d_150x90", synth.laplacian_2d(150, 90), 2),
    ]


def candidate_sets(orc, mats, seed):
    """(matrix index, rows, targets or None) of several kinds per matrix."""
    rng = np.random.default_rng(seed)
    out = []
    for m, (_, L, _) in enumerate(mats):
        a = orc.analyze(L.n, L.rowptr, L.colidx)
        if a.num_levels > 1:
            out.append((m, synth.longest_path_rows(L, a.level, 0.02), None))
            out.append((m, *synth.thin_first_rows(a.level, 0.01)))
        rows, _ = synth.random_rowset(a.level, 0.05, int(rng.integers(1 << 30)))
        t = np.array([int(rng.integers(0, lv + 2)) for lv in a.level[rows]], np.int32)
        out.append((m, rows, t))
        out.append((m, np.zeros(0, np.int32), None))                   # empty set
        out.append((m, np.nonzero(a.level == 0)[0][:5].astype(np.int32), None))   # no-op rows
    return out


def pack(cands, with_targets):
    ptr = np.zeros(len(cands) + 1, np.int64)
    rows, tg = [], []
    for c, (m, r, t) in enumerate(cands):
        ptr[c + 1] = ptr[c] + len(r)
        rows.append(np.asarray(r, np.int32))
        tg.append(np.asarray(t if t is not None else np.full(len(r), -1), np.int32))
    rows = np.concatenate(rows) if rows else np.zeros(0, np.int32)
    tg = np.concatenate(tg) if tg else np.zeros(0, np.int32)
    return [m for m, _, _ in cands], ptr.astype(np.int32), rows, tg


def make_batch(mats, cands, with_targets=False, cap_extra=0, pattern_cap=0, cand_mode="auto"):
    from paper_2609_40159_amd.api import Batch
    gm, rhs = [], []
    for _, L, k in mats:
        G = to_gpu(L)
        if k > 0:
            xs, B = synth.rhs(L, k, 31 + L.n)
            Bd = block(B)
            Xd = torch.empty_like(Bd)
            gm.append((G, Bd, Xd))
            rhs.append((xs, B))
        else:
            gm.append((G, None, None))
            rhs.append((None, None))
    cm, ptr, rows, tg = pack(cands, with_targets)
    cap = rows.size + cap_extra
    d_rows = torch.zeros(max(cap, 1), dtype=torch.int32, device=DEV)
    d_rows[:rows.size] = torch.as_tensor(rows, device=DEV)
    d_ptr = torch.as_tensor(ptr, device=DEV)
    d_t = None
    if with_targets:
        d_t = torch.zeros(max(cap, 1), dtype=torch.int32, device=DEV)
        d_t[:tg.size] = torch.as_tensor(tg, device=DEV)
    bt = Batch(gm, cm, d_ptr, d_rows, d_t, cand_rows_cap=cap, pattern_cap=pattern_cap,
               cand_mode=cand_mode)
    return bt, gm, rhs


def check_solves(orc, mats, gm, rhs):
    for (name, L, k), (G, Bd, Xd), (xs, B) in zip(mats, gm, rhs):
        if k == 0:
            continue
        ref = orc.solve(L.n, L.rowptr, L.colidx, L.vals, B)
        assert relerr(host(Xd), ref) <= 1e-12, name


def check_cands(orc, mats, cands, got, levels):
    for c, (m, rows, t) in enumerate(cands):
        L = mats[m][1]
        ref = oracle_cand(orc, L, levels[m], rows, t)
        same_stats(got[c], ref)


def pattern_need(orc, mats, cands, levels):
    """Entries of all rewritten rows of all candidates (exact capacity)."""
    need = 0
    for m, rows, t in cands:
        L = mats[m][1]
        rw = orc.rewrite(L.n, L.rowptr, L.colidx, L.vals, levels[m], rows, t)
        need += int(np.sum(rw.rowptr[np.asarray(rows) + 1] - rw.rowptr[np.asarray(rows)]))
    return need


def explicit(cands, levels):
    """The same candidates with explicit targets (level - 1, floored at 0,
    where none was drawn)."""
    out = []
    for m, r, t in cands:
        if t is None:
            t = np.maximum(levels[m][r] - 1, 0).astype(np.int32)
        out.append((m, r, np.asarray(t, np.int32)))
    return out


def levels_of(orc, mats):
    return [orc.analyze(L.n, L.rowptr, L.colidx).level for _, L, _ in mats]


def test_batch_solves_and_candidates_eager(orc):
    mats = mixed_matrices()
    cands = candidate_sets(orc, mats, 1)
    bt, gm, rhs = make_batch(mats, cands)
    info = bt.info
    assert info["tasks"] > info["solve_tasks"] > 0
    bt.run()
    torch.cuda.synchronize()
    check_solves(orc, mats, gm, rhs)
    # default targets (level - 1) when no target array is given
    cands_nt = [(m, r, None) for m, r, _ in cands]
    bt2, _, _ = make_batch(mats, cands_nt)
    bt2.run()
    check_cands(orc, mats, cands_nt, bt2.stats(), levels_of(orc, mats))


def test_batch_explicit_targets(orc):
    mats = mixed_matrices()
    cands = candidate_sets(orc, mats, 2)
    levels = levels_of(orc, mats)
    # explicit targets for every candidate (level - 1 where none was drawn)
    full = explicit(cands, levels)
    need = pattern_need(orc, mats, full, levels)
    bt, gm, rhs = make_batch(mats, full, with_targets=True, pattern_cap=need)
    bt.run()
    check_solves(orc, mats, gm, rhs)
    check_cands(orc, mats, full, bt.stats(), levels)


def test_batch_solve_bitwise_equals_single_plan(orc):
    """The schedule the batch chose per matrix (the row-order walk, or
    sync-free blocks with the same block size and lanes: the batched block
    body is the plain one) gives the single-matrix plan's bits."""
    from paper_2609_40159_amd.api import Plan
    mats = [m for m in mixed_matrices() if m[2] > 0]
    bt, gm, rhs = make_batch(mats, [])
    bt.run()
    kinds = set()
    for i, ((name, L, k), (G, Bd, Xd)) in enumerate(zip(mats, gm)):
        pi = bt.plan_info(i)
        kinds.add(pi["algo"] == "walk")
        if pi["algo"] == "walk":
            p = Plan(G, algo="walk", kmax=k)
        else:
            p = Plan(G, algo="syncfree", kmax=k, block_rows=pi["block_rows"],
                     lanes_per_row=pi["lanes_per_row"], rhs_chunk=pi["rhs_chunk"])
        X1 = p.solve(Bd)
        assert torch.equal(X1, Xd), name
    assert kinds == {True, False}     # both kinds of schedule in the batch


def test_batch_graph_replays_with_changing_candidates(orc):
    """Graph replays: new right-hand sides and new candidate lists each time,
    eager work and synchronisations in between, every replay checked."""
    mats = mixed_matrices()[:4]
    levels = levels_of(orc, mats)
    rounds = [explicit(candidate_sets(orc, mats, 10 + r), levels) for r in range(4)]
    # the candidate -> matrix map is fixed at creation; the kinds of sets per
    # matrix do not depend on the seed, so it is the same in every round
    for cs in rounds[1:]:
        assert [m for m, _, _ in cs] == [m for m, _, _ in rounds[0]]
    cap = max(sum(len(r) for _, r, _ in cs) for cs in rounds)
    need = max(pattern_need(orc, mats, cs, levels) for cs in rounds)
    bt, gm, rhs = make_batch(mats, rounds[0], with_targets=True, cap_extra=cap, pattern_cap=need)
    bt.capture()
    assert bt.info["captured"]
    for r, cs in enumerate(rounds):
        _, ptr, rows, tg = pack(cs, True)
        bt.cand_ptr.copy_(torch.as_tensor(ptr, device=DEV))
        bt.cand_rows[:rows.size] = torch.as_tensor(rows, device=DEV)
        bt.cand_targets[:tg.size] = torch.as_tensor(tg, device=DEV)
        new_rhs = []
        for (name, L, k), (G, Bd, Xd) in zip(mats, gm):
            if k == 0:
                new_rhs.append((None, None))
                continue
            xs, B = synth.rhs(L, k, 500 + 7 * r + L.n)
            Bd.copy_(block(B))
            Xd.fill_(0.0)
            new_rhs.append((xs, B))
        bt.launch()
        junk = torch.randn(1 << 16, device=DEV).sum()      # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        check_solves(orc, mats, gm, new_rhs)
        check_cands(orc, mats, cs, bt.stats(), levels)
        if r == 1:
            bt.run()                                       # eager launch between replays
            torch.cuda.synchronize()
            check_cands(orc, mats, cs, bt.stats(), levels)


def test_batch_epoch_tags_wrap(orc):
    """Level arrays are cleared only once per 255 launches: check results
    across the wrap of the launch tag."""
    mats = [("lap2d_30", synth.laplacian_2d(30, 30), 1), ("powerlaw_2k", synth.power_law(2000, 41), 0)]
    cands = [(m, r, None) for m, r, _ in candidate_sets(orc, mats, 5)]    # default targets
    levels = levels_of(orc, mats)
    bt, gm, rhs = make_batch(mats, cands, pattern_cap=pattern_need(orc, mats, cands, levels))
    bt.capture()
    for it in range(1, 262):
        bt.launch()
        if it in (1, 253, 254, 255, 256, 257, 261):
            torch.cuda.synchronize()
            check_cands(orc, mats, cands, bt.stats(), levels)
            check_solves(orc, mats, gm, rhs)


def test_batch_rejects_bad_lists(orc):
    mats = mixed_matrices()[:3]
    levels = levels_of(orc, mats)
    good = candidate_sets(orc, mats, 7)[:4]
    n0 = mats[0][1].n
    bad = [
        (0, np.array([5, 3], np.int32), None),          # unsorted
        (0, np.array([4, 4], np.int32), None),          # duplicate
        (0, np.array([1, n0], np.int32), None),         # out of range
        (1, np.array([7, 9], np.int32), np.array([-1, 0], np.int32)),   # negative target
    ]
    # explicit targets everywhere: level - 1 (floored at 0) where none was drawn
    good = explicit(good, levels)
    bad = [(m, r, t if t is not None else np.zeros(len(r), np.int32)) for m, r, t in bad]
    cands = good[:2] + bad + good[2:]
    bt, gm, rhs = make_batch(mats, cands, with_targets=True,
                             pattern_cap=pattern_need(orc, mats, good, levels) + 64 * 8)
    _, ptr, _, _ = pack(cands, True)
    bt.run()
    st = bt.stats()
    assert bt.last_status == "BAD_ROWSET"
    for c, (m, r, t) in enumerate(cands):
        if 2 <= c < 2 + len(bad):
            assert not st[c]["valid"]
            # a rejected candidate reports the levels of the unchanged matrix
            a = orc.analyze(mats[m][1].n, mats[m][1].rowptr, mats[m][1].colidx)
            assert st[c]["num_levels"] == a.num_levels and st[c]["S1"] == a.S1
        else:
            same_stats(st[c], oracle_cand(orc, mats[m][1], levels[m], r, t))
    check_solves(orc, mats, gm, rhs)
    # offsets that decrease reject every candidate, and nothing is read past them
    p2 = torch.as_tensor(ptr, device=DEV).clone()
    p2[1] = p2[2] + 1
    bt.cand_ptr.copy_(p2)
    bt.run()
    st = bt.stats()
    assert bt.last_status == "BAD_ROWSET" and not any(s["valid"] for s in st)
    check_solves(orc, mats, gm, rhs)


def test_batch_pattern_capacity_is_reported(orc):
    from paper_2609_40159_amd.api import RwtError
    mats = [("lap2d_40", synth.laplacian_2d(40, 40), 1)]
    cands = candidate_sets(orc, mats, 3)[:2]
    bt, gm, rhs = make_batch(mats, cands, pattern_cap=8)
    bt.run()
    with pytest.raises(RwtError) as e:
        bt.stats()
    assert e.value.name == "TOO_LARGE"


def test_batch_one_pass_and_two_pass_patterns_agree(orc):
    """Rewritten-row patterns built in one pass (a 32-entry slot per row,
    longer rows in the rest of the capacity) and in two passes (lengths, a
    scan, then patterns) give the same statistics, equal to the oracle's:
    rows past the slot, past both LDS tiers (targets down to level 0) and
    rows and no-op rows included.  When the one-pass layout does not fit the
    capacity but the exact sizes do, the two passes follow within the same
    launch; a capacity below the exact sizes is reported as TOO_LARGE."""
    from paper_2609_40159_amd.api import RwtError
    mats = mixed_matrices()
    levels = levels_of(orc, mats)
    # deep targets (down to level 0: long rows) and one level down (short)
    for cands in (explicit(candidate_sets(orc, mats, 7), levels),
                  explicit([(m, r, None) for m, r, _ in candidate_sets(orc, mats, 8)], levels)):
        need = pattern_need(orc, mats, cands, levels)
        nrows = sum(len(r) for _, r, _ in cands)
        # room for every row past its slot: the one pass fits; the exact
        # sizes: one pass then (if it does not fit) the two passes, or the
        # two passes alone below 48 entries per row
        one, gm, rhs = make_batch(mats, cands, with_targets=True,
                                  pattern_cap=max(need + 32 * nrows, 48 * nrows))
        two, _, _ = make_batch(mats, cands, with_targets=True, pattern_cap=need)
        assert one.info["pattern_slot"] == 32
        assert two.info["pattern_slot"] == (32 if need >= 48 * nrows else 0)
        got = {}
        for name, bt in (("one", one), ("two", two)):
            bt.capture()
            for _ in range(2):
                bt.launch()
                torch.cuda.synchronize()
                got[name] = bt.stats()
                check_cands(orc, mats, cands, got[name], levels)
        assert got["one"] == got["two"]
        check_solves(orc, mats, gm, rhs)
    # rows of a dense factor rewritten one level down: nearly all longer
    # than the slot, more than the 16 entries per row left after the slots
    dense = [("random_dense", synth.random_lower(200, 0.5, 24), 0)]
    lv = levels_of(orc, dense)
    deep = explicit([(0, np.arange(100, 200, dtype=np.int32), None)], lv)
    L = dense[0][1]
    rw = orc.rewrite(L.n, L.rowptr, L.colidx, L.vals, lv[0], deep[0][1], deep[0][2])
    lens = np.diff(rw.rowptr)[100:200]
    assert (lens > 32).mean() > 0.9 and lens.sum() > 48 * 100 - 32 * 100
    small, _, _ = make_batch(dense, deep, with_targets=True, pattern_cap=48 * 100)
    assert small.info["pattern_slot"] == 32
    small.run()
    with pytest.raises(RwtError) as e:
        small.stats()
    assert e.value.name == "TOO_LARGE"
    exact = int(lens.sum())   # one-pass layout would need 32 * 100 more
    for cap in (exact, 256 * 100):
        bt, _, _ = make_batch(dense, deep, with_targets=True, pattern_cap=cap)
        assert bt.info["pattern_slot"] == 32
        bt.capture()
        for _ in range(2):
            bt.launch()
            torch.cuda.synchronize()
            check_cands(orc, dense, deep, bt.stats(), lv)


def test_batch_solves_only_and_candidates_only(orc):
    mats = [("lap2d_20", synth.laplacian_2d(20, 20), 4), ("chain", synth.laplacian_2d(300, 1), 1)]
    bt, gm, rhs = make_batch(mats, [])
    bt.run()
    torch.cuda.synchronize()
    check_solves(orc, mats, gm, rhs)
    assert bt.stats() == []
    mats0 = [(n, L, 0) for n, L, _ in mats]
    lv = levels_of(orc, mats0)
    cands = explicit(candidate_sets(orc, mats0, 4), lv)
    bt, gm, rhs = make_batch(mats0, cands, with_targets=True,
                             pattern_cap=pattern_need(orc, mats0, cands, lv))
    assert bt.info["solve_tasks"] == 0
    bt.run()
    check_cands(orc, mats0, cands, bt.stats(), lv)


def test_batch_argument_errors():
    from paper_2609_40159_amd.api import Batch, RwtError
    L = to_gpu(synth.laplacian_2d(8, 8))
    B = torch.ones(17, L.n, dtype=torch.float64, device=DEV)
    with pytest.raises(RwtError):
        Batch([(L, B, torch.empty_like(B))], [], None, None)        # k > 16
    Lf = to_gpu(synth.laplacian_2d(8, 8), dtype=torch.float32)
    with pytest.raises(TypeError):
        Batch([(Lf, None, None)], [], None, None)
    ptr = torch.zeros(2, dtype=torch.int32, device=DEV)
    rows = torch.zeros(1, dtype=torch.int32, device=DEV)
    with pytest.raises(RwtError):
        Batch([(L, None, None)], [3], ptr, rows)                      # bad matrix index


def test_batch_candidate_modes_agree(orc):
    """Row-block chains, per-candidate level sweeps and row-order walks give
    the same statistics (all equal to the oracle's), for every matrix and
    mode."""
    mats = mixed_matrices()
    cands = explicit(candidate_sets(orc, mats, 5), levels_of(orc, mats))
    levels = levels_of(orc, mats)
    need = pattern_need(orc, mats, cands, levels)
    got = {}
    for mode in ("blocks", "sweep", "walk", "auto"):
        bt, gm, rhs = make_batch(mats, cands, with_targets=True, pattern_cap=need, cand_mode=mode)
        info = bt.info
        if mode == "blocks":
            assert info["sweep_cands"] == 0
        elif mode == "sweep":
            assert info["sweep_cands"] == len(cands)
        bt.run()
        check_solves(orc, mats, gm, rhs)
        got[mode] = bt.stats()
        check_cands(orc, mats, cands, got[mode], levels)
        if mode == "sweep":
            # replays reuse the level arrays under new launch tags
            bt.capture()
            for _ in range(3):
                bt.launch()
                torch.cuda.synchronize()
                assert bt.stats() == got[mode]
    assert got["blocks"] == got["sweep"] == got["auto"]


@pytest.mark.parametrize("mode", ["blocks", "sweep"])
def test_batch_candidate_groups(orc, mode):
    """Groups of candidates of one matrix (up to eight per task): many
    candidates per matrix, runs broken by other matrices' candidates, and a
    rejected list inside a group -- every statistic equal to the oracle's."""
    mats = [("lap2d_48x40", synth.laplacian_2d(48, 40), 0),
            ("powerlaw_6k", synth.power_law(6000, 61), 0),
            ("lap3d_11x10x9", synth.laplacian_3d(11, 10, 9), 0)]
    levels = levels_of(orc, mats)
    rng = np.random.default_rng(62)
    per = []
    for m, (_, L, _) in enumerate(mats):
        lst = []
        for c in range(19):
            rows, _ = synth.random_rowset(levels[m], 0.01 + 0.002 * c, int(rng.integers(1 << 30)))
            t = np.array([int(rng.integers(max(0, lv - 3), lv + 1)) for lv in levels[m][rows]],
                         np.int32)
            lst.append((m, rows, t))
        per.append(lst)
    # 12 consecutive candidates of matrix 0, then the matrices interleaved
    cands = per[0][:12]
    for c in range(7):
        cands += [per[1][c], per[2][c], per[0][12 + c]]
    cands += per[1][7:] + per[2][7:]
    bad_at = 5
    m_bad = cands[bad_at][0]
    cands[bad_at] = (m_bad, np.array([9, 3], np.int32), np.zeros(2, np.int32))   # unsorted
    good = [x for i, x in enumerate(cands) if i != bad_at]
    need = pattern_need(orc, mats, good, levels) + 64
    bt, _, _ = make_batch(mats, cands, with_targets=True, pattern_cap=need, cand_mode=mode)
    assert bt.info["sweep_cands"] == (len(cands) if mode == "sweep" else 0)
    for rep in range(2):
        bt.run()
        st = bt.stats()
        assert bt.last_status == "BAD_ROWSET"
        for c, (m, r, t) in enumerate(cands):
            if c == bad_at:
                assert not st[c]["valid"]
                a = orc.analyze(mats[m][1].n, mats[m][1].rowptr, mats[m][1].colidx)
                assert st[c]["num_levels"] == a.num_levels and st[c]["S1"] == a.S1
            else:
                same_stats(st[c], oracle_cand(orc, mats[m][1], levels[m], r, t))
