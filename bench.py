#!/usr/bin/env python3
"""Benchmark: SpTRSV on an equation-rewritten DAG, forward + adjoint, MI355X.

Workload (default): lower triangle of the 3D 7-point Laplacian on a 128^3
grid in natural order (n = 2,097,152, nnz = 8,339,456), FP64, one
right-hand side from x* ~ U[-1,1]; 1% of the rows rewritten (whole thin
levels, target = level - 1), which cuts the DAG from 382 to 344 levels.

One timed step = the per-solve hot path on the rewritten system:
  rewrite (numeric): L' = M L and B' = M B for the current values / RHS
  forward solve:     X = L'^{-1} B'           (autotuned schedule)
  adjoint:           Y = L'^{-T} G, grad_B = Y - C^T Y, grad_L = -grad_B X^T
The structure-only preprocessing (validation, level analysis, symbolic
rewrite, solve plan) is timed separately and reported under "preprocess".

value = algorithmic HBM bytes of all kernels of a step x steps / elapsed.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# sources of the solve kernels and their schedules (a change invalidates the
# committed counter measurements)
SOLVE_SOURCES = ["paper_2609_40159_amd/csrc/solve.hip", "paper_2609_40159_amd/csrc/solve.hpp",
                 "paper_2609_40159_amd/csrc/sf_block.hpp", "paper_2609_40159_amd/csrc/sf_staged.hpp",
                 "paper_2609_40159_amd/csrc/common.hpp",
                 "paper_2609_40159_amd/csrc/plan.hip"]
METRIC = "SpTRSV HBM GB/s & solves/s, rewritten vs original DAG, fwd+adjoint, batched"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lap3d_128")
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate CPU budget of the oracle baseline")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the comparison solves (original DAG, forced schedules)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload")
    ap.add_argument("--no-pair", action="store_true", help="skip the L-then-U pair section")
    ap.add_argument("--no-generator", action="store_true",
                    help="skip the rewrite-list generator section")
    ap.add_argument("--no-env", action="store_true", help="skip the environment-step section")
    ap.add_argument("--block-rows", type=int, default=0,
                    help="main solve plan: rows per sync-free block (0: timed at plan creation; "
                         "fix it for counter runs)")
    ap.add_argument("--stage-outside", default="auto", choices=["auto", "on", "off"],
                    help="main solve plan: helper waves prefetch outside x values (auto: timed "
                         "at plan creation; fix it for counter runs, whose timings are distorted)")
    ap.add_argument("--env-count", type=int, default=1024, help="environments stepped together")
    ap.add_argument("--env-steps", type=int, default=200, help="timed environment steps")
    ap.add_argument("--batch-count", type=int, default=256, help="matrices in the batch")
    ap.add_argument("--batch-steps", type=int, default=5, help="timed batched launches")
    ap.add_argument("--gen-workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="host processes generating the batch")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# algorithmic bytes (the method's own traffic; cached re-reads not counted)
# ---------------------------------------------------------------------------
def bytes_solve(n, nnz, k, s):
    """Forward solve: row pointers, column indices + values, read B, write X."""
    return 4 * (n + 1) + nnz * (4 + s) + 2 * n * k * s


def bytes_solve_t(n, nnz, k, s):
    """Transposed solve over the successor lists: column pointers, successor
    rows + CSR positions + gathered values, diagonals via row pointers,
    read G, write Y."""
    noff = nnz - n
    return 4 * (n + 1) + noff * (4 + 4 + s) + 4 * (n + 1) + n * s + 2 * n * k * s


def bytes_rewrite_numeric(n, nnz, nnz_p, k, s, nC):
    """Copy of the untouched rows plus the merged rows: read L, write L'
    (values and column indices), read B, write B', write the multipliers."""
    return (4 * (n + 1) * 2 + nnz * (4 + s) + nnz_p * (4 + s) + 2 * n * k * s
            + nC * (4 + 4 + s))


def bytes_apply_mt(n, k, s, nC):
    return 2 * n * k * s + nC * (4 + 4 + s) * 2 + 4 * (n + 1)


def bytes_grad_vals(n, nnz, k, s):
    return 4 * (n + 1) + 4 * nnz + s * nnz + 2 * n * k * s


def src_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_key: str, srchash: str, stage: str, block_rows: int):
    """HBM bytes per launch from committed counter runs, if they are current
    (same solve sources, same block size and staging of outside values)."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except (OSError, ValueError):
        return None
    e = d.get(kernel_key)
    if (not e or e.get("src_hash") != srchash or e.get("stage_outside") != stage
            or e.get("block_rows") != block_rows):
        return None
    return e.get("hbm_bytes_per_launch")


def log(msg: str) -> None:
    """Progress to stderr (the JSON result is the only line on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def compare(cmp, time_solve, plan, plan_orig, rw, B, Bp, G, k, Plan):
    """Original vs rewritten DAG, and the two schedules forced (not part of value)."""
    cmp["orig_fwd_ms"] = time_solve(plan_orig, B)
    cmp["orig_bwd_ms"] = time_solve(plan_orig, G, True)
    cmp["rewritten_fwd_ms"] = time_solve(plan, Bp)
    cmp["rewritten_bwd_ms"] = time_solve(plan, G, True)
    for algo in ("level", "syncfree"):
        pl = Plan(rw.Lp, algo=algo, kmax=k)
        cmp[f"rewritten_fwd_{algo}_ms"] = time_solve(pl, Bp)
        del pl
    cmp["speedup_rewritten_vs_original_fwd"] = cmp["orig_fwd_ms"] / cmp["rewritten_fwd_ms"]
    cmp["speedup_rewritten_vs_original_fwd_adj"] = (
        (cmp["orig_fwd_ms"] + cmp["orig_bwd_ms"]) / (cmp["rewritten_fwd_ms"] + cmp["rewritten_bwd_ms"]))


def bytes_levels(n, nnz):
    """Level computation of one candidate: row pointers, dependency columns,
    the level written per row (the rewritten rows' patterns are extra)."""
    return 4 * (n + 1) + 4 * (nnz - n) + 4 * n


def run_batched(args, man, gen, dev):
    """Many uneven matrices with 1-16 right-hand sides each and 32 candidate
    rewrite sets per matrix: one captured persistent launch, against one
    solve launch per matrix and against per-candidate rewrite + analysis."""
    import numpy as np
    import torch

    import synth
    from paper_2609_40159_amd.api import Batch, CSRMatrix, Rewriter, analyze

    res = {"matrices": len(man)}
    t0 = time.perf_counter()
    mats, xstar = [], []
    for spec, (Lh, xs, Bh) in zip(man, gen):
        L = CSRMatrix.from_arrays(Lh.rowptr, Lh.colidx, Lh.vals, device=dev, dtype=torch.float64)
        Bd = torch.as_tensor(Bh).to(dev).contiguous()
        mats.append((L, Bd, torch.empty_like(Bd)))
        xstar.append(xs)
    torch.cuda.synchronize()
    res["upload_s"] = time.perf_counter() - t0
    n_tot = sum(L.n for L, _, _ in mats)
    nnz_tot = sum(L.nnz for L, _, _ in mats)
    sum_k = sum(spec["k"] for spec in man)
    t0 = time.perf_counter()
    infos = [analyze(L) for L, _, _ in mats]
    res["analyze_all_s"] = time.perf_counter() - t0
    levels = [inf.level for inf in infos]
    cand_mat, rows_l, ptr = [], [], [0]
    for m, spec in enumerate(man):
        lv = levels[m].cpu().numpy()
        for c in range(len(spec["phis"])):
            r = synth.candidate_rows(spec, lv, c)
            cand_mat.append(m)
            rows_l.append(r)
            ptr.append(ptr[-1] + len(r))
    rows = np.concatenate(rows_l).astype(np.int32)
    d_rows = torch.as_tensor(rows, device=dev)
    d_ptr = torch.as_tensor(np.asarray(ptr, np.int32), device=dev)
    C = len(cand_mat)
    pcap = 256 * max(1, rows.size)
    res.update({"n_total": n_tot, "nnz_total": nnz_tot, "rhs_total": sum_k,
                "max_levels": max(inf.num_levels for inf in infos), "candidates": C,
                "candidate_rows": int(rows.size)})

    def timed(bt, fn, reps):
        fn()
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(bt.stream)
            fn()
            b.record(bt.stream)
            b.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    log(f"batch uploaded and analysed; {C} candidates")
    # (1) everything in one launch: solves of all matrices + all candidates
    full = Batch(mats, cand_mat, d_ptr, d_rows, None, pattern_cap=pcap)
    R = [full.plan_info(m)["block_rows"] for m in range(len(mats))]
    res["create_ms"] = full.info["create_ms"]
    res["tasks"] = full.info["tasks"]
    full.capture()
    log(f"full batch created in {res['create_ms']:.0f} ms")
    res["full_ms"] = timed(full, full.launch, args.batch_steps)
    log(f"full batch launch {res['full_ms']:.2f} ms")
    st = full.stats()
    assert full.last_status == "OK" and all(x["valid"] for x in st), full.last_status
    err = 0.0
    for (L, Bd, Xd), xs in zip(mats, xstar):
        xt = torch.as_tensor(xs, device=dev)
        err = max(err, float((Xd - xt).abs().max() / xt.abs().max()))
    res["relerr_vs_xstar_max"] = err
    b_solve = sum(bytes_solve(L.n, L.nnz, spec["k"], 8) for (L, _, _), spec in zip(mats, man))
    b_cand = sum(bytes_levels(mats[m][0].n, mats[m][0].nnz) for m in cand_mat)
    res["full_gbs"] = (b_solve + b_cand) / res["full_ms"] / 1e6
    res["solve_bytes"] = b_solve
    del full
    # (2) solves only: one launch vs one launch per matrix (same schedules)
    solves = Batch(mats, [], None, None, block_rows=R)
    solves.capture()
    res["solves_batched_ms"] = timed(solves, solves.launch, args.batch_steps)
    res["solves_plain_ms"] = timed(solves, solves.solve_plain, max(1, args.batch_steps // 2))
    log("batched and per-matrix solves timed")
    res["solves_per_s_batched"] = sum_k / res["solves_batched_ms"] * 1e3
    res["solves_per_s_plain"] = sum_k / res["solves_plain_ms"] * 1e3
    res["solve_gbs_batched"] = b_solve / res["solves_batched_ms"] / 1e6
    res["solve_gbs_plain"] = b_solve / res["solves_plain_ms"] / 1e6
    res["speedup_solves_batched_vs_plain"] = res["solves_plain_ms"] / res["solves_batched_ms"]
    del solves
    # (3) candidates only: one launch vs rewrite + analysis per candidate
    mats0 = [(L, None, None) for L, _, _ in mats]
    cands = Batch(mats0, cand_mat, d_ptr, d_rows, None, pattern_cap=pcap, block_rows=R)
    cands.capture()
    res["cands_batched_ms"] = timed(cands, cands.launch, args.batch_steps)
    stc = cands.stats()
    res["candidates_per_s_batched"] = C / res["cands_batched_ms"] * 1e3
    log("candidate-only batch timed")
    # per-candidate path on a sample: symbolic + numeric rewrite, then analysis
    sample = list(range(0, C, max(1, C // 64)))[:64]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    same = True
    for c in sample:
        m = cand_mat[c]
        rw = Rewriter(mats[m][0], levels[m], rows_l[c])
        rw.numeric()
        a = analyze(rw.Lp)
        same = same and (a.num_levels == stc[c]["num_levels"] and a.stats["S1"] == stc[c]["S1"]
                         and a.stats["S2"] == stc[c]["S2"] and a.stats["cv"] == stc[c]["cv"])
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / len(sample)
    res["candidates_per_s_plain"] = 1.0 / t_plain
    res["speedup_candidates_batched_vs_plain"] = res["candidates_per_s_batched"] * t_plain
    res["plain_candidate_sample"] = len(sample)
    res["batched_stats_equal_plain"] = bool(same)
    return res


def gen_grid():
    """1024 parameter sets of the rewrite-list generator: MAX_REWRITE_DISTANCE,
    threshold relaxation alpha, thin-ratio stop, move limit."""
    import itertools
    md = [1, 2, 3, 4, 6, 8, 12, 16]
    al = [0.0, 0.25, 0.5, 0.75, 1.0, 1.5, 2.0, 3.0]
    ts = [0.02, 0.3, 0.5, 0.7, 0.8, 0.85, 0.9, 0.95]
    mm = [0, 2048]
    return [dict(max_dist=a, alpha=b, thin_stop=c, max_moves=d)
            for a, b, c, d in itertools.product(md, al, ts, mm)]


def run_generator(args, L, Lh, info, dev):
    """Rewrite-list generation for a grid of parameter sets on the workload's
    matrix (one launch, one wave per environment), the lists turned into
    candidate row sets and scored in one batched launch (levels and CV of
    each rewritten matrix).  Returns the figures and a sample of lists for
    the CPU-baseline leg."""
    import numpy as np
    import torch

    from paper_2609_40159_amd import _lib
    from paper_2609_40159_amd.api import Batch, gen_rowsets, generate

    params = gen_grid()
    ne, cap = len(params), 8192
    res = {"workload": "matrix of the main workload", "envs": ne, "cap": cap}
    generate(L, info, params[:4], cap)          # warm-up
    torch.cuda.synchronize()
    ts = []
    for _ in range(3):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        g = generate(L, info, params, cap, sync=False)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    g = generate(L, info, params, cap)
    steps = sum(r["steps"] for r in g.results)
    moves = sum(r["moves"] for r in g.results)
    res.update({"generate_ms": float(np.median(ts)), "steps_total": steps, "moves_total": moves})
    res["steps_per_s"] = steps / res["generate_ms"] * 1e3
    res["envs_per_s"] = ne / res["generate_ms"] * 1e3
    ts = []
    for _ in range(3):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        ptr, rows, tg = gen_rowsets(g)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    res["rowsets_ms"] = float(np.median(ts))
    log("generator timed")
    # scoring: every list as a batch candidate (L' is not formed)
    total = int(ptr[-1])
    pcap = 16 * max(1, total) + (1 << 20)
    bt = None
    for _ in range(4):
        try:
            bt = Batch([(L, None, None)], [0] * ne, ptr, rows, tg, cand_rows_cap=max(1, rows.numel()),
                       pattern_cap=pcap)
            bt.run()
            st = bt.stats()
            break
        except _lib.RwtError as e:
            if e.name != "TOO_LARGE":
                raise
            bt = None
            pcap *= 4
    res["pattern_cap"] = pcap
    bt.capture()
    ts = []
    for _ in range(3):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(bt.stream)
        bt.launch()
        b.record(bt.stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    st = bt.stats()
    res["score_ms"] = float(np.median(ts))
    res["candidates_per_s"] = ne / res["score_ms"] * 1e3
    best = min(range(ne), key=lambda e: (st[e]["num_levels"], st[e]["cv"]))
    res["best"] = {"params": params[best], "moves": g.results[best]["moves"],
                   "levels": st[best]["num_levels"], "cv": st[best]["cv"],
                   "levels_original": info.num_levels, "cv_original": info.stats["cv"],
                   "env_levels": g.results[best]["levels"], "env_cv": g.results[best]["cv"]}
    log("generated lists scored")
    # a sample of environments for the CPU-baseline leg (oracle rate and
    # equality of the lists), taken to the host here
    sample = list(range(0, ne, ne // 16))[:16]
    cmp = {"params": [params[e] for e in sample], "cap": cap,
           "results": [g.results[e] for e in sample],
           "rows": g.rows[sample].cpu().numpy(), "src": g.src[sample].cpu().numpy(),
           "tgt": g.tgt[sample].cpu().numpy(), "level": info.level.cpu().numpy(),
           "D": info.num_levels, "alc": info.stats["alc"], "cv": info.stats["cv"]}
    del bt
    return res, cmp


def run_env(args, L, info, dev):
    """Environment steps (Algorithms 1 and 2) for env_count environments on
    the workload's matrix under a uniform random policy over each mask.  A
    rollout step -- the policy's draw (torch) from the current mask, then the
    step with the observation of the new state in the same launch -- is
    captured in a HIP graph and replayed; the observation and the policy
    alone are timed as well."""
    import numpy as np
    import torch

    from paper_2609_40159_amd.api import Env

    E, K = args.env_count, args.env_steps
    t0 = time.perf_counter()
    env = Env(L, info, E, cap=max(8, 4 * K))
    torch.cuda.synchronize()
    init_ms = (time.perf_counter() - t0) * 1e3

    def one():
        # the mask of the current state was written by the previous step
        score = torch.rand(env.mask.shape, device=dev) * env.mask
        return env.step(score.argmax(dim=1).to(torch.int32), observe=True)

    env.observe()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(3):
            one()
    torch.cuda.current_stream().wait_stream(s)
    # CH rollout steps per graph, the returns summed inside it: one replay
    # per CH steps keeps the host's launch cost off the step
    CH = 20
    K = (K + CH - 1) // CH * CH
    rewards = torch.zeros(E, dtype=torch.float64, device=dev)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(CH):
            st = one()
            rewards += st.reward
    env.reset()
    env.observe()
    rewards.zero_()
    torch.cuda.synchronize()
    a0 = torch.cuda.Event(enable_timing=True)
    a1 = torch.cuda.Event(enable_timing=True)
    a0.record()
    for _ in range(K // CH):
        g.replay()
    a1.record()
    torch.cuda.synchronize()
    total = a0.elapsed_time(a1)
    res = st.results()
    moves = sum(r["moves"] for r in res)
    done = sum(1 for r in res if r["done"] >= 0)
    # the observation and the policy alone, back to back in a graph (they
    # do not change the state); the step is the rest of the rollout step
    mask_fixed = env.mask.clone()

    def timed(fn, reps=50):
        fn()
        torch.cuda.synchronize()
        b0 = torch.cuda.Event(enable_timing=True)
        b1 = torch.cuda.Event(enable_timing=True)
        gg = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gg):
            for _ in range(reps):
                fn()
        b0.record()
        gg.replay()
        b1.record()
        torch.cuda.synchronize()
        return b0.elapsed_time(b1) / reps

    obs_ms = timed(lambda: env.observe())
    pol_ms = timed(lambda: (torch.rand(mask_fixed.shape, device=dev) * mask_fixed)
                   .argmax(dim=1).to(torch.int32))
    out = {"workload": "matrix of the main workload", "envs": E, "steps": K,
           "policy": "uniform over each environment's mask (torch), in the graph",
           "steps_per_graph": CH,
           "init_ms": init_ms, "rollout_ms_per_step": total / K,
           "env_steps_per_s": E * K / total * 1e3,
           "observe_ms": obs_ms, "policy_ms": pol_ms,
           "step_observe_ms_by_difference": total / K - pol_ms,
           "moves": moves, "episodes_ended": done,
           "mean_return": float(rewards.mean().item())}
    del env, g
    return out


def run_pair(args, L, Lh, dev, k, plan_rw=None, rwres=None):
    """The L-then-U pair of an incomplete factorization M = L L^T (U = L^T, an
    upper CSR with the diagonal first): one preconditioner application per
    call, and the upper solve alone."""
    import numpy as np
    import torch

    import synth
    from paper_2609_40159_amd.api import CSRMatrix, Plan, UpperPlan, apply_M, solve_pair

    Uh = synth.transpose_upper(Lh)
    U = CSRMatrix.from_arrays(Uh.rowptr, Uh.colidx, Uh.vals, device=dev, dtype=L.dtype)
    t0 = time.perf_counter()
    Up = UpperPlan(U, kmax=k)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    Lp = Plan(L, kmax=k)
    rng = np.random.default_rng(5)
    Bh = rng.standard_normal((k, Lh.n))
    B = torch.as_tensor(Bh).to(device=dev, dtype=L.dtype).contiguous()
    X = torch.empty_like(B)

    def timed(fn, reps=20):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    pair_ms = timed(lambda: solve_pair(Lp, Up, B, out=X))
    up_ms = timed(lambda: Up.solve(B, out=X))
    rw_pair_ms = None
    if plan_rw is not None:
        # with the rewritten factor: X = U^-1 L'^-1 (M B) = U^-1 L^-1 B
        rw_pair_ms = timed(lambda: solve_pair(plan_rw, Up, apply_M(rwres, B), out=X))
    Up.check()
    s = 8 if L.dtype == torch.float64 else 4
    b_pair = bytes_solve(Lh.n, Lh.nnz, k, s) * 2
    Xh = solve_pair(Lp, Up, B, out=X).double().cpu().numpy()
    Xr = None
    if plan_rw is not None:
        Xr = solve_pair(plan_rw, Up, apply_M(rwres, B)).double().cpu().numpy()
    res = {"what": "X = U^-1 L^-1 B with U = L^T (upper CSR), main workload's original factor",
           "rhs": k, "upper_plan_ms": plan_ms, "upper_algo": Up.info["algo_fwd"],
           "upper_block_rows": Up.info["block_rows"], "pair_ms": pair_ms, "upper_ms": up_ms,
           "pair_gbs": b_pair / pair_ms / 1e6, "applications_per_s": 1e3 / pair_ms,
           "rewritten_pair_ms": rw_pair_ms,
           "speedup_rewritten_pair": None if rw_pair_ms is None else pair_ms / rw_pair_ms}
    return res, {"Uh": Uh, "Bh": Bh, "X": Xh, "X_rewritten": Xr}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: the build targets a "
                          "single MI355X (multi-GPU sharding is described, not run)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import synth

    # batched workload inputs: generated first, in forked host processes,
    # before anything touches the GPU
    man = gen = None
    gen_s = 0.0
    if not args.no_batch:
        t0 = time.perf_counter()
        man = synth.batch_manifest(count=args.batch_count)
        gen = synth.build_batch(man, args.gen_workers)
        gen_s = time.perf_counter() - t0
        log(f"batch inputs generated in {gen_s:.1f} s")

    from paper_2609_40159_amd import _lib
    from paper_2609_40159_amd.api import (CSRMatrix, Plan, Rewriter, analyze, apply_MT,
                                          grad_vals, validate)

    _lib.load()   # fails loudly without the HIP library
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    dev = "cuda:0"
    torch.cuda.set_device(0)
    dtype = torch.float64 if args.dtype == "f64" else torch.float32
    s = 8 if args.dtype == "f64" else 4
    spec = synth.WORKLOADS[args.workload]
    k = 1 if args.workload == "lap3d_128" else spec["k"]

    # ---------------- inputs (host generation, not timed) ----------------
    Lh = synth.build_matrix(spec)
    xs, Bh = synth.rhs(Lh, k, spec["seed"])
    rng = np.random.default_rng(spec["seed"] + 100)
    Gh = rng.standard_normal((k, Lh.n))
    n, nnz = Lh.n, Lh.nnz
    L = CSRMatrix.from_arrays(Lh.rowptr, Lh.colidx, Lh.vals, device=dev, dtype=dtype)
    B = torch.as_tensor(Bh).to(device=dev, dtype=dtype).contiguous()
    G = torch.as_tensor(Gh).to(device=dev, dtype=dtype).contiguous()
    vals = L.vals.clone()
    torch.cuda.synchronize()

    def ev():
        return torch.cuda.Event(enable_timing=True)

    # ---------------- preprocessing (structure only), timed once ----------
    pre = {}
    t0 = time.perf_counter()
    st, _ = validate(L)
    assert st == "OK", st
    torch.cuda.synchronize()
    pre["validate_ms"] = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    info = analyze(L)
    pre["analyze_ms"] = (time.perf_counter() - t0) * 1e3
    level_h = info.level.cpu().numpy()
    frac = spec["frac"]
    if spec["rule"] == "longest_path":
        rows = synth.longest_path_rows(Lh, level_h, frac)
        targets = None
    else:
        rows, targets = synth.thin_first_rows(level_h, frac)
    t0 = time.perf_counter()
    rw = Rewriter(L, info.level, rows, targets)
    torch.cuda.synchronize()
    pre["rewrite_symbolic_ms"] = (time.perf_counter() - t0) * 1e3
    Bp = rw.numeric(vals, B)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = Plan(rw.Lp, algo="auto", kmax=k, block_rows=args.block_rows,
                stage_outside=args.stage_outside)
    torch.cuda.synchronize()
    pre["plan_ms"] = (time.perf_counter() - t0) * 1e3
    pinfo = plan.info
    plan_orig = Plan(L, algo="auto", kmax=k)
    oinfo = plan_orig.info
    nnz_p = rw.nnz
    nC = rw.nc
    Dp = pinfo["stats"]["num_levels"]
    D0 = info.num_levels
    rwres = rw.result()

    # ---------------- per-step phases ----------------
    b_rw = bytes_rewrite_numeric(n, nnz, nnz_p, k, s, nC)
    b_fwd = bytes_solve(n, nnz_p, k, s)
    b_bwd = bytes_solve_t(n, nnz_p, k, s)
    b_mt = bytes_apply_mt(n, k, s, nC)
    b_gv = bytes_grad_vals(n, nnz, k, s)
    b_step = b_rw + b_fwd + b_bwd + b_mt + b_gv

    def step(evs=None):
        e = evs
        if e: e[0].record()
        Bp = rw.numeric(vals, B)
        if e: e[1].record()
        X = plan.solve(Bp)
        if e: e[2].record()
        Y = plan.solve_transpose(G)
        if e: e[3].record()
        gB = apply_MT(rwres, Y)
        if e: e[4].record()
        gV = grad_vals(L, gB, X)
        if e: e[5].record()
        return X, gB, gV

    log("main workload prepared")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.check()

    evsets = [[ev() for _ in range(6)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        X, gB, gV = step(evsets[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    plan.check()

    ph = {"rewrite_numeric": [], "fwd": [], "bwd": [], "apply_MT": [], "grad_vals": []}
    names = list(ph)
    for e in evsets:
        for j, nm in enumerate(names):
            ph[nm].append(e[j].elapsed_time(e[j + 1]))
    ms = {nm: float(np.mean(v)) for nm, v in ph.items()}

    # correctness of the timed result (cheap checks against the known solution)
    Xh = X.double().cpu().numpy()
    err = float(np.max(np.abs(Xh - xs)) / np.max(np.abs(xs)))

    # ---------------- comparisons (not part of value) ----------------
    def time_solve(pl, Bt, transposed=False, reps=10):
        f = pl.solve_transpose if transposed else pl.solve
        for _ in range(2):
            f(Bt)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, b = ev(), ev()
            a.record()
            f(Bt)
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        pl.check()
        return float(np.median(ts))

    cmp = {}
    if args.no_compare:
        cmp = None
    else:
        compare(cmp, time_solve, plan, plan_orig, rw, B, Bp, G, k, Plan)

    # stream-copy rate of the device, reported with every run (a reference
    # for the roofline; the counter runs also scale FETCH/WRITE_SIZE by it)
    a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    b2 = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record()
    for _ in range(5):
        b2.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    copy_probe = {"bytes_each": 2 * a.numel() * 8, "ms_each": e0.elapsed_time(e1) / 5}
    del a, b2

    log("main workload timed")
    generator = gen_cmp = None
    if not args.no_generator:
        generator, gen_cmp = run_generator(args, L, Lh, info, dev)
    pair = pair_cmp = None
    if not args.no_pair:
        pair, pair_cmp = run_pair(args, L, Lh, dev, k, plan, rwres)
    envres = None
    if not args.no_env:
        envres = run_env(args, L, info, dev)
        log("environment steps timed")
    # ---------------- CPU oracle baseline ----------------
    # The oracle runs here only: the main step on a bounded sample, and
    # beside it the generator sample and the pair (their lists and results
    # compared with the GPU's)
    cpu = None
    if not args.no_cpu:
        import oracle
        a = oracle.analyze(n, Lh.rowptr, Lh.colidx)
        # one oracle step: rewrite (it has no separate numeric phase), forward
        # solve of the rewritten system, adjoint of the original system
        reps = 0
        t_cpu = 0.0
        t_start = time.perf_counter()
        while True:
            t1 = time.perf_counter()
            ro = oracle.rewrite(n, Lh.rowptr, Lh.colidx, Lh.vals, a.level, rows, targets, Bh)
            Xo = oracle.solve(n, ro.rowptr, ro.colidx, ro.vals, ro.Bp)
            oracle.adjoint(n, Lh.rowptr, Lh.colidx, Lh.vals, Xo, Gh)
            t_cpu += time.perf_counter() - t1
            reps += 1
            if time.perf_counter() - t_start > args.cpu_seconds or reps >= 500:
                break
        cpu = {"value": b_step * reps / t_cpu / 1e9, "unit": "GB/s", "cores": 1,
               "kind": "oracle", "ms_per_step": t_cpu / reps * 1e3,
               "sample": f"{reps} full steps (rewrite, forward solve, adjoint) of the same "
                         f"workload, single-threaded FP64 oracle"}
        if gen_cmp is not None:
            t_or, steps_or, same = 0.0, 0, True
            for q, prm in enumerate(gen_cmp["params"]):
                t1 = time.perf_counter()
                o = oracle.generate(n, Lh.rowptr, gen_cmp["level"], gen_cmp["D"], gen_cmp["alc"],
                                    gen_cmp["cv"], cap=gen_cmp["cap"], **prm)
                t_or += time.perf_counter() - t1
                steps_or += o.steps
                r = gen_cmp["results"][q]
                m = o.moves
                same = same and m == r["moves"] and o.steps == r["steps"] and o.cv == r["cv"] \
                    and np.array_equal(gen_cmp["rows"][q, :m], o.rows) \
                    and np.array_equal(gen_cmp["src"][q, :m], o.src) \
                    and np.array_equal(gen_cmp["tgt"][q, :m], o.tgt)
            cpu["generator"] = {"value": steps_or / t_or, "unit": "steps/s", "cores": 1,
                                "sample": f"{len(gen_cmp['params'])} environments of the grid",
                                "lists_equal_gpu": bool(same)}
        if envres is not None:
            # one oracle environment under the same kind of policy, about 3 s
            rng = np.random.default_rng(7)
            oe = oracle.Env(n, Lh.rowptr, a.level, a.num_levels, a.alc, a.cv, cap=4 * args.env_steps)
            t1 = time.perf_counter()
            ks = 0
            while time.perf_counter() - t1 < 3.0 and ks < args.env_steps:
                _, _, m = oe.observe()
                v = np.flatnonzero(m)
                r = oe.step(int(rng.choice(v)) if v.size else 0)
                ks += 1
                if r["done"] >= 0:
                    oe.reset()
            cpu["env"] = {"value": ks / (time.perf_counter() - t1), "unit": "env steps/s",
                          "cores": 1, "sample": f"{ks} steps of one environment with its "
                                                 "observation and mask"}
        if pair_cmp is not None:
            Uh = pair_cmp["Uh"]
            t1 = time.perf_counter()
            ref = oracle.solve_pair(n, Lh.rowptr, Lh.colidx, Lh.vals, Uh.rowptr, Uh.colidx,
                                    Uh.vals, pair_cmp["Bh"])
            t_or = time.perf_counter() - t1
            rel = lambda x: float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))
            cpu["pair"] = {"value": 1.0 / t_or, "unit": "applications/s", "cores": 1,
                           "sample": "one application", "relerr_gpu": rel(pair_cmp["X"]),
                           "relerr_gpu_rewritten": (None if pair_cmp["X_rewritten"] is None
                                                    else rel(pair_cmp["X_rewritten"]))}

    # ---------------- roofline of the dominant kernel ----------------
    # the forward and the transposed solve take most of a step; the longer
    # of the two is the dominant kernel (its phase also holds the sentinel
    # prefill of the output, a plain n*k store)
    srch = src_hash(SOLVE_SOURCES)
    tname = "double" if s == 8 else "float"
    roofs = {}
    for ph_name, trans, nbytes in (("fwd", False, b_fwd), ("bwd", True, b_bwd)):
        algo = pinfo["algo_fwd"] if not trans else pinfo["algo_bwd"]
        kname = f"k_solve_{'sf' if algo == 'syncfree' else 'level'}<{tname}, {str(trans).lower()}, 1>"
        achieved = nbytes / (ms[ph_name] * 1e-3) / 1e9
        roofs[ph_name] = {
            "bound": "hbm", "kernel": kname, "achieved": achieved, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
            "traffic": load_traffic(f"{args.workload}:{args.dtype}:{kname}", srch,
                                    pinfo["stage_outside"], pinfo["block_rows"]),
            "algorithmic_bytes_per_launch": nbytes, "avg_launch_ms": ms[ph_name],
            "latency_floor_note": f"{Dp} dependent levels on the critical path"}
    dom = "fwd" if ms["fwd"] >= ms["bwd"] else "bwd"
    roof = roofs[dom]
    # floors of the solves: HBM time of their algorithmic bytes, and one
    # measured cross-workgroup hand-off per dependent level
    from paper_2609_40159_amd.api import probe_handoff
    hop_ns = probe_handoff(2000)
    for rf in roofs.values():
        rf["bandwidth_floor_ms"] = rf["algorithmic_bytes_per_launch"] / (PEAK_HBM_GBS * 1e9) * 1e3
        rf["handoff_ns"] = hop_ns
        rf["latency_floor_ms"] = Dp * hop_ns * 1e-6
    batched = run_batched(args, man, gen, dev) if man is not None else None
    if batched is not None:
        # floors of the batched solves: all their bytes at 8 TB/s, and the
        # deepest matrix's levels times the measured hand-off
        batched["solve_bandwidth_floor_ms"] = batched["solve_bytes"] / (PEAK_HBM_GBS * 1e9) * 1e3
        batched["solve_latency_floor_ms"] = batched["max_levels"] * hop_ns * 1e-6
        batched["handoff_ns"] = hop_ns
    if batched is not None:
        batched["host_generation_s"] = gen_s

    ms_per_step = elapsed / args.steps * 1e3
    value = b_step * args.steps / elapsed / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"{args.workload}: 3D 7-point Laplacian lower factor 128^3 natural "
                               f"order, n={n}, nnz={nnz}, k={k} RHS, 1% rows rewritten "
                               f"(thin-first whole levels, depth 1)" if args.workload == "lap3d_128"
                   else args.workload,
                   "n": n, "nnz": nnz, "nnz_rewritten": nnz_p, "rewritten_rows": int(len(rows)),
                   "levels_original": D0, "levels_rewritten": Dp,
                   "cv_original": info.stats["cv"], "cv_rewritten": pinfo["stats"]["cv"],
                   "rhs": k, "parallelism": "single GPU"},
        "solves_per_s": args.steps / elapsed,
        "step_phase_ms": ms,
        "phase_gbs": {"rewrite_numeric": b_rw / ms["rewrite_numeric"] / 1e6,
                      "fwd": b_fwd / ms["fwd"] / 1e6, "bwd": b_bwd / ms["bwd"] / 1e6,
                      "apply_MT": b_mt / ms["apply_MT"] / 1e6,
                      "grad_vals": b_gv / ms["grad_vals"] / 1e6},
        "plan": {"rewritten": {kk: pinfo[kk] for kk in ("algo_fwd", "algo_bwd", "block_rows",
                                                          "lanes_per_row", "narrow_rows", "grid",
                                                          "stage_outside", "tuned_ms_level",
                                                          "tuned_ms_syncfree")},
                 "original": {kk: oinfo[kk] for kk in ("algo_fwd", "tuned_ms_level",
                                                         "tuned_ms_syncfree")}},
        "compare": cmp,
        "preprocess": pre,
        "relerr_vs_xstar": err,
        "roofline": roof,
        "roofline_other": roofs["bwd" if dom == "fwd" else "fwd"],
        "generator": generator,
        "pair": pair,
        "env": envres,
        "batched": batched,
        "cpu_baseline": cpu,
    }
    if copy_probe:
        out["copy_probe"] = copy_probe
        out["stream_copy_gbs"] = copy_probe["bytes_each"] / (copy_probe["ms_each"] * 1e-3) / 1e9
    print(json.dumps(out))


if __name__ == "__main__":
    main()
