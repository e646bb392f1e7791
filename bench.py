#!/usr/bin/env python3
"""Benchmark: SpTRSV on equation-rewritten DAGs with level-set analysis, MI355X.

Headline workload (the largest one that fits one GPU): the batch of 256
uneven lower-triangular matrices, n ~ U[2k, 200k] (64 lower factors of 2D
5-point and 64 of 3D 7-point Laplacians, 128 power-law matrices), each with
1-16 right-hand sides (2,178 in all) and 32 candidate rewrite sets of
0.5-1.5% of its rows (8,192 in all).  One step = one batched launch: every
matrix solved (sync-free row blocks, FP64) and, for every candidate, the
levels of the rewritten matrix with their cost histogram and exact CV --
the setup kernels (candidate checks, batched symbolic rewrite) followed by
one persistent kernel.  value = algorithmic HBM bytes of a step x steps /
elapsed; the roofline entry is the persistent kernel alone, timed with
events recorded on its stream around it.

Beside it (not part of value), each with its bandwidth and latency floors:
  step128   128^3 Laplacian factor, 1% of rows rewritten, FP64, k = 1: the
            per-solve hot path (numeric rewrite, forward solve, adjoint =
            transposed solve + M^T + grad_vals), rewritten vs original DAG,
            level-scheduled vs sync-free;
  fp32      the same factor in FP32, forward + transposed, rewritten vs
            original;
  powerlaw1m power-law n = 1M, 64 right-hand sides, 0.8% rewritten: forward
            and adjoint, rewritten vs original;
  autograd  torch.autograd over the solve, 64^3 factor and power-law 262k,
            32 right-hand sides, forward on the 1% rewrite + backward;
  generator / pair / env: the rewrite-list generator, the L-then-U pair
            and the environment step on the 128^3 factor;
  ppo       masked PPO (Section 4.5) trained over the environment step on a
            power-law matrix, its rewrite lists scored against an untrained
            policy, the thin-first rule and the generator.
The CPU baseline runs the FP64 oracle on a sample of the batch with one
worker thread per host core (the oracle's C calls release the GIL).
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
                 "paper_2609_40159_amd/csrc/common.hpp", "paper_2609_40159_amd/csrc/walk.hpp",
                 "paper_2609_40159_amd/csrc/plan.hip"]
# sources of the batched persistent kernel
BATCH_SOURCES = SOLVE_SOURCES + ["paper_2609_40159_amd/csrc/batch.hip",
                                 "paper_2609_40159_amd/csrc/batch.hpp",
                                 "paper_2609_40159_amd/csrc/rewrite.hip",
                                 "paper_2609_40159_amd/csrc/u128.hpp"]
METRIC = "SpTRSV HBM GB/s & solves/s, rewritten vs original DAG, fwd+adjoint, batched"
SECTIONS = ["batch", "step128", "fp32", "powerlaw1m", "autograd", "generator", "pair", "env", "ppo"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed steps of the headline workload")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sections", default=",".join(SECTIONS),
                    help="comma list of " + ",".join(SECTIONS) + "; the headline is the batch "
                         "when present, else the 128^3 step")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate single-core budget of the 128^3 oracle step")
    ap.add_argument("--cpu-threads", type=int, default=min(16, os.cpu_count() or 1),
                    help="oracle worker threads of the batched CPU baseline")
    ap.add_argument("--cpu-batch-stride", type=int, default=2,
                    help="the batched CPU baseline runs every this many matrices of the batch")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the comparison runs (original DAG, forced schedules, per-matrix batch)")
    ap.add_argument("--block-rows", type=int, default=0,
                    help="128^3 step plan: rows per sync-free block (0: timed at plan creation; "
                         "fix it for counter runs)")
    ap.add_argument("--stage-outside", default="auto", choices=["auto", "on", "off"],
                    help="128^3 step plan: helper waves prefetch outside x values (auto: timed "
                         "at plan creation; fix it for counter runs, whose timings are distorted)")
    ap.add_argument("--step128-steps", type=int, default=20, help="timed 128^3 steps")
    ap.add_argument("--env-count", type=int, default=1024, help="environments stepped together")
    ap.add_argument("--env-steps", type=int, default=200, help="timed environment steps")
    ap.add_argument("--ppo-n", type=int, default=20000, help="rows of the PPO training matrix")
    ap.add_argument("--ppo-envs", type=int, default=4, help="environments PPO trains with")
    ap.add_argument("--ppo-updates", type=int, default=10, help="PPO rollout iterations")
    ap.add_argument("--ppo-seconds", type=float, default=60.0, help="PPO training time limit")
    ap.add_argument("--batch-count", type=int, default=256, help="matrices in the batch")
    ap.add_argument("--gen-workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="host processes generating the batch")
    args = ap.parse_args()
    args.sections = [x for x in args.sections.split(",") if x]
    bad = [x for x in args.sections if x not in SECTIONS]
    if bad:
        ap.error(f"unknown sections {bad}")
    return args


# ---------------------------------------------------------------------------
# algorithmic bytes (the method's own traffic; cached re-reads not counted)
# ---------------------------------------------------------------------------
def bytes_solve(n, nnz, k, s):
    """One triangular solve with k right-hand sides: row pointers, column
    indices + values, read B, write X."""
    return 4 * (n + 1) + nnz * (4 + s) + 2 * n * k * s


def bytes_solve_t(n, nnz, k, s):
    """The transposed solve moves the same algorithmic bytes as the forward
    one (the system's pattern and values, G read, Y written); reading the
    pattern through the successor lists is the implementation's extra."""
    return bytes_solve(n, nnz, k, s)


def bytes_rewrite_numeric(n, nnz, nnz_p, k, s, nC):
    """Copy of the untouched rows plus the merged rows: read L, write L'
    (values and column indices), read B, write B', write the multipliers."""
    return (4 * (n + 1) * 2 + nnz * (4 + s) + nnz_p * (4 + s) + 2 * n * k * s
            + nC * (4 + 4 + s))


def bytes_apply_mt(n, k, s, nC):
    return 2 * n * k * s + nC * (4 + 4 + s) * 2 + 4 * (n + 1)


def bytes_grad_vals(n, nnz, k, s):
    return 4 * (n + 1) + 4 * nnz + s * nnz + 2 * n * k * s


def bytes_levels(n, nnz):
    """Level computation of one candidate: row pointers, dependency columns,
    the level written per row (the rewritten rows' patterns are extra)."""
    return 4 * (n + 1) + 4 * (nnz - n) + 4 * n


def src_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_key: str, srchash: str, stage: str, block_rows: int):
    """HBM bytes per launch from committed counter runs, if they are current
    (same sources, same block size and staging of outside values)."""
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


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def roof(bytes_per_launch, avg_ms, kernel, levels=None, hop_ns=None, traffic=None):
    """Roofline entry of one kernel: algorithmic bytes over its average
    event-timed duration, against the HBM peak, with its floors."""
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    r = {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": PEAK_HBM_GBS,
         "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
         "algorithmic_bytes_per_launch": bytes_per_launch, "avg_launch_ms": avg_ms,
         "bandwidth_floor_ms": bytes_per_launch / (PEAK_HBM_GBS * 1e9) * 1e3}
    if levels is not None and hop_ns is not None:
        r["levels"] = levels
        r["handoff_ns"] = hop_ns
        r["latency_floor_ms"] = levels * hop_ns * 1e-6
    return r


def solve_kernel(algo: str, tname: str, trans: bool, k: int, rhs_chunk: int) -> str:
    """Name of the kernel a plan launches for one solve (as the profiler shows it)."""
    t = str(trans).lower()
    if algo == "walk":
        return f"k_solve_walk<{tname}, {t}>"
    if algo == "syncfree":
        return f"k_solve_sf<{tname}, {t}, {4 if rhs_chunk > 1 else 1}>"
    return f"k_solve_level<{tname}, {t}, {4 if k > 1 else 1}>"


def timed_events(fn, reps, warm=2, stream=None):
    """Median event time (ms) of fn() on the current (or given) stream."""
    import numpy as np
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


# ---------------------------------------------------------------------------
# headline: the batched workload
# ---------------------------------------------------------------------------
def batch_inputs(args, man, gen, dev):
    """Upload the batch, analyse every matrix, draw the candidate row sets."""
    import numpy as np
    import torch

    import synth
    from paper_2609_40159_amd.api import CSRMatrix, analyze

    t0 = time.perf_counter()
    mats, xstar = [], []
    for spec, (Lh, xs, Bh) in zip(man, gen):
        L = CSRMatrix.from_arrays(Lh.rowptr, Lh.colidx, Lh.vals, device=dev, dtype=torch.float64)
        Bd = torch.as_tensor(Bh).to(dev).contiguous()
        mats.append((L, Bd, torch.empty_like(Bd)))
        xstar.append(xs)
    torch.cuda.synchronize()
    upload_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    infos = [analyze(L) for L, _, _ in mats]
    analyze_s = time.perf_counter() - t0
    cand_mat, rows_l, ptr = [], [], [0]
    for m, spec in enumerate(man):
        lv = infos[m].level.cpu().numpy()
        for c in range(len(spec["phis"])):
            r = synth.candidate_rows(spec, lv, c)
            cand_mat.append(m)
            rows_l.append(r)
            ptr.append(ptr[-1] + len(r))
    rows = np.concatenate(rows_l).astype(np.int32)
    return {"mats": mats, "xstar": xstar, "infos": infos, "cand_mat": cand_mat, "rows_l": rows_l,
            "d_rows": torch.as_tensor(rows, device=dev),
            "d_ptr": torch.as_tensor(np.asarray(ptr, np.int32), device=dev),
            "nrows": int(rows.size), "upload_s": upload_s, "analyze_all_s": analyze_s}


def run_batched(args, man, gen, dev, hop_ns):
    """The headline: K timed batched launches (setup + persistent kernel,
    events around the persistent kernel), plus the graph replay, the
    solves-only batch against one launch per matrix, and the candidates-only
    batch against per-candidate rewrite + analysis."""
    import numpy as np
    import torch

    from paper_2609_40159_amd.api import Batch, Rewriter, analyze

    bi = batch_inputs(args, man, gen, dev)
    mats, infos, cand_mat, rows_l = bi["mats"], bi["infos"], bi["cand_mat"], bi["rows_l"]
    C = len(cand_mat)
    n_tot = sum(L.n for L, _, _ in mats)
    nnz_tot = sum(L.nnz for L, _, _ in mats)
    sum_k = sum(spec["k"] for spec in man)
    res = {"matrices": len(mats), "n_total": n_tot, "nnz_total": nnz_tot, "rhs_total": sum_k,
           "max_levels": max(inf.num_levels for inf in infos), "candidates": C,
           "candidate_rows": bi["nrows"], "upload_s": bi["upload_s"],
           "analyze_all_s": bi["analyze_all_s"]}
    log(f"batch uploaded and analysed; {C} candidates")
    pcap = 64 * max(1, bi["nrows"])   # >= 48 per row: one-pass patterns
    full = Batch(mats, cand_mat, bi["d_ptr"], bi["d_rows"], None, pattern_cap=pcap)
    R = [full.plan_info(m)["block_rows"] for m in range(len(mats))]
    res["create_ms"] = full.info["create_ms"]
    res["tasks"] = full.info["tasks"]
    res["grid"] = full.info["grid"]
    log(f"full batch created in {res['create_ms']:.0f} ms")
    b_solve = sum(bytes_solve(L.n, L.nnz, spec["k"], 8) for (L, _, _), spec in zip(mats, man))
    b_cand = sum(bytes_levels(mats[m][0].n, mats[m][0].nnz) for m in cand_mat)
    b_step = b_solve + b_cand
    # ---- the timed steps ----
    for _ in range(args.warmup):
        full.run_timed()
    torch.cuda.synchronize()
    K = args.steps
    t0 = time.perf_counter()
    evs = [full.run_timed() for _ in range(K)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    main_ms = [a.elapsed_time(b) for a, b in evs]
    st = full.stats()
    assert full.last_status == "OK" and all(x["valid"] for x in st), full.last_status
    err = 0.0
    for (L, Bd, Xd), xs in zip(mats, bi["xstar"]):
        xt = torch.as_tensor(xs, device=dev)
        err = max(err, float((Xd - xt).abs().max() / xt.abs().max()))
    res["relerr_vs_xstar_max"] = err
    res["solve_bytes"] = b_solve
    res["candidate_bytes"] = b_cand
    res["step_bytes"] = b_step
    res["main_kernel_ms"] = float(np.mean(main_ms))
    res["main_kernel_ms_min"] = float(np.min(main_ms))
    log(f"batched steps: {elapsed / K * 1e3:.2f} ms per step, persistent kernel "
        f"{res['main_kernel_ms']:.2f} ms")
    # the same launch replayed from its captured graph
    full.capture()
    res["graph_ms"] = timed_events(full.launch, 3, warm=1, stream=full.stream)
    del full
    head = {"elapsed_s": elapsed, "steps": K, "step_bytes": b_step,
            "main_ms": res["main_kernel_ms"]}
    cpu_in = {"cand_mat": cand_mat, "rows_l": rows_l, "levels": [inf.level.cpu().numpy()
                                                                 for inf in infos]}
    if args.no_compare:   # counter runs: the timed launches only
        return res, head, cpu_in
    # ---- solves only: one launch vs one launch per matrix (same schedules) ----
    solves = Batch(mats, [], None, None, block_rows=R)
    solves.capture()
    res["solves_batched_ms"] = timed_events(solves.launch, 3, warm=1, stream=solves.stream)
    res["solves_plain_ms"] = timed_events(solves.solve_plain, 2, warm=1, stream=solves.stream)
    res["solves_per_s_batched"] = sum_k / res["solves_batched_ms"] * 1e3
    res["solves_per_s_plain"] = sum_k / res["solves_plain_ms"] * 1e3
    res["solve_gbs_batched"] = b_solve / res["solves_batched_ms"] / 1e6
    res["solve_gbs_plain"] = b_solve / res["solves_plain_ms"] / 1e6
    res["speedup_solves_batched_vs_plain"] = res["solves_plain_ms"] / res["solves_batched_ms"]
    res["solve_bandwidth_floor_ms"] = b_solve / (PEAK_HBM_GBS * 1e9) * 1e3
    if hop_ns:
        res["solve_latency_floor_ms"] = res["max_levels"] * hop_ns * 1e-6
    del solves
    log("batched and per-matrix solves timed")
    # ---- candidates only: one launch vs rewrite + analysis per candidate ----
    mats0 = [(L, None, None) for L, _, _ in mats]
    cands = Batch(mats0, cand_mat, bi["d_ptr"], bi["d_rows"], None, pattern_cap=pcap, block_rows=R)
    cands.capture()
    res["cands_batched_ms"] = timed_events(cands.launch, 3, warm=1, stream=cands.stream)
    stc = cands.stats()
    res["candidates_per_s_batched"] = C / res["cands_batched_ms"] * 1e3
    sample = list(range(0, C, max(1, C // 64)))[:64]
    levels = [inf.level for inf in infos]
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
    del cands
    log("candidate-only batch timed")
    return res, head, cpu_in


def cpu_batched(args, man, gen, cpu_in):
    """The oracle on every cpu_batch_stride-th matrix of the batch: its
    solve (all its right-hand sides) and its 32 candidates (rewrite, then
    levels and statistics of the rewritten matrix), one matrix per worker
    thread (the oracle's C calls release the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    ms = list(range(0, len(man), max(1, args.cpu_batch_stride)))
    by_mat = {}
    for c, m in enumerate(cpu_in["cand_mat"]):
        by_mat.setdefault(m, []).append(c)

    def one(m):
        Lh, _, Bh = gen[m]
        if Bh is not None:
            oracle.solve(Lh.n, Lh.rowptr, Lh.colidx, Lh.vals, Bh)
        lv = cpu_in["levels"][m]
        for c in by_mat.get(m, []):
            rw = oracle.rewrite(Lh.n, Lh.rowptr, Lh.colidx, Lh.vals, lv, cpu_in["rows_l"][c], None)
            oracle.analyze(Lh.n, rw.rowptr, rw.colidx)
        return m

    nb = sum(bytes_solve(gen[m][0].n, gen[m][0].nnz, man[m]["k"], 8) for m in ms)
    nb += sum(bytes_levels(gen[m][0].n, gen[m][0].nnz) * len(by_mat.get(m, [])) for m in ms)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=args.cpu_threads) as ex:
        list(ex.map(one, ms))
    wall = time.perf_counter() - t0
    return {"value": nb / wall / 1e9, "unit": "GB/s", "cores": args.cpu_threads, "kind": "oracle",
            "cpu_model": cpu_model(), "wall_s": wall,
            "sample": f"{len(ms)} of the batch's {len(man)} matrices (one in every "
                      f"{args.cpu_batch_stride}): each solved for all its right-hand sides and "
                      f"its 32 candidates rewritten and analysed (levels, costs, CV) by the FP64 "
                      f"oracle, one matrix per thread on {args.cpu_threads} threads; the same "
                      f"algorithmic bytes per matrix as the GPU step (the oracle's rewrite also "
                      f"forms the values, which the batched analysis does not need)"}


# ---------------------------------------------------------------------------
# the 128^3 factor: per-solve hot path on the rewritten system
# ---------------------------------------------------------------------------
def prepare_system(spec, k, dev, dtype):
    """Host generation, upload, analysis and the thin-first rewrite's
    symbolic part of one named workload (structure-only work, timed once)."""
    import numpy as np
    import torch

    import synth
    from paper_2609_40159_amd.api import CSRMatrix, Rewriter, analyze, validate

    Lh = synth.build_matrix(spec)
    xs, Bh = synth.rhs(Lh, k, spec["seed"])
    Gh = np.random.default_rng(spec["seed"] + 100).standard_normal((k, Lh.n))
    L = CSRMatrix.from_arrays(Lh.rowptr, Lh.colidx, Lh.vals, device=dev, dtype=dtype)
    B = torch.as_tensor(Bh).to(device=dev, dtype=dtype).contiguous()
    G = torch.as_tensor(Gh).to(device=dev, dtype=dtype).contiguous()
    torch.cuda.synchronize()
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
    if spec["rule"] == "longest_path":
        rows, targets = synth.longest_path_rows(Lh, level_h, spec["frac"]), None
    else:
        rows, targets = synth.thin_first_rows(level_h, spec["frac"])
    t0 = time.perf_counter()
    rw = Rewriter(L, info.level, rows, targets)
    torch.cuda.synchronize()
    pre["rewrite_symbolic_ms"] = (time.perf_counter() - t0) * 1e3
    return {"Lh": Lh, "xs": xs, "Bh": Bh, "Gh": Gh, "L": L, "B": B, "G": G, "info": info,
            "rows": rows, "targets": targets, "rw": rw, "pre": pre}


def solve_pair_times(plan, Bt, Gt):
    """Median event times of the forward and the transposed solve."""
    f = timed_events(lambda: plan.solve(Bt), 5)
    t = timed_events(lambda: plan.solve_transpose(Gt), 5)
    plan.check()
    return f, t


def run_step128(args, dev, dtype, hop_ns, steps):
    """rewrite (numeric) + forward solve + adjoint on the rewritten 128^3
    factor, the original DAG and the two schedules beside it."""
    import numpy as np
    import torch

    import synth
    from paper_2609_40159_amd.api import Plan, apply_MT, grad_vals

    spec = synth.WORKLOADS["lap3d_128"]
    k = 1
    s = 8 if dtype == torch.float64 else 4
    P = prepare_system(spec, k, dev, dtype)
    L, B, G, rw, info = P["L"], P["B"], P["G"], P["rw"], P["info"]
    vals = L.vals.clone()
    n, nnz = L.n, L.nnz
    Bp = rw.numeric(vals, B)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = Plan(rw.Lp, algo="auto", kmax=k, block_rows=args.block_rows,
                stage_outside=args.stage_outside)
    torch.cuda.synchronize()
    P["pre"]["plan_ms"] = (time.perf_counter() - t0) * 1e3
    pinfo = plan.info
    plan_orig = Plan(L, algo="auto", kmax=k)
    oinfo = plan_orig.info
    rwres = rw.result()
    nnz_p, nC = rw.nnz, rw.nc
    Dp, D0 = pinfo["stats"]["num_levels"], info.num_levels
    b_rw = bytes_rewrite_numeric(n, nnz, nnz_p, k, s, nC)
    b_fwd = bytes_solve(n, nnz_p, k, s)
    b_bwd = bytes_solve_t(n, nnz_p, k, s)
    b_mt = bytes_apply_mt(n, k, s, nC)
    b_gv = bytes_grad_vals(n, nnz, k, s)
    b_step = b_rw + b_fwd + b_bwd + b_mt + b_gv

    def step(e=None):
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

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    plan.check()
    evsets = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        X, gB, gV = step(evsets[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    plan.check()
    names = ["rewrite_numeric", "fwd", "bwd", "apply_MT", "grad_vals"]
    ms = {nm: float(np.mean([e[j].elapsed_time(e[j + 1]) for e in evsets]))
          for j, nm in enumerate(names)}
    err = float(np.max(np.abs(X.double().cpu().numpy() - P["xs"])) / np.max(np.abs(P["xs"])))
    tname = "double" if s == 8 else "float"
    srch = src_hash(SOLVE_SOURCES)
    roofs = {}
    for ph, trans, nbytes in (("fwd", False, b_fwd), ("bwd", True, b_bwd)):
        algo = pinfo["algo_fwd"] if not trans else pinfo["algo_bwd"]
        kname = solve_kernel(algo, tname, trans, k, pinfo["rhs_chunk"])
        tr = load_traffic(f"lap3d_128:{'f64' if s == 8 else 'f32'}:{kname}", srch,
                          pinfo["stage_outside"], pinfo["block_rows"])
        roofs[ph] = roof(nbytes, ms[ph], kname, Dp, hop_ns, tr)
    out = {"workload": f"3D 7-point Laplacian lower factor 128^3 natural order, n={n}, "
                       f"nnz={nnz}, k={k}, 1% rows rewritten (thin-first whole levels, depth 1), "
                       f"{'FP64' if s == 8 else 'FP32'}",
           "n": n, "nnz": nnz, "nnz_rewritten": nnz_p, "rewritten_rows": int(len(P["rows"])),
           "levels_original": D0, "levels_rewritten": Dp, "cv_original": info.stats["cv"],
           "cv_rewritten": pinfo["stats"]["cv"], "steps": steps,
           "ms_per_step": elapsed / steps * 1e3, "gbs": b_step * steps / elapsed / 1e9,
           "step_phase_ms": ms,
           "phase_gbs": {"rewrite_numeric": b_rw / ms["rewrite_numeric"] / 1e6,
                         "fwd": b_fwd / ms["fwd"] / 1e6, "bwd": b_bwd / ms["bwd"] / 1e6,
                         "apply_MT": b_mt / ms["apply_MT"] / 1e6,
                         "grad_vals": b_gv / ms["grad_vals"] / 1e6},
           "solve_gbs_fwd_adj": (b_fwd + b_bwd) / (ms["fwd"] + ms["bwd"]) / 1e6,
           "plan": {"rewritten": {kk: pinfo[kk] for kk in (
               "algo_fwd", "algo_bwd", "block_rows", "lanes_per_row", "narrow_rows", "grid",
               "stage_outside", "tuned_ms_level", "tuned_ms_syncfree")},
               "original": {kk: oinfo[kk] for kk in ("algo_fwd", "block_rows", "tuned_ms_level",
                                                      "tuned_ms_syncfree")}},
           "preprocess": P["pre"], "relerr_vs_xstar": err,
           "roofline_fwd": roofs["fwd"], "roofline_bwd": roofs["bwd"]}
    if not args.no_compare:
        cmp = {}
        cmp["orig_fwd_ms"], cmp["orig_bwd_ms"] = solve_pair_times(plan_orig, B, G)
        cmp["rewritten_fwd_ms"], cmp["rewritten_bwd_ms"] = solve_pair_times(plan, Bp, G)
        for algo in ("level", "syncfree"):
            for which, LL, BB in (("rewritten", rw.Lp, Bp), ("orig", L, B)):
                pl = Plan(LL, algo=algo, kmax=k)
                cmp[f"{which}_fwd_{algo}_ms"], cmp[f"{which}_bwd_{algo}_ms"] = \
                    solve_pair_times(pl, BB, G)
                del pl
        cmp["speedup_rewritten_vs_original_fwd"] = cmp["orig_fwd_ms"] / cmp["rewritten_fwd_ms"]
        cmp["speedup_rewritten_vs_original_fwd_adj"] = (
            (cmp["orig_fwd_ms"] + cmp["orig_bwd_ms"]) /
            (cmp["rewritten_fwd_ms"] + cmp["rewritten_bwd_ms"]))
        for algo in ("level", "syncfree"):
            cmp[f"speedup_rewritten_vs_original_fwd_{algo}"] = (
                cmp[f"orig_fwd_{algo}_ms"] / cmp[f"rewritten_fwd_{algo}_ms"])
        out["compare"] = cmp
    ctx = {"P": P, "plan": plan, "rwres": rwres, "b_step": b_step, "k": k}
    return out, ctx


def run_fp32(args, dev, hop_ns):
    """128^3 in FP32: forward and transposed solves, rewritten vs original."""
    import torch

    import synth
    from paper_2609_40159_amd.api import Plan

    spec = synth.WORKLOADS["lap3d_128"]
    P = prepare_system(spec, 1, dev, torch.float32)
    L, B, G, rw = P["L"], P["B"], P["G"], P["rw"]
    Bp = rw.numeric(None, B)
    plan = Plan(rw.Lp, algo="auto", kmax=1)
    plan_o = Plan(L, algo="auto", kmax=1)
    f, t = solve_pair_times(plan, Bp, G)
    fo, to = solve_pair_times(plan_o, B, G)
    X = plan.solve(Bp)
    err = float((X.double().cpu() - torch.as_tensor(P["xs"])).abs().max() /
                torch.as_tensor(P["xs"]).abs().max())
    n, nnzp = L.n, rw.nnz
    Dp = plan.info["stats"]["num_levels"]
    kf = solve_kernel(plan.info["algo_fwd"], "float", False, 1, plan.info["rhs_chunk"])
    kb = solve_kernel(plan.info["algo_bwd"], "float", True, 1, plan.info["rhs_chunk"])
    return {"workload": "128^3 Laplacian factor, FP32, k = 1, 1% rows rewritten",
            "fwd_ms": f, "bwd_ms": t, "orig_fwd_ms": fo, "orig_bwd_ms": to,
            "speedup_rewritten_vs_original_fwd": fo / f,
            "speedup_rewritten_vs_original_fwd_adj": (fo + to) / (f + t),
            "relerr_vs_xstar": err, "plan": {kk: plan.info[kk] for kk in (
                "algo_fwd", "block_rows", "stage_outside")},
            "roofline_fwd": roof(bytes_solve(n, nnzp, 1, 4), f, kf, Dp, hop_ns),
            "roofline_bwd": roof(bytes_solve_t(n, nnzp, 1, 4), t, kb, Dp, hop_ns)}


def run_powerlaw1m(args, dev, hop_ns):
    """Power-law n = 1M, 64 right-hand sides, 0.8% of rows rewritten:
    forward solve and adjoint (transposed solve, M^T, grad_vals), rewritten
    vs original DAG."""
    import numpy as np
    import torch

    import synth
    from paper_2609_40159_amd.api import Plan, apply_MT, grad_vals

    spec = synth.WORKLOADS["powerlaw_1m"]
    k = spec["k"]
    t0 = time.perf_counter()
    P = prepare_system(spec, k, dev, torch.float64)
    L, B, G, rw, info = P["L"], P["B"], P["G"], P["rw"], P["info"]
    Bp = rw.numeric(None, B)
    rwres = rw.result()
    plan = Plan(rw.Lp, algo="auto", kmax=k)
    plan_o = Plan(L, algo="auto", kmax=k)
    prep_s = time.perf_counter() - t0
    log(f"power-law 1M system prepared in {prep_s:.1f} s")
    f = timed_events(lambda: plan.solve(Bp), 3, warm=1)
    t = timed_events(lambda: plan.solve_transpose(G), 3, warm=1)
    X = plan.solve(Bp)
    Y = plan.solve_transpose(G)
    mt = timed_events(lambda: apply_MT(rwres, Y), 3, warm=1)
    gB = apply_MT(rwres, Y)
    gv = timed_events(lambda: grad_vals(L, gB, X), 3, warm=1)
    plan.check()
    fo = timed_events(lambda: plan_o.solve(B), 3, warm=1)
    to = timed_events(lambda: plan_o.solve_transpose(G), 3, warm=1)
    plan_o.check()
    err = float(np.max(np.abs(X.cpu().numpy() - P["xs"])) / np.max(np.abs(P["xs"])))
    n, nnz, nnzp = L.n, L.nnz, rw.nnz
    Dp, D0 = plan.info["stats"]["num_levels"], info.num_levels
    adj = t + mt + gv
    kf = solve_kernel(plan.info["algo_fwd"], "double", False, k, plan.info["rhs_chunk"])
    kb = solve_kernel(plan.info["algo_bwd"], "double", True, k, plan.info["rhs_chunk"])
    return {"workload": f"power-law n={n}, nnz={nnz}, k={k} RHS column-major, 0.8% rows "
                        f"rewritten (thin-first whole levels), FP64",
            "levels_original": D0, "levels_rewritten": Dp, "nnz_rewritten": nnzp,
            "rewritten_rows": int(len(P["rows"])), "prepare_s": prep_s,
            "fwd_ms": f, "bwd_ms": t, "apply_MT_ms": mt, "grad_vals_ms": gv, "adjoint_ms": adj,
            "orig_fwd_ms": fo, "orig_bwd_ms": to,
            "speedup_rewritten_vs_original_fwd": fo / f,
            "speedup_rewritten_vs_original_fwd_adj": (fo + to) / (f + t),
            "solves_per_s_fwd": k / f * 1e3, "relerr_vs_xstar": err,
            "plan": {kk: plan.info[kk] for kk in ("algo_fwd", "block_rows", "rhs_chunk",
                                                  "lanes_per_row", "stage_outside",
                                                  "tuned_ms_level", "tuned_ms_syncfree",
                                                  "tuned_ms_walk", "chunk_rounds")},
            "plan_original": {kk: plan_o.info[kk] for kk in ("algo_fwd", "tuned_ms_syncfree",
                                                             "tuned_ms_walk", "chunk_rounds")},
            "roofline_fwd": roof(bytes_solve(n, nnzp, k, 8), f, kf, Dp, hop_ns),
            "roofline_bwd": roof(bytes_solve_t(n, nnzp, k, 8), t, kb, Dp, hop_ns),
            "adjoint_gbs": (bytes_solve_t(n, nnzp, k, 8) + bytes_apply_mt(n, k, 8, rw.nc)
                            + bytes_grad_vals(n, nnz, k, 8)) / adj / 1e6}


def run_autograd(args, dev, hop_ns):
    """torch.autograd.Function over the solve: forward on the thin-first 1%
    rewrite, backward = transposed solve, M^T and grad_vals, 32 RHS."""
    import numpy as np
    import torch

    import synth
    from paper_2609_40159_amd.autograd import TriangularSolve

    out = {}
    for name in ("lap3d_64", "powerlaw_262k"):
        spec = synth.WORKLOADS[name]
        k = spec["k"]
        P = prepare_system(spec, k, dev, torch.float64)
        L = P["L"]
        solver = TriangularSolve(L, P["rows"], P["targets"], kmax=k)
        vals = L.vals.clone().requires_grad_(True)
        Bt = P["B"].clone().requires_grad_(True)
        Gd = P["G"]

        def fwd():
            return solver(vals, Bt)

        def fwd_bwd():
            X = solver(vals, Bt)
            X.backward(Gd)
            return X

        f = timed_events(fwd, 5)
        fb = timed_events(fwd_bwd, 5)
        X = fwd()
        err = float(np.max(np.abs(X.detach().cpu().numpy() - P["xs"])) / np.max(np.abs(P["xs"])))
        n, nnz, nnzp = L.n, L.nnz, solver.rw.nnz
        info = solver.plan.info
        b_f = bytes_rewrite_numeric(n, nnz, nnzp, k, 8, solver.rw.nc) + bytes_solve(n, nnzp, k, 8)
        b_b = (bytes_solve_t(n, nnzp, k, 8) + bytes_apply_mt(n, k, 8, solver.rw.nc)
               + bytes_grad_vals(n, nnz, k, 8))
        out[name] = {"n": n, "nnz": nnz, "k": k, "levels_rewritten": info["stats"]["num_levels"],
                     "forward_ms": f, "backward_ms": fb - f, "fwd_bwd_ms": fb,
                     "forward_gbs": b_f / f / 1e6, "backward_gbs": b_b / (fb - f) / 1e6,
                     "relerr_vs_xstar": err, "algo": info["algo_fwd"],
                     "tuned_ms": {kk: info[kk] for kk in ("tuned_ms_level", "tuned_ms_syncfree",
                                                          "tuned_ms_walk", "chunk_rounds")},
                     "block_rows": info["block_rows"], "rhs_chunk": info["rhs_chunk"],
                     "bandwidth_floor_ms_fwd_bwd": (b_f + b_b) / (PEAK_HBM_GBS * 1e9) * 1e3,
                     "latency_floor_ms_fwd_bwd": (2 * info["stats"]["num_levels"] * hop_ns * 1e-6
                                                  if hop_ns else None)}
        del solver, vals, Bt, P
    return out


# ---------------------------------------------------------------------------
# the next rows on the 128^3 factor: generator, environment, L-then-U pair
# ---------------------------------------------------------------------------
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
    pcap = 48 * max(1, total) + (1 << 20)   # one-pass patterns
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




# ---------------------------------------------------------------------------
# Maskable PPO over the environment step (Section 4.5)
# ---------------------------------------------------------------------------
def run_ppo(args, dev):
    """Train the masked PPO policy on a deep power-law matrix (about 1,300
    levels, the size class of the paper's training matrices), then score
    its rewrite lists -- the best of five sampled episodes, as the paper's
    inference -- against an untrained policy, the thin-first rule with as
    many rewritten rows, and the fixed-policy generator: each list applied
    with the rewrite and scored by the analysis of L'."""
    import torch

    import synth
    from paper_2609_40159_amd import ppo
    from paper_2609_40159_amd.api import CSRMatrix, Env, Rewriter, analyze, generate

    Lh = synth.power_law(args.ppo_n, 11)
    L = CSRMatrix.from_arrays(Lh.rowptr, Lh.colidx, Lh.vals, device=dev)
    info = analyze(L)
    D0 = info.num_levels

    def score(rows, tg):
        if len(rows) == 0:
            return {"levels": D0, "cv": info.stats["cv"], "rows": 0}
        rw = Rewriter(L, info.level, rows, tg)
        rw.numeric()
        a = analyze(rw.Lp)
        return {"levels": a.num_levels, "cv": a.stats["cv"], "rows": int(len(rows))}

    def best_of(lists):
        sc = [dict(score(li["rows"], li["targets"]), moves=li["moves"], steps=li["steps"])
              for li in lists]
        return min(sc, key=lambda d: (d["levels"], d["cv"])), sc

    torch.manual_seed(0)
    pol = ppo.LevelPolicy().to(dev)
    env5 = Env(L, info, 5)
    untrained, _ = best_of(ppo.rollout_lists(env5, pol, seed=1))
    env = Env(L, info, args.ppo_envs)
    cfg = ppo.PPOConfig(updates=args.ppo_updates, time_limit_s=args.ppo_seconds, seed=0)
    tr = ppo.train(env, pol, cfg, log=lambda r: log(f"ppo update {r['update']}: "
                                                   f"{r['env_steps']} env steps, "
                                                   f"{r['elapsed_s']:.1f} s"))
    trained, runs = best_of(ppo.rollout_lists(env5, pol, seed=2))
    rows_tf, tg_tf = synth.thin_first_rows(info.level.cpu().numpy(),
                                           max(trained["rows"], 1) / Lh.n)
    thin_first = score(rows_tf, tg_tf)
    g = generate(L, info, [dict(max_dist=8, alpha=1.0, thin_stop=0.02)], cap=Lh.n)
    m = g.results[0]["moves"]
    gr, gt = ppo.final_rewrite_list(g.rows[0, :m].cpu().numpy(), g.tgt[0, :m].cpu().numpy())
    generator = score(gr, gt)
    last = tr["last"] or {}
    return {"matrix": f"power-law n={Lh.n}, nnz={Lh.nnz}, {D0} levels, CV {info.stats['cv']:.4f}",
            "envs": args.ppo_envs, "updates": tr["updates"], "env_steps": tr["env_steps"],
            "episodes": tr["episodes"], "train_s": tr["elapsed_s"],
            "train_env_steps_per_s": tr["env_steps"] / tr["elapsed_s"],
            "hyper": {"lr": cfg.lr, "n_steps": cfg.n_steps, "epochs": cfg.epochs,
                      "batch_size": cfg.batch_size, "clip": cfg.clip},
            "last_update": {k: last.get(k) for k in ("policy_loss", "value_loss", "entropy",
                                                    "approx_kl", "clip_fraction",
                                                    "explained_variance", "mean_episode_return")},
            "levels_original": D0, "cv_original": info.stats["cv"],
            "trained_best_of_5": trained, "trained_runs": runs, "untrained_best_of_5": untrained,
            "thin_first_same_rows": thin_first, "generator": generator}


def cpu_step128(args, ctx):
    """The 128^3 step on the oracle, single-threaded, for about cpu_seconds."""
    import oracle
    P = ctx["P"]
    Lh, n = P["Lh"], P["Lh"].n
    a = oracle.analyze(n, Lh.rowptr, Lh.colidx)
    reps, t_cpu = 0, 0.0
    t_start = time.perf_counter()
    while True:
        t1 = time.perf_counter()
        ro = oracle.rewrite(n, Lh.rowptr, Lh.colidx, Lh.vals, a.level, P["rows"], P["targets"],
                            P["Bh"])
        Xo = oracle.solve(n, ro.rowptr, ro.colidx, ro.vals, ro.Bp)
        oracle.adjoint(n, Lh.rowptr, Lh.colidx, Lh.vals, Xo, P["Gh"])
        t_cpu += time.perf_counter() - t1
        reps += 1
        if time.perf_counter() - t_start > args.cpu_seconds or reps >= 500:
            break
    return {"value": ctx["b_step"] * reps / t_cpu / 1e9, "unit": "GB/s", "cores": 1,
            "kind": "oracle", "ms_per_step": t_cpu / reps * 1e3, "cpu_model": cpu_model(),
            "sample": f"{reps} full 128^3 steps (rewrite, forward solve, adjoint), "
                      f"single-threaded FP64 oracle"}, a


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

    secs = set(args.sections)
    # batched workload inputs: generated first, in forked host processes,
    # before anything touches the GPU
    man = gen = None
    gen_s = 0.0
    if "batch" in secs:
        t0 = time.perf_counter()
        man = synth.batch_manifest(count=args.batch_count)
        gen = synth.build_batch(man, args.gen_workers)
        gen_s = time.perf_counter() - t0
        log(f"batch inputs generated in {gen_s:.1f} s")

    from paper_2609_40159_amd import _lib
    from paper_2609_40159_amd.api import probe_handoff

    _lib.load()   # fails loudly without the HIP library
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    dev = "cuda:0"
    torch.cuda.set_device(0)

    # one cross-workgroup hand-off (the latency floor's unit), and the
    # device's copy rate (a reference for the roofline and the counters)
    hop_ns = probe_handoff(2000)
    a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    b2 = torch.empty_like(a)
    a.fill_(1.0)
    copy_ms = timed_events(lambda: b2.copy_(a), 5)
    copy_probe = {"bytes_each": 2 * a.numel() * 8, "ms_each": copy_ms}
    del a, b2

    out = {"metric": METRIC, "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic"}
    batched = head = cpu_in = None
    if "batch" in secs:
        batched, head, cpu_in = run_batched(args, man, gen, dev, hop_ns)
        batched["host_generation_s"] = gen_s
    step128 = ctx = None
    if secs & {"step128", "generator", "pair", "env"} or head is None:
        steps = args.step128_steps if head is not None else args.steps
        step128, ctx = run_step128(args, dev, torch.float64, hop_ns, steps)
        log("128^3 step timed")
    extras = {}
    if "fp32" in secs:
        extras["fp32"] = run_fp32(args, dev, hop_ns)
        log("128^3 FP32 timed")
    if "powerlaw1m" in secs:
        extras["powerlaw1m"] = run_powerlaw1m(args, dev, hop_ns)
        log("power-law 1M x 64 timed")
    if "autograd" in secs:
        extras["autograd"] = run_autograd(args, dev, hop_ns)
        log("autograd workloads timed")
    if "ppo" in secs:
        extras["ppo"] = run_ppo(args, dev)
        log("PPO trained and scored")
    generator = gen_cmp = pair = pair_cmp = envres = None
    if ctx is not None:
        P = ctx["P"]
        if "generator" in secs:
            generator, gen_cmp = run_generator(args, P["L"], P["Lh"], P["info"], dev)
        if "pair" in secs:
            pair, pair_cmp = run_pair(args, P["L"], P["Lh"], dev, 1, ctx["plan"], ctx["rwres"])
        if "env" in secs:
            envres = run_env(args, P["L"], P["info"], dev)
            log("environment steps timed")

    # ---------------- CPU oracle baseline ----------------
    cpu = None
    if not args.no_cpu:
        import oracle
        if head is not None:
            cpu = cpu_batched(args, man, gen, cpu_in)
            log("batched oracle baseline timed")
        if ctx is not None:
            c128, a = cpu_step128(args, ctx)
            if cpu is None:
                cpu = c128
            else:
                cpu["step128"] = c128
            P = ctx["P"]
            Lh, n = P["Lh"], P["Lh"].n
            if gen_cmp is not None:
                t_or, steps_or, same = 0.0, 0, True
                for q, prm in enumerate(gen_cmp["params"]):
                    t1 = time.perf_counter()
                    o = oracle.generate(n, Lh.rowptr, gen_cmp["level"], gen_cmp["D"],
                                        gen_cmp["alc"], gen_cmp["cv"], cap=gen_cmp["cap"], **prm)
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
                rng = np.random.default_rng(7)
                oe = oracle.Env(n, Lh.rowptr, a.level, a.num_levels, a.alc, a.cv,
                                cap=4 * args.env_steps)
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

    # ---------------- the headline line ----------------
    if head is not None:
        K = head["steps"]
        tr = load_traffic("batch256:f64:k_batch_main", src_hash(BATCH_SOURCES), "n/a", 0)
        roofline = roof(head["step_bytes"], head["main_ms"], "k_batch_main", batched["max_levels"],
                        hop_ns, tr)
        roofline["note"] = ("persistent kernel of the batched launch: all solves and all candidate "
                            "level analyses; algorithmic bytes = solve bytes + candidate bytes")
        out.update({
            "value": head["step_bytes"] * K / head["elapsed_s"] / 1e9, "unit": "GB/s",
            "steps": K, "warmup": args.warmup, "ms_per_step": head["elapsed_s"] / K * 1e3,
            "config": {"workload": f"batched: {batched['matrices']} matrices n~U[2k,200k] (a "
                                   f"quarter 2D and a quarter 3D Laplacian factors, half "
                                   f"power-law), {batched['rhs_total']} RHS (1-16 each), "
                                   f"{batched['candidates']} candidate rewrite sets (32 each, "
                                   f"0.5-1.5% of rows), one setup + one persistent launch per step",
                       "n_total": batched["n_total"], "nnz_total": batched["nnz_total"],
                       "rhs_total": batched["rhs_total"], "candidates": batched["candidates"],
                       "max_levels": batched["max_levels"], "parallelism": "single GPU"},
            "solves_per_s": batched["rhs_total"] * K / head["elapsed_s"],
            "candidates_per_s": batched["candidates"] * K / head["elapsed_s"],
            "roofline": roofline, "batched": batched})
    else:
        K = step128["steps"]
        rf = step128["roofline_fwd"] if step128["step_phase_ms"]["fwd"] >= \
            step128["step_phase_ms"]["bwd"] else step128["roofline_bwd"]
        out.update({
            "value": step128["gbs"], "unit": "GB/s", "steps": K, "warmup": 3,
            "ms_per_step": step128["ms_per_step"],
            "config": {"workload": "step128: " + step128["workload"], "n": step128["n"],
                       "nnz": step128["nnz"], "parallelism": "single GPU"},
            "solves_per_s": 1e3 / step128["ms_per_step"], "roofline": rf})
    out["step128"] = step128
    out.update(extras)
    out["generator"] = generator
    out["pair"] = pair
    out["env"] = envres
    out["cpu_baseline"] = cpu
    out["copy_probe"] = copy_probe
    out["stream_copy_gbs"] = copy_probe["bytes_each"] / (copy_ms * 1e-3) / 1e9
    out["handoff_ns"] = hop_ns
    print(json.dumps(out))


if __name__ == "__main__":
    main()
