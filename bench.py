"""Benchmark of the fast directional Helmholtz matvec on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload uniform1m]

One step is one full matvec (Alg. 4: S2M, M2M, M2L, L2L, L2T, near field)
of the mixed-precision plan (FP32 coupling step on the matrix cores, FP64
everywhere else) on the workload's synthetic input, already resident in HBM.
The plain FP64 plan is timed beside it for the speedup, and the relative l2
error against the FP64 oracle is taken on the stored oracle rows of the
workload.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "matvecs/s at N=1e6 mixed vs FP64 plain; rel l2 err vs FP64 oracle"
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6, "bf16x3": 2500.0}
M2L_KERNEL = {"fp32": "k_m2l_f32", "fp64": "k_m2l_f64", "bf16x3": "k_m2l_bf16x3"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="uniform1m")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16x3"])
    ap.add_argument("--plain-steps", type=int, default=1,
                    help="timed steps of the plain FP64 plan (0 = skip)")
    ap.add_argument("--bf16-steps", type=int, default=1,
                    help="timed steps of the BF16 split (bf16x3) plan (0 = skip)")
    ap.add_argument("--batch-steps", type=int, default=2,
                    help="timed batched matvecs of the 64-problem workload (0 = skip)")
    ap.add_argument("--bank-budget-gb", type=float, default=0.0,
                    help="> 0: generate the coupling bank during each matvec into a "
                         "workspace of this many GB (for banks that do not fit)")
    ap.add_argument("--compact", type=int, default=1, choices=[0, 1, 2],
                    help="FP32 column compaction: 0 never, 1 sparse levels, 2 every level")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device to device (calibrates HBM byte counters)")
    ap.add_argument("--cpu-groups", type=int, default=40)
    return ap.parse_args()


def describe(P) -> str:
    return (f"{P.name}: N_T={P.points_T.shape[0]} N_S={P.points_S.shape[0]} uniform in "
            f"(0,1]^3, kappa={P.kappa:g}, {P.levels} levels, m={P.m} "
            f"(K={(P.m + 1) ** 3}), complex128 v with N(0,1) parts")


def time_plan(plan, v, y, steps, warmup, tag=""):
    """Warmup and timed matvecs; the launch schedule (and a streamed bank's
    workspace) is built before.  Matvecs with several coupling launches
    report each launch as it completes."""
    import torch
    plan.set_timing(True)
    plan.prepare()
    n_launch = plan.coupling_launches()
    for _ in range(warmup):
        plan.matvec(v, out=y)
    torch.cuda.synchronize()
    phases = []
    t0 = time.perf_counter()
    for k in range(steps):
        plan.matvec(v, out=y)
        if n_launch > 1:
            for i in range(n_launch):
                ms = plan.wait_launch(i)
                print(f"[bench] {tag} step {k + 1}/{steps}: coupling launch {i + 1}/{n_launch} "
                      f"done at {ms / 1000:.1f} s", file=sys.stderr, flush=True)
        phases.append(plan.phase_ms())  # waits for this step's events
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, phases


def plan_shape(plan, levels: int, l_min: int) -> dict:
    """Boxes per level of both trees and directions per level (plan export)."""
    nbS = [int(plan.export(f"keys_S{l}").shape[0]) for l in range(levels + 1)]
    nbT = [int(plan.export(f"keys_T{l}").shape[0]) for l in range(levels + 1)]
    nd = [int(plan.export(f"dirs_{l}").shape[0]) if l >= l_min else 1 for l in range(levels + 1)]
    return {"nbS": nbS, "nbT": nbT, "nd": nd, "levels": levels, "l_min": l_min}


def hbm_phases(shape: dict, phase_ms: dict, K: int, nT: int, nS: int, mixed: bool) -> dict:
    """Compulsory HBM bytes of the transfer phases (each array read or written
    once; 16-byte complex FP64 vectors of Kp entries per (box, direction),
    plus the 8-byte FP32 copy of the moments in the mixed precisions) and the
    rate they imply at the measured phase times, against 8 TB/s."""
    Kp = (K + 31) // 32 * 32
    p, lm = shape["levels"], shape["l_min"]
    nbS, nbT, nd = shape["nbS"], shape["nbT"], shape["nd"]
    vec = Kp * 16
    mom_w = vec + (Kp * 8 if mixed else 0)
    b = {}
    # permute in + S2M: v read and written, points and tree-order v read, leaf moments written
    b["s2m"] = 16 * nS * 2 + (24 + 16) * nS + nbS[p] * nd[p] * mom_w if lm <= p else 0
    # M2M: child moments read, parent moments written
    b["m2m"] = sum(nbS[l + 1] * nd[l + 1] * vec + nbS[l] * nd[l] * mom_w for l in range(lm, p))
    # L2L: parent locals read, child locals read and written (completed in place)
    b["l2l"] = sum(nbT[l] * nd[l] * vec + nbT[l + 1] * nd[l + 1] * 2 * vec for l in range(lm, p))
    # L2T: leaf locals and points read, y read and written
    b["l2t"] = (nbT[p] * nd[p] * vec if lm <= p else 0) + 24 * nT + 32 * nT
    # near field: target and source points, tree-order v read, y written
    b["near"] = 24 * nT + 40 * nS + 16 * nT
    out = {}
    for k, v in b.items():
        ms = phase_ms.get(k, 0.0)
        rate = v / (ms * 1e-3) / 1e9 if ms > 0.01 else None  # empty phase: no rate
        out[k] = {"bytes": v, "ms": ms, "GB/s": rate,
                  "frac_of_8TB/s": (rate / 8000.0) if rate else None}
    return out


def kernel_source_sha(kernel: str) -> str:
    """SHA-256 of the sources that define a coupling kernel (shared device
    code + its precision's file)."""
    csrc = os.path.join(ROOT, "paper_2004_14229_amd", "csrc")
    part = {"k_m2l_f32": "m2l_f32.hip", "k_m2l_f64": "m2l_f64.hip",
            "k_m2l_bf16x3": "m2l_bf16.hip"}[kernel]
    h = hashlib.sha256()
    for f in ("m2l_device.hpp", part):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


def traffic_for(kernel: str, workload: str, launch_flops: float):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if
    they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != kernel_source_sha(kernel):
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(P, stats, groups: int, seed: int = 7):
    """The oracle's coupling step (its Alg. 4 M2L: one coupling matrix per
    level and offset applied to all blocks of that offset), timed on a seeded
    sample of (level, offset) groups with their full block lists, then scaled
    to a whole matvec as N_SC * (matrix time) + N_C * (time per block)."""
    import oracle
    from oracle.fdmvm import apply_coupling
    from oracle.interpolation import coupling_matrix
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    rng = np.random.default_rng(seed)
    TT = oracle.build_box_tree(P.points_T, P.box, P.levels)
    TS = oracle.build_box_tree(P.points_S, P.box, P.levels)
    side = P.box[3] - P.box[0]
    l_hf = oracle.high_frequency_level(P.kappa, side, P.levels)
    dirs = oracle.DirectionSets(l_hf, P.levels)
    level = P.levels - 1  # the level with the most blocks at this workload
    h = TT.side(level)
    # admissible offsets of the level whose parent offset is inadmissible
    R = 2 ** level - 1
    r = np.arange(-R, R + 1)
    cand = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    cand = cand[oracle.admissible(P.kappa, h, cand)]
    par = -((-cand) // 2)  # ceil(o / 2): parent offset for target octant 0
    cand = cand[~oracle.admissible(P.kappa, TT.side(level - 1), par)]
    groups = min(groups, cand.shape[0])
    pick = cand[rng.choice(cand.shape[0], groups, replace=False)]
    src_index = {tuple(c): i for i, c in enumerate(TS.coords[level])}
    t_mat, t_all, n_blocks = [], [], 0
    K = (P.m + 1) ** 3
    start = time.perf_counter()
    for o in pick:
        tc = TT.coords[level]
        octant0 = np.all(tc % 2 == 0, axis=1)  # targets whose parent pair was refined
        srcs = [src_index.get(tuple(x)) for x in (tc[octant0] - o)]
        n = sum(1 for s in srcs if s is not None)
        c = dirs.vectors(level)[int(dirs.dir_index(level, o))]
        M = rng.standard_normal((n, K)) + 1j * rng.standard_normal((n, K))
        t0 = time.perf_counter()
        coupling_matrix(P.m, h, o, P.kappa, c)
        t1 = time.perf_counter()
        apply_coupling(P.m, h, o, P.kappa, c, M)
        t2 = time.perf_counter()
        t_mat.append(t1 - t0)
        t_all.append(t2 - t1)
        n_blocks += n
    sample_s = time.perf_counter() - start
    per_matrix = float(np.mean(t_mat))
    # apply_coupling forms the matrix again: its time, measured apart, is
    # taken off (never below zero, which timer noise allows on tiny samples)
    per_block = max(sum(t_all) - sum(t_mat), 0.0) / max(n_blocks, 1)
    t_full = stats["n_stored_couplings"] * per_matrix + stats["n_couplings"] * per_block
    return {"value": 1.0 / t_full, "unit": "matvecs/s", "cores": int(cores), "kind": "oracle",
            "sample": (f"oracle coupling step (the >99% of Alg. 4's arithmetic here) on "
                       f"{groups} seeded level-{level} offset groups, {n_blocks} blocks, "
                       f"{sample_s:.1f} s; scaled to N_SC={stats['n_stored_couplings']} "
                       f"matrices + N_C={stats['n_couplings']} blocks = {t_full:.0f} s "
                       f"per matvec (S2M/M2M/L2L/L2T/near field not counted)")}


def batched(steps: int, compact: int = 1) -> dict:
    """The batched workload: 64 independent problems (N log-uniform in
    [1e4, 2e5], kappa uniform in [10, 80], half uniform, half clustered, m=5,
    complex64 v) in one batch: mixed FP32 coupling, banks generated into the
    batch's workspace during each matvec, coupling and near-field work of all
    problems from one device queue, the whole batched matvec replayed as a
    HIP graph, launch shape picked by the autotuner."""
    import torch
    import paper_2004_14229_amd as F
    import workloads as W
    probs = W.batch_problems()
    t0 = time.perf_counter()
    plans = []
    for Q in probs:
        qt = torch.from_numpy(Q.points_T).cuda()
        qs = torch.from_numpy(Q.points_S).cuda()
        plans.append(F.Plan(qt, qs, Q.kappa, Q.box, Q.levels, Q.m, precision="fp32",
                            bank_budget=1 << 30, tune={"compact": compact}))
        del qt, qs
    b = F.Batch(plans)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    vs = [torch.from_numpy(Q.v.astype(np.complex64)).cuda() for Q in probs]
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        best, tune_ms, ys = b.autotune(vs, max_candidates=4, stream=stream)
        b.matvec(vs, ys, stream=stream)  # graph capture + first replay
    stream.synchronize()
    t1 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(steps):
            b.matvec(vs, ys, stream=stream)
    stream.synchronize()
    wall = (time.perf_counter() - t1) / steps
    K = (probs[0].m + 1) ** 3
    stats = [p.stats() for p in plans]
    flops = sum(8.0 * K * K * st["n_couplings"] for st in stats)
    res = {"workload": ("64 problems, N log-uniform in [1e4, 2e5] (sum %d), kappa U[10,80], "
                        "32 uniform + 32 clustered (8 blobs, sigma 0.05), 4-5 levels, m=5, "
                        "complex64 v and y" % sum(Q.points_T.shape[0] for Q in probs)),
           "value": 1.0 / wall, "unit": "batches/s", "problem_matvecs_per_s": 64.0 / wall,
           "ms_per_batch": 1000.0 * wall, "steps": steps, "setup_s": setup_s,
           "precision": "FP32 coupling, banks generated per matvec into the batch workspace",
           "tune": best, "autotune_m2l_ms": tune_ms,
           "m2l_flops": flops, "tflops_whole_batch": flops / wall / 1e12}
    golden = os.path.join(ROOT, "tests", "golden", "batch_rows.npz")
    if os.path.exists(golden):
        g = np.load(golden)
        errs, num, den = {}, 0.0, 0.0
        for key in g.files:
            if not key.startswith("rows"):
                continue
            i = int(key[4:])
            yy = ys[i].cpu().numpy().astype(np.complex128)[g[key]]
            yo = g[f"y{i}"]
            errs[str(i)] = float(np.linalg.norm(yy - yo) / np.linalg.norm(yo))
            num += float(np.linalg.norm(yy - yo) ** 2)
            den += float(np.linalg.norm(yo) ** 2)
        res["rel_l2_err_vs_oracle"] = errs
        res["rel_l2_err_vs_oracle_pooled"] = (num / den) ** 0.5
    b.close()
    for p in plans:
        p.close()
    print(f"[bench] batched: {1000.0 * wall:.1f} ms per batch of 64", file=sys.stderr, flush=True)
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "sharding of this method is a design note, not built", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2004_14229_amd as F
    import workloads as W

    if args.copy_probe:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 4}))
        return

    P = W.config(args.workload)
    dev = torch.device("cuda:0")
    pt = torch.from_numpy(P.points_T).to(dev)
    ps = torch.from_numpy(P.points_S).to(dev)
    v = torch.from_numpy(P.v).to(dev)
    y = torch.empty(P.points_T.shape[0], dtype=torch.complex128, device=dev)

    t0 = time.perf_counter()
    budget = int(args.bank_budget_gb * 1e9)
    plan = F.Plan(pt, ps, P.kappa, P.box, P.levels, P.m, precision=args.precision,
                  bank_budget=budget, tune={"compact": args.compact})
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    stats = plan.stats()
    print(f"[bench] {args.precision} plan built in {setup_s:.1f} s: N_C={stats['n_couplings']} "
          f"N_SC={stats['n_stored_couplings']}", file=sys.stderr, flush=True)
    shape = plan_shape(plan, P.levels, stats["l_min"])
    wall, phases = time_plan(plan, v, y, args.steps, args.warmup, args.precision)
    y_mixed = y.cpu().numpy()
    plan.close()
    del plan
    ms_per_step = 1000.0 * wall / args.steps
    m2l_ms = float(np.mean([p["m2l"] for p in phases]))
    K = (P.m + 1) ** 3
    flops = 8.0 * K * K * stats["n_couplings"]
    achieved = flops / (m2l_ms * 1e-3) / 1e12
    print(f"[bench] {args.precision}: {ms_per_step:.1f} ms/matvec, M2L {m2l_ms:.1f} ms",
          file=sys.stderr, flush=True)

    out = {"metric": METRIC, "value": 1000.0 / ms_per_step, "unit": "matvecs/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None,
           "dtype": {"fp32": "f32", "fp64": "f64", "bf16x3": "bf16"}[args.precision],
           "data": "synthetic",
           "config": {"workload": describe(P),
                      "precision": {
                          "fp32": "FP32 coupling products on MFMA, FP64 phases, transfers, "
                                  "near field and sums into y",
                          "bf16x3": "BF16 hi/lo split coupling products (3 per real "
                                    "product) on MFMA with FP32 sums, FP64 elsewhere",
                          "fp64": "FP64 throughout"}[args.precision]}}
    out["roofline"] = {"bound": "mfma", "kernel": M2L_KERNEL[args.precision],
                       "achieved": achieved, "peak": PEAK_TFLOPS[args.precision],
                       "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[args.precision],
                       "traffic": traffic_for(M2L_KERNEL[args.precision], args.workload, flops),
                       "flops_per_launch": flops, "avg_launch_ms": m2l_ms}
    out["phase_ms"] = {k: float(np.mean([p[k] for p in phases])) for k in phases[0]}
    out["hbm_phases"] = hbm_phases(shape, out["phase_ms"], (P.m + 1) ** 3, P.points_T.shape[0],
                                   P.points_S.shape[0], args.precision != "fp64")
    out["setup_s"] = setup_s
    out["plan"] = {k: stats[k] for k in ("n_couplings", "n_stored_couplings", "m2l_columns",
                                         "near_entries", "device_bytes", "l_hf", "l_min")}
    out["plan"]["bank"] = (f"generated per matvec into a {args.bank_budget_gb:g} GB workspace"
                           if budget else "resident")

    golden = os.path.join(ROOT, "tests", "golden", f"{args.workload}_rows.npz")
    if os.path.exists(golden):
        g = np.load(golden)
        rows, yo = g["rows"], g["y"]
        out["rel_l2_err_vs_oracle"] = float(np.linalg.norm(y_mixed[rows] - yo) / np.linalg.norm(yo))
        out["oracle_rows"] = int(rows.shape[0])

    y_plain = None
    if args.plain_steps > 0 and args.precision != "fp64":
        plain = F.Plan(pt, ps, P.kappa, P.box, P.levels, P.m, precision="fp64",
                       bank_budget=budget)
        pwall, pph = time_plan(plain, v, y, args.plain_steps, min(args.warmup, 1), "fp64")
        y_plain = y.cpu().numpy()
        plain.close()
        del plain
        pms = 1000.0 * pwall / args.plain_steps
        pm2l = float(np.mean([p["m2l"] for p in pph]))
        out["plain_fp64"] = {"value": 1000.0 / pms, "ms_per_step": pms, "steps": args.plain_steps,
                             "m2l_ms": pm2l, "m2l_tflops": flops / (pm2l * 1e-3) / 1e12}
        out["speedup_vs_plain"] = pms / ms_per_step
        out["rel_l2_err_vs_plain_gpu"] = float(np.linalg.norm(y_mixed - y_plain) /
                                               np.linalg.norm(y_plain))
        if os.path.exists(golden):
            out["plain_fp64"]["rel_l2_err_vs_oracle"] = float(
                np.linalg.norm(y_plain[rows] - yo) / np.linalg.norm(yo))
        print(f"[bench] fp64 plain: {pms:.1f} ms/matvec", file=sys.stderr, flush=True)

    if args.bf16_steps > 0 and args.precision != "bf16x3":
        bf = F.Plan(pt, ps, P.kappa, P.box, P.levels, P.m, precision="bf16x3",
                    bank_budget=budget)
        bwall, bph = time_plan(bf, v, y, args.bf16_steps, min(args.warmup, 1), "bf16x3")
        y_bf = y.cpu().numpy()
        bf.close()
        del bf
        bms = 1000.0 * bwall / args.bf16_steps
        bm2l = float(np.mean([p["m2l"] for p in bph]))
        alg = flops / (bm2l * 1e-3) / 1e12
        out["bf16x3"] = {"value": 1000.0 / bms, "ms_per_step": bms, "steps": args.bf16_steps,
                         "m2l_ms": bm2l, "m2l_tflops_algorithmic": alg,
                         "m2l_tflops_issued": 3.0 * alg,
                         "frac_of_bf16_peak_issued": 3.0 * alg / PEAK_TFLOPS["bf16x3"],
                         "speedup_vs_mixed": ms_per_step / bms}
        if os.path.exists(golden):
            g = np.load(golden)
            out["bf16x3"]["rel_l2_err_vs_oracle"] = float(
                np.linalg.norm(y_bf[rows] - yo) / np.linalg.norm(yo))
            if "y_bf16x3" in g.files:
                out["bf16x3"]["emulated_rel_l2_err"] = float(
                    np.linalg.norm(g["y_bf16x3"] - yo) / np.linalg.norm(yo))
        if y_plain is not None:
            out["bf16x3"]["rel_l2_err_vs_plain_gpu"] = float(
                np.linalg.norm(y_bf - y_plain) / np.linalg.norm(y_plain))
        print(f"[bench] bf16x3: {bms:.1f} ms/matvec, M2L {bm2l:.1f} ms", file=sys.stderr,
              flush=True)

    if args.batch_steps > 0:
        del pt, ps, v, y
        torch.cuda.empty_cache()
        out["batched"] = batched(args.batch_steps, args.compact)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(P, stats, args.cpu_groups)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
