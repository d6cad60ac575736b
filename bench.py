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
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6, "bf16x3": 2500.0, "bf16x6": 2500.0}
M2L_KERNEL = {"fp32": "k_m2l_f32", "fp64": "k_m2l_f64", "bf16x3": "k_m2l_bf16x3",
              "bf16x6": "k_m2l_bf16x6"}
SPLIT_PRODUCTS = {"bf16x3": 3, "bf16x6": 6}  # BF16 products issued per real product


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="uniform1m")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16x3", "bf16x6"])
    ap.add_argument("--plain-steps", type=int, default=1,
                    help="timed steps of the plain FP64 plan (0 = skip)")
    ap.add_argument("--bf16-steps", type=int, default=1,
                    help="timed steps of each BF16 split plan (bf16x3, bf16x6; 0 = skip)")
    ap.add_argument("--aca-eps", type=float, default=1e-7,
                    help="tolerance of the low-rank (ACA) coupling leg, FP32 (0 = skip)")
    ap.add_argument("--aca-steps", type=int, default=1,
                    help="timed steps of the low-rank coupling plan")
    ap.add_argument("--batch-steps", type=int, default=2,
                    help="timed batched matvecs of the 64-problem workload (0 = skip)")
    ap.add_argument("--batch-adaptive-n-max", type=int, default=0,
                    help="> 0: also time the batched workload with its clustered half on "
                         "adaptive trees of at most this many points per leaf")
    ap.add_argument("--bank-budget-gb", type=float, default=0.0,
                    help="> 0: generate the coupling bank during each matvec into a "
                         "workspace of this many GB (for banks that do not fit)")
    ap.add_argument("--resident-main", action="store_true",
                    help="keep the timed plan's bank resident even with --bank-budget-gb "
                         "(the other legs still stream theirs)")
    ap.add_argument("--compact", type=int, default=1, choices=[0, 1, 2],
                    help="FP32 column compaction: 0 never, 1 sparse levels, 2 every level")
    ap.add_argument("--nb", type=int, default=None, choices=[32, 64],
                    help="target boxes per coupling work item of the timed plan "
                         "(default: the library's for the precision)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device to device (calibrates HBM byte counters)")
    ap.add_argument("--cpu-sub", type=int, default=4,
                    help="CPU baseline sample: the sub-cube of side 1/cpu-sub of the box")
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
            "k_m2l_bf16x3": "m2l_bf16.hip", "k_m2l_bf16x6": "m2l_bf16x6.hip"}[kernel]
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


def cpu_baseline(P, stats, shape, sub_div: int = 4):
    """The oracle's whole Alg. 4 (S2M, M2M, M2L, L2L, L2T, near field, in the
    oracle's own code) timed on a bounded sample of the workload: the points
    of the workload inside the sub-cube (0, 1/sub_div]^3 with their charges,
    the same kappa, m and leaf size (levels - log2(sub_div)), so that every
    box size of the workload's coupling levels occurs with the same
    direction counts.  Each phase's time is scaled to the whole workload by
    its own work count (points for S2M and L2T, box-directions for M2M and
    L2L, stored matrices and admissible blocks for M2L, point pairs for the
    near field): measured on the sample, extrapolated per phase."""
    import oracle
    from oracle.interpolation import coupling_matrix
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    lo = np.asarray(P.box[:3])
    side = P.box[3] - P.box[0]
    sub_side = side / sub_div
    hi = lo + sub_side
    inT = np.all((P.points_T > lo) & (P.points_T <= hi), axis=1)
    inS = np.all((P.points_S > lo) & (P.points_S <= hi), axis=1)
    levels = P.levels - int(round(np.log2(sub_div)))
    box = tuple(lo) + tuple(hi)
    t0 = time.perf_counter()
    plan = oracle.build(P.points_T[inT], P.points_S[inS], P.kappa, box, levels, P.m)
    build_s = time.perf_counter() - t0
    oracle.matvec(plan, P.v[inS])
    tm = dict(plan.timings)
    st = oracle.structure(plan)
    nc_sub = sum(int(st[f"nc{l}"][0]) for l in range(levels + 1))
    nsc_sub = sum(int(st[f"off{l}"].shape[0]) for l in range(levels + 1))
    # time of one coupling matrix (its K^2 kernel evaluations), apart from the products
    l_hf = plan.l_hf
    lv = max(l for l in range(levels + 1) if int(st[f"nc{l}"][0]) > 0)
    offs = st[f"off{lv}"][:8]
    dirs = oracle.DirectionSets(l_hf, levels)
    t1 = time.perf_counter()
    for o in offs:
        coupling_matrix(P.m, plan.side(lv), o, P.kappa,
                        dirs.vectors(lv)[int(dirs.dir_index(lv, o))])
    per_matrix = (time.perf_counter() - t1) / max(len(offs), 1)
    per_block = max(tm["m2l"] - nsc_sub * per_matrix, 0.0) / max(nc_sub, 1)
    # work counts: sample (oracle plan) and whole workload (GPU plan)
    off = P.levels - levels
    nbS_sub = [int(plan.TS.keys[l].shape[0]) for l in range(levels + 1)]
    nbT_sub = [int(plan.TT.keys[l].shape[0]) for l in range(levels + 1)]
    nd_full = shape["nd"]
    lm = shape["l_min"]

    def boxdirs(nb, lvl_of, first, last):
        return sum(nb[l] * nd_full[lvl_of(l)] for l in range(first, last))

    sub = {"s2m": int(inS.sum()), "l2t": int(inT.sum()),
           "m2m": boxdirs(nbS_sub, lambda l: l + off, max(lm - off, 0), levels),
           "l2l": boxdirs(nbT_sub, lambda l: l + off, max(lm - off, 0), levels),
           "near": int(st["near_entries"][0])}
    full = {"s2m": int(P.points_S.shape[0]), "l2t": int(P.points_T.shape[0]),
            "m2m": boxdirs(shape["nbS"], lambda l: l, lm, P.levels),
            "l2l": boxdirs(shape["nbT"], lambda l: l, lm, P.levels),
            "near": int(stats["near_entries"])}
    phases = {}
    for k in ("s2m", "m2m", "l2l", "l2t", "near"):
        phases[k] = {"sample_s": tm[k], "sample_units": sub[k], "full_units": full[k],
                     "extrapolated_s": tm[k] * full[k] / max(sub[k], 1)}
    m2l_full = stats["n_stored_couplings"] * per_matrix + stats["n_couplings"] * per_block
    phases["m2l"] = {"sample_s": tm["m2l"], "sample_blocks": nc_sub, "sample_matrices": nsc_sub,
                     "s_per_matrix": per_matrix, "s_per_block": per_block,
                     "full_blocks": int(stats["n_couplings"]),
                     "full_matrices": int(stats["n_stored_couplings"]),
                     "extrapolated_s": m2l_full}
    total = sum(ph["extrapolated_s"] for ph in phases.values())
    return {"value": 1.0 / total, "unit": "matvecs/s", "cores": int(cores), "kind": "oracle",
            "sample": (f"oracle Alg. 4 run whole on the workload's points in the sub-cube "
                       f"(0,{sub_side:g}]^3 ({int(inT.sum())} targets, {int(inS.sum())} "
                       f"sources, {levels} levels: the same kappa, m and box sizes), "
                       f"{tm['total']:.1f} s measured (+{build_s:.1f} s set-up); each phase "
                       f"scaled by its work count to the whole workload: {total:.0f} s per "
                       f"matvec"),
            "measured_s": tm["total"], "extrapolated_s_per_matvec": total, "phases": phases}


def batched(steps: int, compact: int = 1, aca_eps: float = 0.0, n_max: int = 0) -> dict:
    """The batched workload: 64 independent problems (N log-uniform in
    [1e4, 2e5], kappa uniform in [10, 80], half uniform, half clustered, m=5,
    complex64 v) in one batch: mixed FP32 coupling, every problem's bank
    resident (one matrix per offset pair), coupling and near-field work of
    all problems from one device queue in one persistent launch, the whole
    batched matvec replayed as a HIP graph, launch shape picked by the
    autotuner.  aca_eps > 0: every coupling matrix compressed by ACA (low-rank
    launch pairs over all problems' offset groups, near field apart).
    n_max > 0: the clustered half on adaptive trees (Alg. 1 with at most
    n_max points per leaf above the last level; near field apart)."""
    import torch
    import paper_2004_14229_amd as F
    import workloads as W
    probs = W.batch_problems()
    t0 = time.perf_counter()
    plans = []
    adaptive = [n_max > 0 and Q.meta.get("kind") == "clustered" for Q in probs]
    for Q, ad in zip(probs, adaptive):
        qt = torch.from_numpy(Q.points_T).cuda()
        qs = torch.from_numpy(Q.points_S).cuda()
        plans.append(F.Plan(qt, qs, Q.kappa, Q.box, Q.levels, Q.m, precision="fp32",
                            n_max=n_max if ad else 0,
                            **({"aca_eps": aca_eps} if aca_eps > 0 else
                               {"tune": {"compact": compact}})))
        del qt, qs
    b = F.Batch(plans)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    vs = [torch.from_numpy(Q.v.astype(np.complex64)).cuda() for Q in probs]
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        # launch shapes, then (dense couplings) the two other compaction modes
        best, tune_ms, ys = b.autotune(vs, max_candidates=4 if aca_eps > 0 else 6,
                                       stream=stream)
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
    if aca_eps > 0:  # the low-rank products' own flops
        flops = sum(st["aca_flops"] for st in stats)
    res = {"workload": ("64 problems, N log-uniform in [1e4, 2e5] (sum %d), kappa U[10,80], "
                        "32 uniform + 32 clustered (8 blobs, sigma 0.05), 4-5 levels, m=5, "
                        "complex64 v and y" % sum(Q.points_T.shape[0] for Q in probs)),
           "value": 1.0 / wall, "unit": "batches/s", "problem_matvecs_per_s": 64.0 / wall,
           "ms_per_batch": 1000.0 * wall, "steps": steps, "setup_s": setup_s,
           "precision": ("FP32 coupling, resident banks (one matrix per offset pair)"
                         if aca_eps <= 0 else
                         f"FP32 low-rank coupling (ACA to {aca_eps:g}), resident low-rank banks"),
           "bank_matrices": sum(st["n_bank_matrices"] for st in stats),
           "device_bytes": sum(st["device_bytes"] for st in stats),
           "tune": best, "autotune_m2l_ms": tune_ms,
           "m2l_flops": flops, "tflops_whole_batch": flops / wall / 1e12}
    if n_max > 0:
        res["adaptive"] = (f"clustered half on adaptive trees, n_max = {n_max}; oracle rows "
                           "compared for uniform-tree problems only")
    golden = os.path.join(ROOT, "tests", "golden", "batch_rows.npz")
    if os.path.exists(golden):
        g = np.load(golden)
        errs, num, den = {}, 0.0, 0.0
        for key in g.files:
            if not key.startswith("rows"):
                continue
            i = int(key[4:])
            if adaptive[i]:  # (the stored rows are of the uniform-tree operator)
                continue
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
    print(f"[bench] batched{' aca' if aca_eps > 0 else ''}"
          f"{f' adaptive n_max={n_max}' if n_max > 0 else ''}: {1000.0 * wall:.1f} ms per batch "
          "of 64", file=sys.stderr, flush=True)
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
                  bank_budget=0 if args.resident_main else budget,
                  tune={"compact": args.compact, **({"nb": args.nb} if args.nb else {})})
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
           "dtype": {"fp32": "f32", "fp64": "f64", "bf16x3": "bf16", "bf16x6": "bf16"}[
               args.precision],
           "data": "synthetic",
           "config": {"workload": describe(P),
                      "precision": {
                          "fp32": "FP32 coupling products on MFMA, FP64 phases, transfers, "
                                  "near field and sums into y",
                          "bf16x3": "BF16 hi/lo split coupling products (3 per real "
                                    "product) on MFMA with FP32 sums, FP64 elsewhere",
                          "bf16x6": "BF16 hi/mid/lo split coupling products (6 per real "
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
    out["plan"] = {k: stats[k] for k in ("n_couplings", "n_stored_couplings", "n_bank_matrices",
                                         "m2l_columns",
                                         "near_entries", "device_bytes", "l_hf", "l_min")}
    out["plan"]["bank"] = (f"generated per matvec into a {args.bank_budget_gb:g} GB workspace"
                           if budget and not args.resident_main else "resident")

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

    for split in ("bf16x3", "bf16x6"):
        if args.bf16_steps <= 0 or args.precision == split:
            continue
        bf = F.Plan(pt, ps, P.kappa, P.box, P.levels, P.m, precision=split,
                    bank_budget=budget)
        bwall, bph = time_plan(bf, v, y, args.bf16_steps, min(args.warmup, 1), split)
        y_bf = y.cpu().numpy()
        bf.close()
        del bf
        bms = 1000.0 * bwall / args.bf16_steps
        bm2l = float(np.mean([p["m2l"] for p in bph]))
        alg = flops / (bm2l * 1e-3) / 1e12
        npr = SPLIT_PRODUCTS[split]
        out[split] = {"value": 1000.0 / bms, "ms_per_step": bms, "steps": args.bf16_steps,
                      "m2l_ms": bm2l, "m2l_tflops_algorithmic": alg,
                      "m2l_tflops_issued": npr * alg,
                      "frac_of_bf16_peak_issued": npr * alg / PEAK_TFLOPS[split],
                      "speedup_vs_mixed": ms_per_step / bms}
        if os.path.exists(golden):
            g = np.load(golden)
            out[split]["rel_l2_err_vs_oracle"] = float(
                np.linalg.norm(y_bf[rows] - yo) / np.linalg.norm(yo))
            if f"y_{split}" in g.files:
                out[split]["emulated_rel_l2_err"] = float(
                    np.linalg.norm(g[f"y_{split}"] - yo) / np.linalg.norm(yo))
        if y_plain is not None:
            out[split]["rel_l2_err_vs_plain_gpu"] = float(
                np.linalg.norm(y_bf - y_plain) / np.linalg.norm(y_plain))
        print(f"[bench] {split}: {bms:.1f} ms/matvec, M2L {bm2l:.1f} ms", file=sys.stderr,
              flush=True)

    if args.aca_eps > 0 and args.aca_steps > 0 and P.m <= 6:
        # (its low-rank bank is resident whatever the dense plans' budget)
        t0 = time.perf_counter()
        ap_ = F.Plan(pt, ps, P.kappa, P.box, P.levels, P.m, precision="fp32",
                     aca_eps=args.aca_eps)
        torch.cuda.synchronize()
        aca_setup = time.perf_counter() - t0
        awall, aph = time_plan(ap_, v, y, args.aca_steps, min(args.warmup, 1), "aca")
        ast = ap_.stats()  # after a matvec: the launch groups exist
        y_aca = y.cpu().numpy()
        ap_.close()
        del ap_
        ams = 1000.0 * awall / args.aca_steps
        am2l = float(np.mean([p["m2l"] for p in aph]))
        # two stages of 8 K r flops per block at its matrix's rank r, and
        # what the kernels issue (padded ranks, Kp rows, 64-slot items)
        alg = ast["aca_flops"]
        issued = ast["aca_issued_flops"]
        out["aca"] = {"eps": args.aca_eps, "value": 1000.0 / ams, "ms_per_step": ams,
                      "steps": args.aca_steps, "m2l_ms": am2l, "setup_s": aca_setup,
                      "rank_cap": ast["aca_rank_cap"], "rank_max": ast["aca_rank_max"],
                      "rank_mean": ast["aca_rank_mean"],
                      "m2l_tflops_algorithmic": alg / (am2l * 1e-3) / 1e12,
                      "m2l_tflops_issued": issued / (am2l * 1e-3) / 1e12,
                      "frac_of_fp32_peak_issued": issued / (am2l * 1e-3) / 1e12 / 157.3,
                      "speedup_vs_mixed": ms_per_step / ams,
                      "device_bytes": ast["device_bytes"]}
        if os.path.exists(golden):
            out["aca"]["rel_l2_err_vs_oracle"] = float(
                np.linalg.norm(y_aca[rows] - yo) / np.linalg.norm(yo))
        print(f"[bench] aca {args.aca_eps:g}: {ams:.1f} ms/matvec, M2L {am2l:.1f} ms, "
              f"rank mean {ast['aca_rank_mean']:.1f} max {ast['aca_rank_max']}",
              file=sys.stderr, flush=True)

    if args.batch_steps > 0:
        del pt, ps, v, y
        torch.cuda.empty_cache()
        out["batched"] = batched(args.batch_steps, args.compact)
        if args.aca_eps > 0 and args.aca_steps > 0:
            torch.cuda.empty_cache()
            out["batched_aca"] = batched(args.batch_steps, args.compact, args.aca_eps)
            out["batched_aca"]["speedup_vs_dense_batch"] = (
                out["batched"]["ms_per_batch"] / out["batched_aca"]["ms_per_batch"])
        if args.batch_adaptive_n_max > 0:
            torch.cuda.empty_cache()
            out["batched_adaptive"] = batched(args.batch_steps, args.compact,
                                              n_max=args.batch_adaptive_n_max)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(P, stats, shape, args.cpu_sub)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
