"""Benchmark: lattice enumeration for market split instances on one MI355X.

One step = the whole GPU path for every instance of the workload: embedding +
LLL (+ BKZ with --bkz) + kernel extraction (msp_reduce),
Gram-Schmidt, root generation and the exhaustive subtree walk (msp_enumerate,
mode all).  Inputs (A, d) are resident on the device before timing starts.
The headline value is enumeration nodes per second over the whole step (a
node is a candidate that passed the l2 test), i.e. total nodes / wall time
of the step.

Also reported:
  roofline      the walk kernel against FP64 vector peak: algorithmic flops
                per node 3 (n+1) + 4 (an axpy and an l1 norm over n+1
                coordinates plus the partial-norm recurrence) and 4 per
                candidate that fails the l2 test, divided by the walk kernel's
                measured duration (HIP events on its launch stream);
  ttfs          time to the first verified solution per instance of the
                TTFS sets (12 planted instances each): m=9 on LLL bases,
                depth-first search in plain root order against the learned
                root order (the committed root-scoring model); m=11 on BKZ-16
                bases, limited discrepancy search in plain against learned
                root order.  Each instance is reduced once; both orders then
                search the same basis.  Each search is capped (a capped run
                is censored and counts as the cap in the medians);
  cpu_baseline  the CPU oracle (plain recursive C enumerator, all host cores,
                the host CPU model named) on a time-capped sample of the
                first instance.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector peak

# HBM bytes per walk-kernel launch measured with rocprofv3 counters
# (FETCH_SIZE and WRITE_SIZE, each scaled by what the same counter reads for a
# 1 GiB device copy in the same run), keyed by (workload, BKZ block size) and
# valid only for the kernel source they were taken on.
WALK_TRAFFIC = {
    ("m9-1", 0): {"bytes": 1.367e13,
                  "sha256": "ca4ede88d54a5e3a7fe52ece06c0d6e4162dbe28a3c3498e154e18cc428f9f36",
                  "profile": "profiles/walk_kernel_m9_n80_D200_seed4508.md"},
    ("m11-b10", 16): {"bytes": 1.278e13,
                      "sha256": "ca4ede88d54a5e3a7fe52ece06c0d6e4162dbe28a3c3498e154e18cc428f9f36",
                      "profile": "profiles/walk_kernel_m11_n100_bkz16_seed5003_budget10.md"},
}


def walk_source_hash() -> str:
    """sha256 of the walk kernel's code: walk.hip, enum_rules.h and
    msp_internal.h with their comments, trailing blanks and blank lines
    removed, so that a traffic figure outlives edits to comments only."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("walk.hip", "enum_rules.h", "msp_internal.h"):
        with open(os.path.join(ROOT, "paper_2508_08702_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        code = [ln.rstrip() for ln in src.splitlines() if ln.strip()]
        h.update("\n".join(code).encode())
    return h.hexdigest()

WORKLOADS = {
    # name: (description, list of (m, D, seed), generator)
    "m9": ("12 planted instances m=9, n=80, 4 each D=50/100/200 (seeds 4500-4511), exhaustive",
           [(9, (50, 100, 200)[i // 4], 4500 + i) for i in range(12)], "planted"),
    "m9-d200": ("4 planted instances m=9, n=80, D=200 (seeds 4508-4511), exhaustive",
                [(9, 200, 4508 + i) for i in range(4)], "planted"),
    "m9-1": ("1 planted instance m=9, n=80, D=200 (seed 4508), exhaustive",
             [(9, 200, 4508)], "planted"),
    "m8": ("4 planted instances m=8, n=70, D=100 (seeds 4000-4003), exhaustive",
           [(8, 100, 4000 + i) for i in range(4)], "planted"),
    "cd8": ("4 Cornuejols-Dawande instances m=8, n=70, D=100, d = floor(row sums / 2) "
            "(seeds 6000-6003), exhaustive (mostly infeasible: empty output after the full walk)",
            [(8, 100, 6000 + i) for i in range(4)], "cd"),
    # the walker variant of the m=11 first-solution passes (one wave per SIMD, budget state),
    # exhaustive within one discrepancy budget on a BKZ-16 basis; extra parameters in the dict
    "m11-b10": ("1 planted instance m=11, n=100, D=50 (seed 5003), BKZ-16 basis, every path with at most "
                "10 discrepancies (rank reading)",
                [(11, 50, 5003)], "planted", {"bkz_block": 16, "disc_budget": 10}),
}


# first-solution sets: reduction and the two strategies compared on it
TTFS_SETS = {
    "m9": {"bkz": 0, "orders": "plain,learned", "cap_ms": 6000.0},
    "m11": {"bkz": 16, "orders": "lds,lds-learned", "cap_ms": 8000.0},
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="m9-1", choices=sorted(WORKLOADS))
    ap.add_argument("--ttfs", default="m9,m11",
                    help="comma-separated first-solution sets timed per order (m9, m11; none to skip)")
    ap.add_argument("--ttfs-cap-ms", type=float, default=0.0, help="cap per search (0: the set's default)")
    ap.add_argument("--ttfs-seeds", default="", help="comma-separated subset of the TTFS sets' seeds")
    ap.add_argument("--orders", default="", help="orders timed on every TTFS set (empty: the set's default)")
    ap.add_argument("--ttfs-bkz", type=int, default=-1, help="BKZ block size of the TTFS reductions (-1: the set's)")
    ap.add_argument("--batch", action="store_true",
                    help="also time the uneven 96-instance batch (msp_solve_batch) with autotuned root counts")
    ap.add_argument("--bkz", type=int, default=0,
                    help="BKZ block size of the main workload's reduction (0: LLL only)")
    ap.add_argument("--model", default=os.path.join(ROOT, "paper_2508_08702_amd", "order_model.npy"))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before timing, run one plain device copy of this size (a known-size kernel that "
                         "calibrates HBM byte counters in a profile of this command)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--time-cap-ms", type=float, default=600000.0)
    return ap.parse_args()


def batch_run(M, ctx, args, np, torch, mi, dev):
    """The uneven batch: 96 planted instances, m in 5..8 (drawn per
    instance), D by thirds.  Root counts are autotuned on 8 instances of the
    disjoint tuning seeds 3900-3931 first (not timed); the context keeps the
    fastest count per shape (m, n bucket), which msp_solve_batch applies to
    the instances of tuned shapes.  Then one msp_solve_batch call (one LLL
    launch for all, then each instance's enumeration) is timed end to end and
    every returned row is checked A x = d."""
    tune = mi.mixed_batch(range(3900, 3932))[:8]
    prm = M.msp_params_default(time_cap_ms=args.time_cap_ms)
    t0 = time.perf_counter()
    best, pts = M.msp_autotune(ctx, [torch.from_numpy(i.A).to(dev) for i in tune],
                               [torch.from_numpy(i.d).to(dev) for i in tune], params=prm)
    tune_s = time.perf_counter() - t0
    insts = mi.mixed_batch()
    As = [torch.from_numpy(i.A).to(dev) for i in insts]
    ds = [torch.from_numpy(i.d).to(dev) for i in insts]
    M.msp_solve_batch(ctx, As, ds, params=prm)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = M.msp_solve_batch(ctx, As, ds, params=prm)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nodes = sum(st["nodes"] for st in r.stats)
    kern = sum(st["kernel_ms"] for st in r.stats)
    for inst, x, status in zip(insts, r.x, r.status):
        xs = x.cpu().numpy().astype(np.int64)
        if status not in (M.MSP_OK, M.MSP_E_CAPACITY) or xs.shape[0] == 0 or \
                not np.all(xs @ inst.A.T.astype(np.int64) == inst.d[None, :]):
            raise RuntimeError(f"batch instance {inst.seed}: status {status} or a row fails A x = d")
    return {"instances": len(insts), "wall_ms": wall * 1e3, "nodes": nodes, "nodes_per_s": nodes / wall,
            "walk_ms_sum": kern, "solutions": int(sum(r.n_found)),
            "tuned_target_roots": best.target_roots, "tune_seconds": tune_s,
            "tuned_per_shape": {f"m{m}_n{n}": M.msp_tune_lookup(ctx, m, n)
                                for m, n in sorted({(i.m, i.n) for i in insts})},
            "tune_points": [{"target_roots": t, "status": s_, "ms": ms} for t, s_, ms in pts]}


def ttfs_set(M, ctx, args, np, torch, mi, dev, which):
    """First-solution search per instance and order.  Each instance is
    reduced once (timed); every order then searches that basis, so the
    end-to-end time of an order is the reduction plus its own search."""
    cfg = TTFS_SETS[which]
    bkz = cfg["bkz"] if args.ttfs_bkz < 0 else args.ttfs_bkz
    cap = args.ttfs_cap_ms if args.ttfs_cap_ms > 0 else cfg["cap_ms"]
    insts = mi.m9_eval() if which == "m9" else mi.m11_eval()
    if args.ttfs_seeds:
        keep = {int(x) for x in args.ttfs_seeds.split(",")}
        insts = [i for i in insts if i.seed in keep]
    # name: (mode, root order): one first-solution walk in an order, or
    # limited discrepancy search (passes with a rising budget) in an order
    orders = {"plain": (M.MSP_FIRST, M.MSP_PLAIN), "learned": (M.MSP_FIRST, M.MSP_LEARNED),
              "discrepancy": (M.MSP_FIRST, M.MSP_DISCREPANCY), "lds": (M.MSP_LDS, M.MSP_PLAIN),
              "lds-learned": (M.MSP_LDS, M.MSP_LEARNED)}
    names = [o for o in (args.orders or cfg["orders"]).split(",") if o]
    if any(o.endswith("learned") for o in names):
        M.msp_model_set(ctx, np.load(args.model))
    per = []
    for inst in insts:
        if not per:
            print(f"  ttfs {which}: {len(insts)} instances, orders {names}, cap {cap:.0f} ms", file=sys.stderr,
                  flush=True)
        A = torch.from_numpy(inst.A).to(dev)
        d = torch.from_numpy(inst.d).to(dev)
        row = {"m": inst.m, "D": int(inst.D), "seed": int(inst.seed)}
        red_ms = None
        Bk = None
        for name in names:
            prm = M.msp_params_default(time_cap_ms=cap, bkz_block=bkz)
            if name.startswith("lds-r"):
                # "lds-r<R>[-learned]": LDS over R shuffled copies, reduced together
                prm.restarts = int(name[5:].split("-")[0])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = M.msp_solve_first(ctx, A, d, params=prm, cap=64, raise_on_error=False,
                                      order=M.MSP_LEARNED if name.endswith("-learned") else M.MSP_PLAIN)
                torch.cuda.synchronize()
                e2e = (time.perf_counter() - t0) * 1e3
            else:
                if Bk is None:
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    Bk = M.msp_reduce(ctx, A, d, prm)
                    torch.cuda.synchronize()
                    red_ms = (time.perf_counter() - t0) * 1e3
                mode, order = orders[name]
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = M.msp_enumerate(ctx, A, d, Bk, params=prm, mode=mode, order=order, cap=64,
                                    raise_on_error=False)
                torch.cuda.synchronize()
                e2e = red_ms + (time.perf_counter() - t0) * 1e3
            xs = r.x.cpu().numpy().astype(np.int64)
            ok = xs.shape[0] > 0 and bool(np.all(xs @ inst.A.T.astype(np.int64) == inst.d[None, :]))
            if r.n_found and not ok:
                raise RuntimeError("a first-mode row does not satisfy A x = d")
            st = r.stats
            row[name] = {"ttfs_ms": st["ttfs_ms"] if ok else None, "end_to_end_ms": e2e if ok else None,
                         "censored": not ok, "status": r.status, "nodes": st["nodes"], "evals": st["evals"],
                         "search_ms": st["total_ms"], "roots": st["roots"],
                         "split_depth": st["split_depth"], "ordering_ms": st["ordering_ms"],
                         "rootgen_ms": st["rootgen_ms"], "stages": st["stages"], "root_level": st["root_level"],
                         "initial_items": st["initial_items"]}
            if name.startswith("lds-r"):
                row[name]["copy"] = st["copy"]
        if red_ms is not None:
            row["reduce_ms"] = red_ms
        print(json.dumps({"ttfs_instance": row}), file=sys.stderr, flush=True)
        per.append(row)

    def lower(r, name):
        # a censored run counts as its lower bound: the reduction plus the cap
        return r[name]["end_to_end_ms"] if not r[name]["censored"] else r.get("reduce_ms", 0.0) + cap

    def med(name):
        return statistics.median([lower(r, name) for r in per])

    out = {"set": f"{len(insts)} planted instances m={insts[0].m}, n={insts[0].n}, 4 each D=50/100/200",
           "reduction": f"BKZ-{bkz}" if bkz else "LLL",
           "mode": "first", "cap_ms": cap, "orders": names,
           "median_end_to_end_ms": {n: med(n) for n in names},
           "median_note": "a censored search counts as the reduction time plus the cap (a lower bound)",
           "censored": {n: sum(r[n]["censored"] for r in per) for n in names},
           "solved_within_cap": {n: sum(not r[n]["censored"] for r in per) for n in names},
           "per_instance": per}
    if len(names) == 2:
        a_, b_ = names
        out[f"median_{a_}_over_{b_}"] = med(a_) / med(b_)
    return out


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the walk runs on one GPU; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import msp_instances as mi
    import paper_2508_08702_amd as M

    desc, spec, gen = WORKLOADS[args.workload][:3]
    extra = WORKLOADS[args.workload][3] if len(WORKLOADS[args.workload]) > 3 else {}
    if gen == "cd":
        insts = [mi.cornuejols_dawande(m, s, D) for (m, D, s) in spec]
    else:
        insts = [mi.msp_class(m, D, s) for (m, D, s) in spec]
    dev = torch.device("cuda", 0)
    dev_in = [(torch.from_numpy(i.A).to(dev), torch.from_numpy(i.d).to(dev)) for i in insts]
    ctx = M.Context(0)
    prm = M.msp_params_default(time_cap_ms=args.time_cap_ms, bkz_block=args.bkz)
    for key, val in extra.items():
        setattr(prm, key, val)
    out = torch.zeros((1 << 16, max(i.n for i in insts)), dtype=torch.uint8, device=dev)

    def step(record):
        tot_nodes = tot_evals = 0
        for inst, (A, d) in zip(insts, dev_in):
            Bk = M.msp_reduce(ctx, A, d, prm)
            o = out[:, : inst.n].contiguous()
            r = M.msp_enumerate(ctx, A, d, Bk, params=prm, out=o, cap=o.shape[0])
            if r.status != M.MSP_OK:
                raise RuntimeError(f"enumeration status {r.status} ({M.msp_strerror(r.status)})")
            xs = r.x.cpu().numpy().astype(np.int64)
            if xs.shape[0] and not np.all(xs @ inst.A.T.astype(np.int64) == inst.d[None, :]):
                raise RuntimeError("a returned row does not satisfy A x = d")
            if gen == "planted" and xs.shape[0] == 0:
                raise RuntimeError("the planted solution was not found")
            st = r.stats
            tot_nodes += st["nodes"]
            tot_evals += st["evals"]
            if record is not None:
                record.append((inst, st))
        return tot_nodes, tot_evals

    if args.copy_probe_mib > 0:
        src = torch.empty(args.copy_probe_mib << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for i in range(args.warmup):
        step(None)
        print(f"  warm-up step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    rec = []
    t0 = time.perf_counter()
    nodes = 0
    for i in range(args.steps):
        n_, _e = step(rec)
        nodes += n_
        print(f"  timed step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    # roofline of the walk kernel: algorithmic flops over measured kernel time
    flops = 0.0
    kern_s = 0.0
    for inst, st in rec:
        dim = inst.n + 1
        flops += st["nodes"] * (3 * dim + 4) + (st["evals"] - st["nodes"]) * 4
        kern_s += st["kernel_ms"] * 1e-3
    achieved = flops / kern_s / 1e12 if kern_s > 0 else 0.0
    tr = WALK_TRAFFIC.get((args.workload, prm.bkz_block))
    traffic = tr["bytes"] if tr and tr["sha256"] == walk_source_hash() else None
    res = {
        "metric": "enum nodes/s + time-to-first-solution, m=9..11, plain vs learned order",
        "value": nodes / wall,
        "unit": "nodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "instances": len(insts), "mode": "all", "order": "plain",
                   "reduction": f"BKZ-{prm.bkz_block}" if prm.bkz_block else "LLL",
                   **({"disc_budget": prm.disc_budget} if "disc_budget" in extra else {}),
                   "nodes_per_step": nodes // max(1, args.steps)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
                     "kernel": "walk_kernel", "walk_ms_total": kern_s * 1e3,
                     "walk_launches": len(rec), "walk_ms_avg": kern_s * 1e3 / max(1, len(rec)),
                     "flops_per_node": "3*(n+1)+4, plus 4 per failed candidate"},
        "phase_ms_per_step": {
            k: sum(st[k] for _, st in rec) / args.steps
            for k in ("gs_ms", "rootgen_ms", "kernel_ms", "total_ms")
        },
    }
    sets = [x for x in args.ttfs.split(",") if x and x != "none"]
    for which in sets:
        if which not in TTFS_SETS:
            raise SystemExit(f"unknown TTFS set {which}")
    if sets:
        res["ttfs"] = {which: ttfs_set(M, ctx, args, np, torch, mi, dev, which) for which in sets}
    if args.batch:
        res["batch"] = batch_run(M, ctx, args, np, torch, mi, dev)
    if not args.no_cpu_baseline:
        from oracle import enum as E
        from oracle import lattice as L
        inst = insts[0]
        P = L.prepare(inst.A, inst.d)
        cores = os.cpu_count() or 1
        r = E.enumerate_prepared(P, split=12, threads=cores, time_cap_s=args.cpu_seconds)
        res["cpu_baseline"] = {"value": r.nodes / r.seconds, "unit": "nodes/s", "cores": cores, "kind": "oracle",
                               "cpu_model": cpu_model(),
                               "sample": f"instance m={inst.m} D={inst.D} seed={inst.seed}, first "
                                         f"{r.seconds:.1f} s of the exhaustive enumeration (time cap), "
                                         f"{r.nodes} nodes"}
    ctx.close()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
