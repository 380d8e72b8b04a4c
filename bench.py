"""Benchmark of the exhaustive AND/OR traversal on one MI355X.

One step = one enumeration per external output (10 targets) of the seeded
central-metabolism-shaped network (60 internal metabolites, 90 + 10 reactions,
seed 0), under a depth cap and a per-level frontier cap (the uncapped traversal
of this shape grows about nine-fold per level and its shortest pathways have
over thirty reactions, so it cannot be enumerated whole by any method).
Inputs are resident in HBM before timing: the network tables are uploaded and
the workspace allocated once.

Prints one JSON line: frontier items/s (parents expanded per second) as `value`,
balanced pathways/s and children/s beside it, the expand kernel's roofline
(algorithmic bytes per launch over its HIP-event duration on the library's
stream), and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def expand_bytes(level: dict, W: int) -> float:
    """Algorithmic HBM bytes of one expand launch: read every parent's key and
    hash (8W + 8), one 8-byte table slot per generated child, one 8-byte reference
    written per distinct child."""
    return level["parents"] * (8 * W + 8) + level["children"] * 8 + level["unique"] * 8


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_batch_networks(count):
    """Seeded batch networks, generated in worker processes (call before any GPU
    use: the workers are forked)."""
    import concurrent.futures as cf
    from paper_1804_02867_amd import netgen
    workers = max(1, min(16, os.cpu_count() or 1))
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(netgen.batch_member, range(count), chunksize=64))


def batch_sweep(args, nets, efm, torch):
    """The batched serving-style sweep: seeded networks of uneven size, one target
    each, in one persistent launch replayed as a HIP graph."""
    import numpy as np
    targets = [n.targets[0] for n in nets]
    handles = [efm.Network(*n.arrays()) for n in nets]
    log(f"batch: {len(nets)} networks uploaded; creating (autotune)")
    b = efm.Batch(handles, targets, depth_cap=args.batch_depth_cap, frontier_cap=args.batch_frontier_cap,
                  unique_cap=args.batch_unique_cap, found_cap=args.batch_found_cap, flags=efm.OPT_AUTOTUNE)
    log(f"batch: tile {b.config()}; warm-up sweep")
    b.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        b.run()
        log(f"batch: sweep {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    res, failed = [], 0
    for i in range(len(nets)):
        try:
            res.append(b.result(i))
        except efm.EfmError:
            failed += 1                     # a capacity of this network overflowed
    pathways = sum(r.count for r in res)
    parents = sum(r.levels[0]["parents"] for r in res)
    lat = b.latency_ns() / 1e6
    cfg = b.config()
    b.close()
    out = {"workload": f"{len(nets)} batch networks (m 10-80, n 15-120 log-uniform, seeds 100000+i), "
                       f"depth cap {args.batch_depth_cap}, frontier cap {args.batch_frontier_cap}",
           "ms_per_sweep": dt * 1e3, "networks_per_s": len(nets) / dt, "pathways_per_s": pathways / dt,
           "pathways_per_sweep": pathways, "frontier_items_per_s": parents / dt,
           "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
           "tile": {"waves_per_network": cfg[0], "networks_per_cu": cfg[1]},
           "networks_over_capacity": failed}
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        k = 0
        cpu_paths = 0
        while k < len(nets) and time.perf_counter() - t < 10.0:
            S, rev, ext = nets[k].arrays()
            cpu_paths += oracle.enumerate_pathways(S, rev, ext, targets[k], depth_cap=args.batch_depth_cap,
                                                   frontier_cap=args.batch_frontier_cap).count
            k += 1
        cdt = time.perf_counter() - t
        out["cpu_baseline"] = {"networks_per_s": k / cdt, "pathways_per_s": cpu_paths / cdt, "cores": 1,
                               "kind": "oracle", "sample": f"first {k} networks of the sweep ({cdt:.1f} s)"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--depth-cap", type=int, default=40)
    ap.add_argument("--frontier-cap", type=int, default=1 << 20)
    ap.add_argument("--targets", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--batch-depth-cap", type=int, default=12)
    ap.add_argument("--batch-frontier-cap", type=int, default=2048)
    ap.add_argument("--batch-unique-cap", type=int, default=1 << 19)
    ap.add_argument("--batch-found-cap", type=int, default=1 << 15)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see the sharding paragraph of the design notes)", file=sys.stderr)
        sys.exit(2)

    batch_nets = None
    if not args.no_batch:
        t = time.perf_counter()
        batch_nets = make_batch_networks(args.batch_count)
        log(f"batch: generated {len(batch_nets)} networks in {time.perf_counter() - t:.1f} s")

    import numpy as np
    import torch
    from paper_1804_02867_amd import efm, netgen

    torch.cuda.set_device(0)
    net = netgen.central(args.seed)
    S, rev, ext = net.arrays()
    W = (net.n + 63) // 64
    targets = net.targets[:args.targets]
    g = efm.Network(S, rev, ext)
    kw = dict(depth_cap=args.depth_cap, frontier_cap=args.frontier_cap,
              unique_cap=max(args.frontier_cap * 24, 1 << 20), found_cap=1 << 16,
              flags=efm.OPT_TIME_KERNELS)
    opts = efm.make_opts(**kw)
    ws = torch.empty(efm.workspace_bytes(g, opts), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        out = []
        for x in targets:
            out.append(efm.enumerate_pathways(g, x, workspace=ws, stream=stream, **kw))
        return out

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("central: warm-up done")
    t0 = time.perf_counter()
    results = []
    for k in range(args.steps):
        results.append(step())
        log(f"central: step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    parents = sum(lv["parents"] for rs in results for r in rs for lv in r.levels)
    children = sum(lv["children"] for rs in results for r in rs for lv in r.levels)
    pathways = sum(r.count for rs in results for r in rs)
    ms_exp = sum(lv["ms_expand"] for rs in results for r in rs for lv in r.levels)
    nlaunch = sum(1 for rs in results for r in rs for lv in r.levels if lv["parents"] > 0)
    bytes_exp = sum(expand_bytes(lv, W) for rs in results for r in rs for lv in r.levels)
    ms_total_kernels = {k: sum(lv[k] for rs in results for r in rs for lv in r.levels)
                        for k in ("ms_expand", "ms_rank", "ms_exact", "ms_select", "ms_materialize")}
    achieved = bytes_exp / (ms_exp * 1e-3) / 1e9 if ms_exp > 0 else 0.0

    cpu = None
    if not args.no_cpu_baseline:
        log("central: CPU oracle sample")
        import oracle
        ncores = 1
        sample_targets = targets[:3]
        cap = 2000
        t = time.perf_counter()
        cpu_parents = 0
        for x in sample_targets:
            r = oracle.enumerate_pathways(S, rev, ext, x, depth_cap=args.depth_cap, frontier_cap=cap)
            cpu_parents += int(r.levels[:, 0].sum())
        dt = time.perf_counter() - t
        cpu = {"value": cpu_parents / dt, "unit": "frontier items/s", "cores": ncores, "kind": "oracle",
               "sample": f"central seed {args.seed}, targets {sample_targets}, depth cap {args.depth_cap}, "
                         f"frontier cap {cap} (single-threaded oracle, {dt:.1f} s)"}

    line = {
        "metric": "balanced pathways/s + frontier items/s (HBM GB/s %peak); learned vs plain recall@speedup",
        "value": parents / elapsed,
        "unit": "frontier items/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"central-shaped 60x100 network seed {args.seed}, {len(targets)} targets, "
                               f"depth cap {args.depth_cap}, frontier cap {args.frontier_cap}",
                   "depth_cap": args.depth_cap, "frontier_cap": args.frontier_cap,
                   "targets": len(targets), "parallelism": "none (1 GPU)"},
        "pathways_per_s": pathways / elapsed,
        "children_per_s": children / elapsed,
        "pathways_per_step": pathways / args.steps,
        "kernel_ms_per_step": {k: v / args.steps for k, v in ms_total_kernels.items()},
        "roofline": {"bound": "hbm", "kernel": "expand_kernel", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "launches": nlaunch, "avg_launch_ms": ms_exp / max(nlaunch, 1),
                     "alg_bytes_per_launch": bytes_exp / max(nlaunch, 1)},
        "cpu_baseline": cpu,
    }
    if not args.no_batch:
        line["batch"] = batch_sweep(args, batch_nets, efm, torch)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
