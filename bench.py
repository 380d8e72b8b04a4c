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
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see the sharding paragraph of the design notes)", file=sys.stderr)
        sys.exit(2)

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
    t0 = time.perf_counter()
    results = []
    for _ in range(args.steps):
        results.append(step())
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
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
