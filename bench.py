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
# Modular multiply-reduce peak (mod 2^31-1), derived from the unit counts: 256 CUs x
# 128 32-bit lanes per clock x 2.4 GHz = 78.6 T lane-ops/s, and 12 issue slots per
# multiply-reduce (two quarter-rate 32-bit multiplies, four full-rate ops).
MULMOD_PEAK_T = 256 * 128 * 2.4e9 / 12 / 1e12
# HBM bytes per launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs of one bench
# step (calibrated on a 1 GiB device copy: FETCH_SIZE x 2, WRITE_SIZE x 1); None
# when the kernel changed after the counters were taken.
TRAFFIC_PER_LAUNCH = {"expand": 749.8e6, "rank": 135.9e6}


def expand_bytes(level: dict, W: int) -> float:
    """Algorithmic HBM bytes of one expand launch, per-unit figures of the step:
    read every parent's key (8W bytes) and, per generated child, its key and an
    8-byte hash slot (8W + 8 bytes).  (The kernel writes an 8-byte reference in
    place of each child's key.)"""
    return level["parents"] * (8 * W) + level["children"] * (8 * W + 8)


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
           "latency_ms_max": float(lat.max()),
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


def learned_section(args, efm, torch):
    """Learned vs plain: traces from the plain traversal of seeded training
    networks, GPU training, then on held-out networks the exhaustive plain set,
    the learned ordering and the canonical truncation at each budget."""
    import numpy as np
    from paper_1804_02867_amd import netgen
    D, UC = args.learned_depth_cap, 1 << 27
    t = time.perf_counter()
    tr = efm.Traces(1024, 400, capacity=1 << 22)
    runs = with_paths = 0
    for i in range(args.learned_train):
        net = netgen.learn_member(200000 + i)
        g = efm.Network(*net.arrays())
        for x in net.targets:
            try:
                info = tr.collect(g, x, depth_cap=D, unique_cap=UC, pos_max=1000, neg_per_pos=3.0, neg_min=500,
                                  seed=i * 7 + x)
            except efm.EfmError as e:
                if "traces full" in str(e):
                    break
                continue                     # a capacity overflowed: this run gives no traces
            runs += 1
            with_paths += info["pathways"] > 0
        if (i + 1) % 5 == 0:
            log(f"learned: traces from {i + 1} networks")
    collect_s = time.perf_counter() - t
    nrec, npos = tr.info()
    m = efm.Model(1024, 400, seed=args.seed)
    tt = time.perf_counter()
    st1 = m.train(tr, epochs=args.learned_epochs, batch=1024, lr=2e-3, seed=1)
    st2 = m.train(tr, epochs=max(1, args.learned_epochs // 2), batch=1024, lr=4e-4, seed=2)
    train_s = time.perf_counter() - tt
    log(f"learned: {nrec} records trained in {train_s:.1f} s (loss {st1['loss_first']:.3f} -> {st2['loss_last']:.3f})")
    tr.close()
    budgets = [1 << int(b) for b in args.learned_budgets.split(",")]
    first = netgen.learn_member(300000)
    g0 = efm.Network(*first.arrays())
    ws_plain = torch.empty(efm.workspace_bytes(g0, efm.make_opts(D, 0, UC, 0, 0)), dtype=torch.uint8, device="cuda")
    ws_learn = torch.empty(max(efm.workspace_bytes(g0, efm.make_opts(D, B, UC, 0, efm.OPT_LEARNED)) for B in budgets),
                           dtype=torch.uint8, device="cuda")
    agg = {B: {"hits": 0, "canon_hits": 0, "t": 0.0, "t_canon": 0.0, "macro": [], "macro_canon": []}
           for B in budgets}
    t_plain, total, pairs = 0.0, 0, 0
    for i in range(args.learned_eval):
        net = netgen.learn_member(300000 + i)
        g = efm.Network(*net.arrays())
        for x in net.targets:
            try:
                t = time.perf_counter()
                p = efm.enumerate_pathways(g, x, depth_cap=D, unique_cap=UC, workspace=ws_plain)
                tp = time.perf_counter() - t
            except efm.EfmError:
                continue                     # exhaustive run too large for the capacity: no reference set
            if p.keys.shape[0] == 0:
                continue
            P = {tuple(k) for k in p.keys.tolist()}
            pairs += 1
            total += len(P)
            t_plain += tp
            for B in budgets:
                t = time.perf_counter()
                lr = efm.enumerate_learned(g, x, B, m, depth_cap=D, unique_cap=UC, workspace=ws_learn)
                tl = time.perf_counter() - t
                t = time.perf_counter()
                cn = efm.enumerate_pathways(g, x, depth_cap=D, frontier_cap=B, unique_cap=UC, workspace=ws_plain)
                tc = time.perf_counter() - t
                hl = len(P & {tuple(k) for k in lr.keys.tolist()})
                hc = len(P & {tuple(k) for k in cn.keys.tolist()})
                a = agg[B]
                a["hits"] += hl
                a["canon_hits"] += hc
                a["t"] += tl
                a["t_canon"] += tc
                a["macro"].append(hl / len(P))
                a["macro_canon"].append(hc / len(P))
        log(f"learned: evaluated {i + 1} networks")
    rows = []
    for B in budgets:
        a = agg[B]
        rows.append({"budget": B, "recall": a["hits"] / max(total, 1), "recall_macro": float(np.mean(a["macro"] or [0])),
                     "speedup_vs_plain": t_plain / max(a["t"], 1e-12), "learned_s": a["t"],
                     "canonical_recall": a["canon_hits"] / max(total, 1),
                     "canonical_recall_macro": float(np.mean(a["macro_canon"] or [0])), "canonical_s": a["t_canon"]})
    return {"workload": f"learned ordering on power-law networks (40 internal metabolites, 60 + 4 reactions), "
                        f"depth cap {D}; train seeds 200000..{200000 + args.learned_train - 1}, held-out seeds "
                        f"300000..{300000 + args.learned_eval - 1}, every target with a non-empty exhaustive set",
            "train": {"runs": runs, "runs_with_pathways": with_paths, "records": nrec, "positives": npos,
                      "collect_s": collect_s, "train_s": train_s, "epochs": args.learned_epochs + max(1, args.learned_epochs // 2),
                      "loss_first": st1["loss_first"], "loss_last": st2["loss_last"]},
            "eval": {"pairs": pairs, "pathways": total, "plain_s": t_plain},
            "budgets": rows, "target_recall": 0.99}


def copy_calibration(torch, nbytes=1 << 30, reps=4):
    """Plain device-to-device copies of a known size: the reference that scales
    the HBM byte counters of a profiled run."""
    src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy calibration: {reps} copies of {nbytes} bytes")
    del src, dst


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
    ap.add_argument("--sections", default="central,batch,learned",
                    help="comma list of central, batch, learned, genome (profiling runs pick one)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device to device 4 times (byte-counter reference)")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--batch-depth-cap", type=int, default=12)
    ap.add_argument("--batch-frontier-cap", type=int, default=2048)
    ap.add_argument("--batch-unique-cap", type=int, default=1 << 19)
    ap.add_argument("--batch-found-cap", type=int, default=1 << 15)
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--learned-train", type=int, default=20)
    ap.add_argument("--learned-eval", type=int, default=12)
    ap.add_argument("--learned-epochs", type=int, default=8)
    ap.add_argument("--learned-depth-cap", type=int, default=16)
    ap.add_argument("--learned-budgets", default="14,16,18,20,22")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the traversal would shard children by hash over GPUs; not implemented)", file=sys.stderr)
        sys.exit(2)
    sections = set(args.sections.split(","))
    if args.no_batch:
        sections.discard("batch")
    if args.no_learned:
        sections.discard("learned")

    batch_nets = None
    if "batch" in sections:
        t = time.perf_counter()
        batch_nets = make_batch_networks(args.batch_count)
        log(f"batch: generated {len(batch_nets)} networks in {time.perf_counter() - t:.1f} s")

    import torch
    from paper_1804_02867_amd import efm

    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(torch)
    line = {"metric": "balanced pathways/s + frontier items/s (HBM GB/s %peak); learned vs plain recall@speedup",
            "value": None, "unit": "frontier items/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u64", "data": "synthetic"}
    if "central" in sections:
        line.update(central_section(args, efm, torch))
    if "batch" in sections:
        line["batch"] = batch_sweep(args, batch_nets, efm, torch)
    if "learned" in sections:
        line["learned"] = learned_section(args, efm, torch)
    if "genome" in sections:
        line["genome"] = genome_section(args, efm, torch)
    print(json.dumps(line), flush=True)


def genome_section(args, efm, torch):
    """The genome-shaped network at its full caps (depth 40, frontier 2^26), once."""
    from paper_1804_02867_amd import netgen
    net = netgen.genome(args.seed)
    g = efm.Network(*net.arrays())
    kw = dict(depth_cap=40, frontier_cap=1 << 26, unique_cap=1 << 30, found_cap=1 << 16, flags=efm.OPT_TIME_KERNELS)
    ws = torch.empty(efm.workspace_bytes(g, efm.make_opts(**kw)), dtype=torch.uint8, device="cuda")
    log(f"genome: workspace {ws.numel() / 2**30:.1f} GiB")
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = efm.enumerate_pathways(g, net.targets[0], workspace=ws, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    parents = sum(lv["parents"] for lv in r.levels)
    children = sum(lv["children"] for lv in r.levels)
    log(f"genome: {parents} parents in {dt:.1f} s")
    return {"workload": f"genome-shaped 400x640 network seed {args.seed}, target {net.targets[0]}, depth cap 40, "
                        f"frontier cap 2^26", "s": dt, "frontier_items_per_s": parents / dt,
            "children_per_s": children / dt, "pathways": int(r.count), "status": int(r.status),
            "workspace_gib": ws.numel() / 2**30,
            "kernel_ms": {k: sum(lv[k] for lv in r.levels)
                          for k in ("ms_expand", "ms_rank", "ms_exact", "ms_select", "ms_materialize")}}


def central_section(args, efm, torch):
    """The headline workload: every target of the central-shaped network."""
    from paper_1804_02867_amd import netgen
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
    # rank stage (the dominant kernels): rows x k^2 modular multiplies per tested
    # child of k reactions (children of loop level i have i + 2 reactions)
    rank_ops = sum(lv["rank_rows"] * (i + 2) ** 2 for rs in results for r in rs for i, lv in enumerate(r.levels))
    ms_rank = ms_total_kernels["ms_rank"]
    achieved_rank = rank_ops / (ms_rank * 1e-3) / 1e12 if ms_rank > 0 else 0.0
    shares = {k: v / max(sum(ms_total_kernels.values()), 1e-12) for k, v in ms_total_kernels.items()}

    cpu = None
    if not args.no_cpu_baseline:
        log("central: CPU oracle sample")
        import oracle
        ncores = 1
        sample_targets = targets[:3]
        cap = 1000
        t = time.perf_counter()
        cpu_parents = 0
        for x in sample_targets:
            r = oracle.enumerate_pathways(S, rev, ext, x, depth_cap=args.depth_cap, frontier_cap=cap)
            cpu_parents += int(r.levels[:, 0].sum())
        dt = time.perf_counter() - t
        cpu = {"value": cpu_parents / dt, "unit": "frontier items/s", "cores": ncores, "kind": "oracle",
               "sample": f"central seed {args.seed}, targets {sample_targets}, depth cap {args.depth_cap}, "
                         f"frontier cap {cap} (single-threaded oracle, {dt:.1f} s)"}

    return {
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
        "kernel_share": shares,
        "roofline": {"bound": "alu", "kernel": "rank stage (rank_parent_kernel + rank_kernel)",
                     "achieved": achieved_rank, "peak": MULMOD_PEAK_T, "unit": "T mulmod/s",
                     "frac": achieved_rank / MULMOD_PEAK_T, "traffic": TRAFFIC_PER_LAUNCH["rank"],
                     "launches": nlaunch, "avg_launch_ms": ms_rank / max(nlaunch, 1),
                     "alg_ops_per_launch": rank_ops / max(nlaunch, 1)},
        "expand_roofline": {"bound": "hbm", "kernel": "expand_kernel", "achieved": achieved, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": TRAFFIC_PER_LAUNCH["expand"],
                            "launches": nlaunch, "avg_launch_ms": ms_exp / max(nlaunch, 1),
                            "alg_bytes_per_launch": bytes_exp / max(nlaunch, 1)},
        "cpu_baseline": cpu,
    }


if __name__ == "__main__":
    main()
