#!/usr/bin/env python3
"""Throughput of the parallel-tempering Metropolis path on one MI355X.

A step is one full run of the throughput workload: every walker of 256
systems (8x8 K4,4 cells x 64 Trotter slices = 32,768 spins, 32 walkers each)
does 100 sequential-order sweeps with a swap round after every sweep.  Inputs
and state are resident in HBM before the timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
BYTES_PER_ATTEMPT = 12         # spin r+w 2 B, field r+w 2 B, MT word r+w 8 B
METRIC = "spin-flip attempts/s + effective samples/s (plain vs learned proposal), 1 GPU"


def cpu_baseline(wl, budget_s=12.0):
    """The oracle on the host's cores over a bounded sample of the same workload."""
    import oracle
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    nsys = min(len(wl.systems), max(2 * ncores, 8))
    idx = list(range(nsys))
    chains = oracle.workload_chains(wl, idx)
    per_sweep = sum(wl.systems[i].N * wl.systems[i].K for i in idx)
    t0 = time.perf_counter()
    oracle.run_many(chains, 1, 1, ncores)
    t1 = time.perf_counter() - t0
    n = max(1, min(int(budget_s / max(t1, 1e-3)), wl.n_sweeps))
    t0 = time.perf_counter()
    oracle.run_many(chains, n, 1, ncores)
    dt = time.perf_counter() - t0
    return {"value": per_sweep * n / dt, "unit": "spin-flip attempts/s", "cores": int(min(ncores, nsys)),
            "kind": "oracle",
            "sample": f"{nsys} of {len(wl.systems)} systems x {wl.systems[0].K} walkers x {n} sweeps "
                      f"(swap every sweep), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="B")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build runs the whole path on a single MI355X "
              "(systems shard independently across GPUs; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1004_0024_amd as pa
    from gen import make_workload

    wl = make_workload(args.config)
    g = pa.Graph(wl.systems)
    tuned = None
    if not args.no_autotune:
        scratch = pa.State(g).init(wl.walker_seeds, wl.swap_seeds)
        trials = g.autotune(scratch, reps=3)
        del scratch
        tuned = {"trials": len(trials), "shapes": [{k: b[k] for k in ("S", "tpw", "G", "cpt", "threads", "lds")}
                                                   for b in g.buckets()]}
    st = pa.State(g).init(wl.walker_seeds, wl.swap_seeds)
    if args.copy_mib:
        src = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        del src, dst
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    n_sw = wl.n_sweeps

    def one_step(evs=None):
        for t in range(n_sw):
            if evs is not None:
                evs[2 * t].record(stream)
            st.sweep(1, 0)
            if evs is not None:
                evs[2 * t + 1].record(stream)
            st.swap(t & 1)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2 * n_sw)] for _ in range(args.steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for k in range(args.steps):
        one_step(evs[k])
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop)
    sweep_ms = [evs[k][2 * t].elapsed_time(evs[k][2 * t + 1]) for k in range(args.steps) for t in range(n_sw)]
    # The same step as one captured HIP graph (sweep + swap kernels, no host work).
    rep = st.capture(n_sw, swap_every=1)
    rep.launch()
    rep.stream.synchronize()
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g0.record(rep.stream)
    for _ in range(max(1, args.steps // 2)):
        rep.launch()
    g1.record(rep.stream)
    rep.stream.synchronize()
    graph_ms = g0.elapsed_time(g1) / max(1, args.steps // 2)
    avg_sweep_s = sum(sweep_ms) / len(sweep_ms) / 1e3
    attempts_step = g.attempts_per_sweep * n_sw
    value = attempts_step * args.steps / (ms / 1e3)
    achieved = BYTES_PER_ATTEMPT * g.attempts_per_sweep / avg_sweep_s / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "spin-flip attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": wl.name, "systems": len(wl.systems), "walkers": g.R,
                   "spins_per_system": wl.systems[0].N, "sweeps_per_step": n_sw, "swap_every": 1,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "sweep_kernel", "kernel_avg_ms": avg_sweep_s * 1e3,
                     "bytes_per_attempt": BYTES_PER_ATTEMPT},
        "wall_s_timed": wall,
        "graph_replay": {"ms_per_step": graph_ms, "value": g.attempts_per_sweep * n_sw / (graph_ms / 1e3)},
        "launch_shapes": tuned,
        "sweep_kernel_ms": {"mean": avg_sweep_s * 1e3, "min": min(sweep_ms), "max": max(sweep_ms)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
