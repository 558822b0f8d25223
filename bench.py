#!/usr/bin/env python3
"""Throughput of the parallel-tempering Metropolis path on one MI355X.

A step is one full run of the throughput workload: every walker of 256
systems (8x8 K4,4 cells x 64 Trotter slices = 32,768 spins, 32 walkers each)
does 100 sequential-order sweeps with a swap round after every sweep.  Inputs
and state are resident in HBM before the timed region; 10 timed steps by
default (median and spread of the step times are reported).  Prints one JSON
line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
BF16_PEAK_TFLOPS = 2500.0      # MI355X dense BF16 matrix peak, TFLOP/s
BYTES_PER_ATTEMPT = 12         # spin r+w 2 B, field r+w 2 B, MT word r+w 8 B
# ALU model of an attempt: 32-bit lane operations (MT19937 word ~14, flip test ~7, update ~32, loop
# and addresses), against the chip's 32-bit integer lane-op rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
LANE_OPS_PER_ATTEMPT = 60
LANE_OPS_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12   # 39.3 T lane-ops/s
FLOPS_PER_CELL = 2 * (17 * 128 + 128 * 128 + 128 * 8)  # one network evaluation: 39,168
METRIC = "spin-flip attempts/s + effective samples/s (plain vs learned proposal), 1 GPU"
# Measured HBM traffic and issue figures of a kernel come from the committed rocprofv3 summary of
# its workload (a "measured:" JSON line in the profile), and are reported only while the kernel's
# sources hash to the value recorded there.
SWEEP_SOURCES = ["sweep.hip", "internal.h", "mt19937.h", "swap_round.h"]
CELL_SOURCES = ["cells.hip", "internal.h", "mlp.h"]


def sources_hash(names):
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_1004_0024_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def sweep_sources_hash():
    return sources_hash(SWEEP_SOURCES)


def measured_counters(config, profile=None, sources=SWEEP_SOURCES):
    """(figures, why): the profile's measured line when its source hash matches, else None."""
    path = os.path.join("profiles", profile or f"sweep_kernel_{config}_counters.md")
    try:
        text = open(os.path.join(ROOT, path)).read()
    except OSError:
        return None, f"no {path}"
    m = re.search(r"^measured: (\{.*\})\s*$", text, re.M)
    if not m:
        return None, f"{path} has no measured line"
    fig = json.loads(m.group(1))
    now = sources_hash(sources)
    if fig.get("sources_sha256") != now:
        return None, f"stale: {path} was taken with sources {fig.get('sources_sha256')}, now {now}"
    fig["source"] = path
    return fig, None


def alu_roofline(attempts_per_s):
    """The ALU side of the same model (the sweep is bound by integer arithmetic as much as by
    bytes): lane operations per second at LANE_OPS_PER_ATTEMPT against the chip's peak."""
    achieved = LANE_OPS_PER_ATTEMPT * attempts_per_s / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": LANE_OPS_PEAK_T, "unit": "T lane-ops/s",
            "frac": achieved / LANE_OPS_PEAK_T, "lane_ops_per_attempt": LANE_OPS_PER_ATTEMPT}


def cpu_baseline(wl, budget_s=20.0):
    """The oracle on the host's cores over a bounded sample of the same workload:
    the first systems (at least two per core), every walker, as many sweeps (with a
    swap round after each) as fit the time budget, at most the workload's own."""
    import oracle
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    nsys = min(len(wl.systems), max(2 * ncores, 8))
    chains = oracle.workload_chains(wl, list(range(nsys)))
    t0 = time.perf_counter()
    oracle.run_many(chains, 1, 1, ncores)
    t1 = time.perf_counter() - t0
    if t1 * wl.n_sweeps < budget_s:  # the whole run of these systems is short: take more systems
        nsys = min(len(wl.systems), int(nsys * budget_s / (t1 * wl.n_sweeps)) + 1)
        chains = oracle.workload_chains(wl, list(range(nsys)))
        t0 = time.perf_counter()
        oracle.run_many(chains, 1, 1, ncores)
        t1 = time.perf_counter() - t0
    per_sweep = sum(wl.systems[i].N * wl.systems[i].K for i in range(nsys))
    n = max(1, min(int(budget_s / max(t1, 1e-3)), wl.n_sweeps - 1))
    t0 = time.perf_counter()
    oracle.run_many(chains, n, 1, ncores)
    dt = time.perf_counter() - t0
    # one thread on the first system, a per-core figure (the paper quotes per-core rates)
    one = oracle.workload_chains(wl, [0])
    t0 = time.perf_counter()
    oracle.run_many(one, 1, 1, 1)
    t1c = time.perf_counter() - t0
    n1 = max(1, min(int(3.0 / max(t1c, 1e-3)), wl.n_sweeps - 2))
    t0 = time.perf_counter()
    oracle.run_many(one, n1, 1, 1)
    d1 = time.perf_counter() - t0
    return {"value": per_sweep * n / dt, "unit": "spin-flip attempts/s", "cores": int(min(ncores, nsys)),
            "kind": "oracle",
            "sample": f"{nsys} of {len(wl.systems)} systems x {wl.systems[0].K} walkers x {n} sweeps "
                      f"(swap every sweep), {dt:.1f} s",
            "one_core": {"value": wl.systems[0].N * wl.systems[0].K * n1 / d1,
                         "sample": f"1 system x {wl.systems[0].K} walkers x {n1} sweeps, 1 thread, {d1:.1f} s"}}


def progress(*a):
    """A line on stderr when a leg ends (the JSON line is the only stdout output)."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def tuned_graph(wl, reps=3):
    """The workload's graph with the launch shapes the autotuner picks (timed on a
    scratch state), as every timed leg here uses it; the parity tests call this
    too, so they run the shapes that are timed.  With several buckets, which run
    side by side, the shapes are then refined by the time of the whole sweep
    (tune.refine_shapes_side_by_side; its steps in g.side_by_side)."""
    import paper_1004_0024_amd as pa
    from paper_1004_0024_amd import tune

    g = pa.Graph(wl.systems)
    scratch = pa.State(g).init(wl.walker_seeds, wl.swap_seeds)
    trials = g.autotune(scratch, reps=reps)
    g.side_by_side = tune.refine_shapes_side_by_side(scratch)
    del scratch
    return g, trials


def throughput_step(st, n_sweeps, stream=None, evs=None):
    """One timed step of the throughput workload: n_sweeps single-sweep launches,
    each followed by a swap round (round t tries the pairs of parity t mod 2; the
    step starts at an even round count); evs, if given, time every sweep launch."""
    for t in range(n_sweeps):
        if evs is not None:
            evs[2 * t].record(stream)
        st.sweep(1, 0)
        if evs is not None:
            evs[2 * t + 1].record(stream)
        st.swap(t & 1)


def batch_leg(name, n_sweeps, reps=3):
    """Attempts/s of another workload shape: the launch shapes autotuned, then one
    captured loop of `n_sweeps` sweeps (each followed by a swap round) replayed
    `reps` times; HIP events on the replay stream."""
    import torch

    import paper_1004_0024_amd as pa
    from gen import make_workload

    wl = make_workload(name)
    g, _ = tuned_graph(wl, reps=2)
    st = pa.State(g).init(wl.walker_seeds, wl.swap_seeds)
    rep = st.capture(n_sweeps, swap_every=1)
    rep.launch()
    rep.stream.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(rep.stream)
    for _ in range(reps):
        rep.launch()
    e1.record(rep.stream)
    rep.stream.synchronize()
    ms = e0.elapsed_time(e1) / reps
    rate = g.attempts_per_sweep * n_sweeps / (ms / 1e3)
    achieved = BYTES_PER_ATTEMPT * rate / 1e9
    return {"workload": wl.name, "systems": len(wl.systems), "walkers": g.R,
            "attempts_per_sweep": g.attempts_per_sweep, "sweeps_per_replay": n_sweeps,
            "buckets": len(g.buckets()), "ms_per_sweep": ms / n_sweeps,
            "launch_shapes": [{k: b[k] for k in ("S", "tpw", "G", "cpt", "threads", "lds", "stream", "work")}
                              for b in g.buckets()],
            "side_by_side_refinement": g.side_by_side,
            "value": rate, "unit": "spin-flip attempts/s",
            # the whole replay (sweep kernels, swap rounds, side-stream joins) against the 12 B model
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "bytes_per_attempt": BYTES_PER_ATTEMPT,
                         "alu": alu_roofline(rate)}}


def two_field_leg(steps, gamma=1.0):
    """The throughput workload in the two-field form (the QMC models' separate in-slice
    and tau fields): every tau coupling +1, Trotter weights of a transverse field gamma
    over the 64 slices, launch shapes autotuned in this form; `steps` steps of 100
    sweeps with a swap round after each, HIP events around every sweep launch."""
    import dataclasses

    import numpy as np
    import torch

    import paper_1004_0024_amd as pa
    from gen import make_workload

    wl = make_workload("B")
    wl.systems = [dataclasses.replace(s, J_tau=np.ones(s.S, np.int8)) for s in wl.systems]
    g = pa.Graph(wl.systems)
    ab = [pa.trotter_weights(s.beta, s.M, gamma) for s in wl.systems]
    g.set_two_field(np.concatenate([x[0] for x in ab]), np.concatenate([x[1] for x in ab]))
    scratch = pa.State(g).init(wl.walker_seeds, wl.swap_seeds)
    g.autotune(scratch, reps=3)
    del scratch
    st = pa.State(g).init(wl.walker_seeds, wl.swap_seeds)
    stream = torch.cuda.current_stream()
    n_sw = wl.n_sweeps
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * n_sw * steps)]
    for t in range(n_sw):  # warm-up step
        st.sweep(1, 0)
        st.swap(t & 1)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for k in range(steps):
        for t in range(n_sw):
            evs[2 * (k * n_sw + t)].record(stream)
            st.sweep(1, 0)
            evs[2 * (k * n_sw + t) + 1].record(stream)
            st.swap(t & 1)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    sweep_ms = [evs[2 * i].elapsed_time(evs[2 * i + 1]) for i in range(n_sw * steps)]
    avg = sum(sweep_ms) / len(sweep_ms)
    stats = st.stats()
    achieved = BYTES_PER_ATTEMPT * g.attempts_per_sweep / (avg / 1e3) / 1e9
    return {"workload": wl.name + ", two-field form (unit tau couplings, gamma %.2f)" % gamma,
            "steps": steps, "ms_per_step": ms / steps,
            "value": g.attempts_per_sweep * n_sw * steps / (ms / 1e3), "unit": "spin-flip attempts/s",
            "sweep_kernel_ms": {"mean": avg, "min": min(sweep_ms), "max": max(sweep_ms)},
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "bytes_per_attempt": BYTES_PER_ATTEMPT,
                         "alu": alu_roofline(g.attempts_per_sweep / (avg / 1e3))},
            "launch_shapes": [{k: b[k] for k in ("S", "tpw", "G", "cpt", "threads", "lds")} for b in g.buckets()],
            "flip_rate": stats["flips"] / max(1, stats["attempts"]),
            "wave_steps_with_flip": stats["wave_flip_steps"] / max(1, stats["wave_steps"])}


def pairs_leg(name, n_sweeps, reps):
    """The layer-pair order (the paper's GPU layout, Sec. 3.2, Fig. 12c) on a workload:
    one launch runs `n_sweeps` sweeps of every walker with a swap round after each
    (whole systems per workgroup); `reps` launches timed with HIP events."""
    import numpy as np
    import torch

    import paper_1004_0024_amd as pa
    from gen import make_workload

    wl = make_workload(name)
    g = pa.Graph(wl.systems)
    st = pa.State(g)
    lanes = sum(s.K * (s.M // 2) for s in wl.systems)
    st.pairs_init((100_000 + np.arange(lanes)).astype(np.uint32), wl.swap_seeds)
    st.pairs_sweep(n_sweeps, 1)  # warm-up
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
    torch.cuda.synchronize()
    for k in range(reps):
        evs[2 * k].record(stream)
        st.pairs_sweep(n_sweeps, 1)
        evs[2 * k + 1].record(stream)
    torch.cuda.synchronize()
    ms = [evs[2 * k].elapsed_time(evs[2 * k + 1]) for k in range(reps)]
    avg = sum(ms) / reps
    attempts = g.attempts_per_sweep * n_sweeps
    achieved = BYTES_PER_ATTEMPT * attempts / (avg / 1e3) / 1e9
    stats = st.stats()
    return {"workload": wl.name + ", layer-pair order", "sweeps_per_launch": n_sweeps, "launches": reps,
            "kernel_ms": {"mean": avg, "min": min(ms), "max": max(ms)}, "us_per_sweep": avg * 1e3 / n_sweeps,
            "value": attempts / (avg / 1e3), "unit": "spin-flip attempts/s",
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "bytes_per_attempt": BYTES_PER_ATTEMPT,
                         "kernel": "pairs_kernel", "alu": alu_roofline(attempts / (avg / 1e3))},
            "flip_rate": stats["flips"] / max(1, g.attempts_per_sweep * st.sweeps)}


def learned_leg(ess_steps, train_rows=1 << 20, burn_in=20000):
    """Learned cell proposal on the 256 x 32-walker, 4,096-spin workload: train the
    network on the GPU from plain-chain samples, then effective samples per second of
    the plain chain (sweep + swap round per step) against the learned chain (sweep +
    swap round + one pass of learned cell moves per step) and the heat-bath chain (the
    same with exact heat-bath cell moves), all from the same state after `burn_in`
    plain sweeps.  The ratios are taken at matched observable accuracy: at the ladder
    positions where both cell-move chains' slot mean energies agree with the plain
    chain's within 4 combined standard errors for at least 99% of the systems."""
    import numpy as np
    import torch

    import paper_1004_0024_amd as pa
    from paper_1004_0024_amd import learn, tune
    from gen import make_workload
    from gen.mlp import initial_params

    wl = make_workload("E")
    g = pa.Graph(wl.systems)
    st = pa.State(g).init(wl.walker_seeds, wl.swap_seeds)
    st.sweep(burn_in, 1)
    t0 = time.perf_counter()
    x, y = learn.collect(st, train_rows, snapshots=8, sweeps_between=5)
    net = pa.Mlp(initial_params(11))
    net0 = pa.Mlp(initial_params(11))
    loss0 = float(net.grad_step(x[:4096], y[:4096]).item())
    losses = np.concatenate([learn.train(net, x, y, batch=4096, epochs=1, lr=lr) for lr in (2e-3, 2e-3, 5e-4)])
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    base = pa.State(g).copy_from(st)
    # acceptance of one pass, untrained vs trained network, from the same state
    acc = {}
    for name, n in (("untrained", net0), ("trained", net)):
        s2 = pa.State(g).copy_from(base)
        mv = torch.zeros((g.R, 2), dtype=torch.int64, device="cuda")
        s2.propose_cells(n, 7, 0, mv)
        m = mv.sum(0).cpu().numpy()
        acc[name] = float(m[1]) / float(m[0])
    # cell-move kernel time: events around passes on the current stream
    s2 = pa.State(g).copy_from(base)
    stream = torch.cuda.current_stream()
    passes = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s2.propose_cells(net, 9, 0)
    e0.record(stream)
    for p in range(passes):
        s2.propose_cells(net, 9, 1 + p)
    e1.record(stream)
    torch.cuda.synchronize()
    # colour classes of the cells: 2, or 4 on a ring of odd length
    launches = passes * max(4 if (s.ring and s.M % 2 == 1) else 2 for s in wl.systems)
    launch_ms = e0.elapsed_time(e1) / launches
    cells_per_pass = sum(s.M * s.L * s.L * s.K for s in wl.systems)
    flops = FLOPS_PER_CELL * cells_per_pass / (launches / passes)
    tflops = flops / (launch_ms / 1e3) / 1e12
    # heat-bath kernel time, the same way
    s2 = pa.State(g).copy_from(base)
    s2.heatbath_cells(19, 0)
    e0.record(stream)
    for p in range(passes):
        s2.heatbath_cells(19, 1 + p)
    e1.record(stream)
    torch.cuda.synchronize()
    hb_ms = e0.elapsed_time(e1) / launches
    # the same kernels where the chains run them: one pass after every sweep and swap
    # round, events around each pass (500 steps after a 100-step warm-up)
    in_chain = {}
    for name, n, hb in (("learned", net, False), ("heatbath", None, True)):
        s2 = pa.State(g).copy_from(base)
        learn.run(s2, 100, n, pass0=500, heatbath=hb)
        r = learn.run(s2, 500, n, pass0=600, heatbath=hb, time_cells=True)
        ms = np.asarray(r["cell_pass_ms"]) / (launches / passes)
        in_chain[name] = {"launch_ms": {"mean": float(ms.mean()), "median": float(np.median(ms)),
                                        "min": float(ms.min()), "max": float(ms.max())}, "passes": len(ms)}
    chain_ms = in_chain["learned"]["launch_ms"]["mean"]
    chain_tflops = flops / (chain_ms / 1e3) / 1e12
    chains, series = {}, {}
    for name, n, hb in (("plain", None, False), ("learned", net, False), ("heatbath", None, True)):
        s2 = pa.State(g).copy_from(base)
        r = learn.run(s2, ess_steps, n, pass0=1000, heatbath=hb)
        series[name] = r["e"]
        if name == "plain":  # the plain chain's next stretch: the null of the accuracy test
            series["plain_next"] = learn.run(s2, ess_steps, None)["e"]
        e = learn.ess_summary(g, r["e"])
        chains[name] = {"ms_per_step": r["ms"] / ess_steps, "ess_coldest": e["coldest_total"],
                        "ess_median_slot": e["median_slot"],
                        "ess_per_s": e["coldest_total"] / (r["ms"] / 1e3),
                        "coldest_mean_energy": float(r["e"][:, 31::32].mean())}
        if "acceptance" in r:
            chains[name]["cell_acceptance" if n is not None else "cell_changed"] = r["acceptance"]
    # cell-move cadence: one pass of learned (or heat-bath) cell moves after every k-th step
    cell_cadence = []
    for every in (2, 4, 8):
        row = {"cell_every": every}
        for name, n, hb in (("learned", net, False), ("heatbath", None, True)):
            s2 = pa.State(g).copy_from(base)
            r = learn.run(s2, ess_steps // 2, n, pass0=2000, heatbath=hb, cell_every=every)
            e = learn.ess_summary(g, r["e"])
            row[name] = {"ms_per_step": r["ms"] / (ess_steps // 2), "ess_coldest": e["coldest_total"],
                         "ess_per_s": e["coldest_total"] / (r["ms"] / 1e3)}
        cell_cadence.append(row)
    # swap cadence, tuned by effective samples per second (it changes the chain)
    cadence = tune.swap_cadence(base, (1, 2, 4, 8), ess_steps // 2)
    # matched observable accuracy: the ladder positions where both cell-move chains agree
    # with the plain chain; ESS per second there
    ms_total = {name: chains[name]["ms_per_step"] * ess_steps for name in chains}
    slots, comp = learn.matched_slots(g, series, null="plain_next")
    matched = {"criterion": "ladder positions where the learned and the heat-bath chain's slot mean "
                            "energies agree with the plain chain's, |z| < 4 (combined standard error from "
                            "variance / ESS), for at least 99% of the 256 systems, or at least as often as "
                            "the plain chain's next 10,000 steps agree with its first (the null)",
               "slots": slots,
               "frac_below_4_by_slot": {k: v["frac_below_4_by_slot"] for k, v in comp.items()}}
    if slots:
        kc = max(slots)  # the coldest matched position (beta ascends along the ladder)
        per_s = {name: learn.slot_ess_totals(g, series[name], [kc])[kc] / (ms_total[name] / 1e3)
                 for name in chains}
        tot = {name: sum(learn.slot_ess_totals(g, series[name], slots).values()) / (ms_total[name] / 1e3)
               for name in chains}
        matched.update({
            "coldest_matched_slot": kc, "beta": float(wl.systems[0].beta[kc]),
            "ess_per_s_at_slot": per_s,
            "learned_over_plain": per_s["learned"] / per_s["plain"],
            "heatbath_over_plain": per_s["heatbath"] / per_s["plain"],
            "summed_over_matched_slots": {"learned_over_plain": tot["learned"] / tot["plain"],
                                          "heatbath_over_plain": tot["heatbath"] / tot["plain"]}})
    cell_roofline = {"bound": "mfma", "kernel": "cell_propose_kernel", "kernel_avg_ms": chain_ms,
                     "timed": "the learned chain: one pass after every sweep and swap round",
                     "achieved": chain_tflops, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": chain_tflops / BF16_PEAK_TFLOPS, "flops_per_cell": FLOPS_PER_CELL,
                     "cells_per_launch": cells_per_pass / (launches / passes), "traffic": None,
                     "traffic_unit": "HBM bytes per launch",
                     "back_to_back": {"kernel_avg_ms": launch_ms, "achieved": tflops,
                                      "frac": tflops / BF16_PEAK_TFLOPS, "passes": passes,
                                      "note": "passes with nothing between them run at a lower, "
                                              "power-limited clock"}}
    fig, why = measured_counters("E", "cell_propose_kernel_E.md", CELL_SOURCES)
    if fig is not None:
        cell_roofline["traffic"] = fig["hbm_bytes_per_launch"]
        cell_roofline["measured"] = {k: fig.get(k) for k in ("source", "sources_sha256", "mfma_busy", "valu_busy")}
    else:
        cell_roofline["traffic_note"] = why
    return {
        "workload": wl.name, "steps": ess_steps, "burn_in_sweeps": burn_in,
        "matched_accuracy": matched,
        "swap_cadence": cadence,
        "cell_cadence": cell_cadence,
        "ess": "energy at the coldest slot (beta 3.0), Sokal window c=5, first 20% dropped, summed over systems; "
               "the coldest slot is not matched (see matched_accuracy)",
        "train": {"rows": int(x.shape[0]), "batch": 4096, "adam_steps": int(len(losses)),
                  "loss_untrained": loss0, "loss_last": float(losses[-1]), "seconds": train_s},
        "acceptance_one_pass": acc,
        "plain": chains["plain"], "learned": chains["learned"], "heatbath": chains["heatbath"],
        "ess_per_s_learned_over_plain": chains["learned"]["ess_per_s"] / chains["plain"]["ess_per_s"],
        "ess_per_s_heatbath_over_plain": chains["heatbath"]["ess_per_s"] / chains["plain"]["ess_per_s"],
        "heatbath_kernel_ms": hb_ms,
        "cell_kernels_in_chain": in_chain,
        # slot mean energies of the cell-move chains against the plain chain, in combined
        # standard errors (per system and slot)
        "means_vs_plain": {k: v for k, v in comp.items() if k != "plain_next"},
        "plain_vs_its_next_stretch": comp["plain_next"],
        "roofline": cell_roofline,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="B")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one device copy of this size (counter calibration)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-proposal leg")
    ap.add_argument("--no-batches", action="store_true", help="skip the many-replica and uneven-batch legs")
    ap.add_argument("--no-two-field", action="store_true", help="skip the two-field (QMC) leg")
    ap.add_argument("--no-pairs", action="store_true", help="skip the layer-pair order leg")
    ap.add_argument("--ess-steps", type=int, default=10000,
                    help="chain steps per ESS estimate in the learned-proposal leg")
    ap.add_argument("--burn-in", type=int, default=20000,
                    help="plain sweeps before the learned-proposal leg collects and compares")
    ap.add_argument("--bucket-shapes", action="store_true",
                    help="also time the uneven batch's whole sweep with each bucket in its other launch shapes")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the whole path runs on a single MI355X "
              "(systems shard independently across GPUs, one process per GPU)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1004_0024_amd as pa
    from gen import make_workload

    wl = make_workload(args.config)
    tuned = None
    if not args.no_autotune:
        g, trials = tuned_graph(wl, reps=3)
        tuned = {"trials": len(trials), "shapes": [{k: b[k] for k in ("S", "tpw", "G", "cpt", "threads", "lds")}
                                                   for b in g.buckets()]}
    else:
        g = pa.Graph(wl.systems)
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
        throughput_step(st, n_sw, stream, evs)

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
    # per-step times: from the first sweep's start event of a step to the next step's
    step_ms = [evs[k][0].elapsed_time(evs[k + 1][0]) for k in range(args.steps - 1)] + \
        [evs[args.steps - 1][0].elapsed_time(stop)]
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
    stats = st.stats()
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
        "step_ms": {"median": sorted(step_ms)[len(step_ms) // 2], "min": min(step_ms), "max": max(step_ms)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": wl.name, "systems": len(wl.systems), "walkers": g.R,
                   "spins_per_system": wl.systems[0].N, "sweeps_per_step": n_sw, "swap_every": 1,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "model": "algorithmic: 12 B per attempt (spin r+w 2, field r+w 2, MT word r+w 8) x "
                              "attempts per launch / live mean launch time; the kernel keeps its state in "
                              "LDS and moves far fewer bytes (traffic, measured)",
                     "traffic": None, "traffic_unit": "HBM bytes per launch",
                     "kernel": "sweep_kernel", "kernel_avg_ms": avg_sweep_s * 1e3,
                     "bytes_per_attempt": BYTES_PER_ATTEMPT,
                     "alu": alu_roofline(g.attempts_per_sweep / avg_sweep_s)},
        "wall_s_timed": wall,
        "graph_replay": {"ms_per_step": graph_ms, "value": g.attempts_per_sweep * n_sw / (graph_ms / 1e3)},
        "launch_shapes": tuned,
        "sweep_kernel_ms": {"mean": avg_sweep_s * 1e3, "min": min(sweep_ms), "max": max(sweep_ms)},
        # accepted flips per attempt, and the share of wavefront steps in which some lane
        # flipped (the analogue of the paper's probability of waiting for a flip)
        "flip_rate": stats["flips"] / max(1, stats["attempts"]),
        "wave_steps_with_flip": stats["wave_flip_steps"] / max(1, stats["wave_steps"]),
        # FP64 swap decisions within 1e-12 of their threshold, over every round of this run
        "near_threshold": {"count": stats["near"], "swap_decisions": stats["swap_att"]},
    }
    fig, why = measured_counters(args.config)
    if fig is not None:
        out["roofline"]["traffic"] = fig["hbm_bytes_per_launch"]
        out["roofline"]["measured"] = {
            "source": fig["source"], "sources_sha256": fig["sources_sha256"],
            "hbm_GBs": fig["hbm_bytes_per_launch"] / avg_sweep_s / 1e9,
            "hbm_frac": fig["hbm_bytes_per_launch"] / avg_sweep_s / 1e9 / HBM_PEAK_GBS,
            "valu_busy": fig.get("valu_busy"), "valu_per_64_attempts": fig.get("valu_per_64_attempts")}
    else:
        out["roofline"]["traffic_note"] = why
    del rep, st
    progress("throughput workload", f"{value:.4g} attempts/s")
    if not args.no_batches:
        out["other_shapes"] = []
        for name, n, reps in (("A", 1000, 3), ("C", 200, 3), ("D", 1000, 2)):
            out["other_shapes"].append(batch_leg(name, n, reps))
            progress("workload", name, f"{out['other_shapes'][-1]['value']:.4g} attempts/s")
    if args.bucket_shapes:
        from paper_1004_0024_amd import tune
        wd = make_workload("D")
        gd, _ = tuned_graph(wd, reps=2)
        out["bucket_shapes_side_by_side"] = tune.bucket_shapes_side_by_side(
            pa.State(gd).init(wd.walker_seeds, wd.swap_seeds))
        progress("bucket shapes side by side done")
    if not args.no_two_field:
        out["two_field"] = two_field_leg(max(2, args.steps // 2))
        out["two_field"]["over_one_field"] = out["two_field"]["value"] / value
        progress("two-field form done")
    if not args.no_pairs:
        out["layer_pairs"] = [pairs_leg("B", 100, max(2, args.steps // 2)), pairs_leg("A", 1000, 3)]
        progress("layer-pair order done")
    if not args.no_learned:
        out["effective_samples"] = learned_leg(args.ess_steps, burn_in=args.burn_in)
        progress("learned proposal done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
        progress("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
