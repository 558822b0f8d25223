"""Parity in the configurations bench.py times, at full size.

The graphs come from bench.tuned_graph (the autotuner as the benchmark runs
it), and the steps are the benchmark's own: the throughput workload's timed
step (single-sweep launches, each followed by a swap round) and its captured
100-sweep replay; the many-replica workload's 200-sweep and the uneven batch's
1,000-sweep captured loops (the uneven batch with its buckets on side
streams).  Sampled systems are compared with the oracle bit for bit after each
stage, including MT windows, labels, swap streams and every counter.  The
shapes the benchmark reported on MI355X (512 threads per walker for the
32,768-spin systems, 128 for the 4,096-spin ones) are also run explicitly, so
they are covered whatever the tuner picks in this process.
"""
import pytest

import bench
import oracle
from gen import make_workload

from .gpu_util import chains_for, compare_system, say

pytestmark = pytest.mark.gpu


def _run_oracle(chains, n, swap_every=1):
    oracle.run_many(chains, n, swap_every, min(16, len(chains)))


def _compare(st, idx, chains, what):
    for s, ch in zip(idx, chains):
        compare_system(st, s, ch, what)


def _shapes(g):
    return [(b["S"], b["tpw"], b["G"], b["cpt"], b["ladder"]) for b in g.buckets()]


def _throughput_run(g, wl, label):
    import torch

    import paper_1004_0024_amd as pa
    idx = [0, 127, 255]
    say("B", label, "shapes", _shapes(g), "compare", idx)
    st = pa.State(g).init(wl.walker_seeds, wl.swap_seeds)
    chains = chains_for(wl, idx)
    bench.throughput_step(st, wl.n_sweeps)  # the timed step
    torch.cuda.synchronize()
    _run_oracle(chains, wl.n_sweeps)
    _compare(st, idx, chains, f"B {label}: one timed step")
    st.sweep(10, 5)  # one call, launches of 5 sweeps, a swap round after each launch
    torch.cuda.synchronize()
    _run_oracle(chains, 10, 5)
    _compare(st, idx, chains, f"B {label}: 5-sweep launches")
    rep = st.capture(wl.n_sweeps, swap_every=1)  # the benchmark's graph_replay leg
    rep.launch()
    rep.stream.synchronize()
    _run_oracle(chains, wl.n_sweeps)
    _compare(st, idx, chains, f"B {label}: captured step replayed")
    assert st.sweeps == 2 * wl.n_sweeps + 10
    assert st.stats()["near"] >= sum(ch.counters()["near"] for ch in chains)


def test_throughput_workload_tuned():
    wl = make_workload("B")
    g, trials = bench.tuned_graph(wl, reps=3)
    assert len(g.buckets()) == 1 and len(trials) > 1
    _throughput_run(g, wl, "autotuned")


def test_throughput_workload_512_threads_per_walker():
    import paper_1004_0024_amd as pa
    wl = make_workload("B")
    g = pa.Graph(wl.systems)
    g.set_launch(0, 512, 1)
    assert _shapes(g) == [(512, 512, 1, 1, 0)]
    _throughput_run(g, wl, "512x1")


def _many_replica_run(g, wl, label):
    import paper_1004_0024_amd as pa
    idx = [0, 1023, 2047]
    say("C", label, "shapes", _shapes(g), "compare", idx)
    st = pa.State(g).init(wl.walker_seeds, wl.swap_seeds)
    chains = chains_for(wl, idx)
    rep = st.capture(wl.n_sweeps, swap_every=1)  # the benchmark's 200-sweep loop
    rep.launch()
    rep.stream.synchronize()
    _run_oracle(chains, wl.n_sweeps)
    _compare(st, idx, chains, f"C {label}: 200-sweep replay")


def test_many_replica_workload_tuned():
    wl = make_workload("C")
    g, _ = bench.tuned_graph(wl, reps=2)
    _many_replica_run(g, wl, "autotuned")


def test_many_replica_workload_128_threads_per_walker():
    import paper_1004_0024_amd as pa
    wl = make_workload("C")
    g = pa.Graph(wl.systems)
    g.set_launch(0, 128, 1)
    assert _shapes(g) == [(128, 128, 1, 1, 0)]
    _many_replica_run(g, wl, "128x1")


def test_uneven_batch_tuned_1000_sweep_replay():
    """The 2,000-system batch: one captured 1,000-sweep loop in the tuned shapes, every
    bucket but the first on a side stream; one system of every template size compared."""
    import paper_1004_0024_amd as pa
    wl = make_workload("D")
    g, _ = bench.tuned_graph(wl, reps=2)
    sizes = {}
    for i, s in enumerate(wl.systems):
        if s.S not in sizes or s.N * s.K < wl.systems[sizes[s.S]].N * wl.systems[sizes[s.S]].K:
            sizes[s.S] = i
    idx = sorted(sizes.values())
    assert len(idx) == len(g.buckets()) == 7
    say("D shapes", _shapes(g), "compare", idx)
    st = pa.State(g).init(wl.walker_seeds, wl.swap_seeds)
    chains = chains_for(wl, idx)
    rep = st.capture(wl.n_sweeps, swap_every=1)
    rep.launch()
    rep.stream.synchronize()
    _run_oracle(chains, wl.n_sweeps)
    _compare(st, idx, chains, "D: 1000-sweep replay")
