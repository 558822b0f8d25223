"""Training and use of the learned cell proposal (driver over the C ABI).

Every numeric step runs in the library's kernels: cells are collected from
the plain chain (ising_collect_cells), the network is trained by its own
forward/backward and Adam kernels (ising_mlp_grad, ising_mlp_adam), and the
chain interleaves one plain sweep (+ swap round) with one pass of learned
cell moves (ising_propose_cells).  This module only sequences the calls.
"""
from __future__ import annotations

import math

import numpy as np

from . import ess as _ess


def _coprime_stride(total, n):
    """Smallest stride >= total/n sharing no factor with total: n rows then visit n
    distinct cells spread over every walker and slice."""
    st = max(1, total // max(1, n))
    while math.gcd(st, total) != 1:
        st += 1
    return st


def collect(state, n_rows, snapshots=4, sweeps_between=10, swap_every=1):
    """n_rows training rows (x [n,17] float32, y [n] uint8) from `snapshots` states of
    the plain chain, `sweeps_between` sweeps apart."""
    import torch
    total = int(sum(s.M * s.L * s.L * len(s.beta) for s in state.graph.systems if getattr(s, "L", 0)))
    per = n_rows // snapshots
    stride = _coprime_stride(total, per)
    xs, ys = [], []
    for k in range(snapshots):
        state.sweep(sweeps_between, swap_every)
        x, y = state.collect_cells(per, stride=stride, offset=(k * 7919) % total)
        xs.append(x)
        ys.append(y)
    return torch.cat(xs), torch.cat(ys)


def train(net, x, y, batch=4096, epochs=2, lr=1e-3):
    """Minibatch Adam; batch k of an epoch takes rows k, k + nb, k + 2 nb, ... (nb batches),
    so each batch mixes every snapshot.  Returns the loss of every step (host)."""
    import torch
    nb = x.shape[0] // batch
    if nb == 0:
        return np.zeros(0)
    xv = x[:nb * batch].view(batch, nb, x.shape[1]).transpose(0, 1).contiguous()
    yv = y[:nb * batch].view(batch, nb).transpose(0, 1).contiguous()
    losses = []
    for _ in range(epochs):
        for k in range(nb):
            losses.append(net.grad_step(xv[k], yv[k]))
            net.adam(lr)
    return torch.stack([l.reshape(()) for l in losses]).cpu().numpy()


def run(state, steps, net=None, key=0, pass0=0, swap_every=1, heatbath=False, cell_every=1, time_cells=False):
    """`steps` steps of the chain: a sweep and its swap round, then, with a network, one
    pass of learned cell moves, or with `heatbath`, one pass of exact heat-bath cell
    moves, after every `cell_every`-th step.  Returns slot energies [steps, slots] (host),
    GPU ms and the fraction of cells accepted (learned) or changed (heat-bath).  With
    `time_cells`, HIP events around every pass also give its GPU time ("cell_pass_ms")."""
    import torch
    g = state.graph
    e = torch.zeros((steps, g.slots), dtype=torch.int32, device=g.tables.device)
    cells = net is not None or heatbath
    moves = torch.zeros((g.R, 2), dtype=torch.int64, device=g.tables.device) if cells else None
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    evs = []
    torch.cuda.synchronize()
    t0.record()
    for t in range(steps):
        state.sweep(1, swap_every)
        if cells and (t + 1) % cell_every == 0:
            if time_cells:
                evs.append((torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)))
                evs[-1][0].record()
            if net is not None:
                state.propose_cells(net, key, pass0 + t, moves)
            else:
                state.heatbath_cells(key, pass0 + t, moves)
            if time_cells:
                evs[-1][1].record()
        state.record(e[t])
    t1.record()
    torch.cuda.synchronize()
    out = {"e": e.cpu().numpy(), "ms": t0.elapsed_time(t1)}
    if time_cells:
        out["cell_pass_ms"] = [a.elapsed_time(b) for a, b in evs]
    if moves is not None:
        mv = moves.cpu().numpy()
        out["acceptance"] = float(mv[:, 1].sum()) / max(1.0, float(mv[:, 0].sum()))
    return out


def ess_summary(graph, series, burn=0.2):
    """ESS of the energy at the coldest slot of every system (summed) and the median
    over all slots."""
    coldest, allv = [], []
    base = 0
    for s in graph.systems:
        K = len(s.beta)
        col = np.argmax(s.beta)
        e = _ess.slot_ess(series[:, base:base + K], burn)
        coldest.append(e[col])
        allv.extend(e.tolist())
        base += K
    return {"coldest_total": float(np.sum(coldest)), "median_slot": float(np.median(allv))}


def slot_ess_totals(graph, series, positions, burn=0.2):
    """ESS of the energy at ladder position k (0 = hottest), summed over systems, for
    every k in `positions` (systems with fewer slots are skipped)."""
    tot = {int(k): 0.0 for k in positions}
    base = 0
    for s in graph.systems:
        K = len(s.beta)
        for k in tot:
            if k < K:
                tot[k] += _ess.ess(series[:, base + k], burn)
        base += K
    return tot


def compare_means(graph, series_a, series_b, burn=0.2):
    """Slot mean energies of two chains on the same systems, in units of their combined
    standard error (variance / ESS per series).  Returns, per slot position in the ladder
    (0 = hottest), the median |z| over systems and the fraction of systems with |z| < 4,
    and the fraction of all (system, slot) pairs with |z| < 4."""
    zs = []
    base = 0
    for s in graph.systems:
        K = len(s.beta)
        za = np.zeros(K)
        for k in range(K):
            xa = series_a[:, base + k][int(burn * len(series_a)):].astype(np.float64)
            xb = series_b[:, base + k][int(burn * len(series_b)):].astype(np.float64)
            ea, eb = _ess.ess(xa, 0.0), _ess.ess(xb, 0.0)
            se = np.sqrt(xa.var() / max(ea, 1.0) + xb.var() / max(eb, 1.0))
            za[k] = (xa.mean() - xb.mean()) / se if se > 0 else 0.0
        zs.append(za)
        base += K
    zs = np.abs(np.array(zs))
    return {"median_abs_z_by_slot": [float(v) for v in np.median(zs, axis=0)],
            "frac_below_4_by_slot": [float(v) for v in np.mean(zs < 4.0, axis=0)],
            "frac_abs_z_below_4": float(np.mean(zs < 4.0))}


def matched_slots(graph, series, reference="plain", null=None, burn=0.2, frac=0.99):
    """Ladder positions where every chain's slot means agree with the reference chain's:
    |z| < 4 (compare_means) for at least `frac` of the systems, for each chain of
    `series` (a dict of [steps, slots] energy series).  With `null` (the name of a later,
    independent stretch of the reference chain) a position also counts when every chain
    agrees with the reference at least as often as that stretch does: the reference
    against itself calibrates the test where the standard errors are loose.  Returns
    (positions, comparisons by chain name, the null's included)."""
    comp = {name: compare_means(graph, e, series[reference], burn)
            for name, e in series.items() if name != reference}
    K = min(len(s.beta) for s in graph.systems)
    chains = [c for name, c in comp.items() if name != null]
    bar = [frac if null is None else min(frac, comp[null]["frac_below_4_by_slot"][k]) for k in range(K)]
    ok = [k for k in range(K) if all(c["frac_below_4_by_slot"][k] >= bar[k] for c in chains)]
    return ok, comp
