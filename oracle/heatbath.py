"""Oracle of the exact cell heat-bath -- TEST INFRASTRUCTURE ONLY.

Plain numpy, FP64.  Only tests/, the smoke check and bench.py's CPU baseline
may import it.

The non-learned control of the learned cell proposal: each 8-spin cell (one
K4,4 cell of one slice) is redrawn from its exact conditional Boltzmann law
given the rest of the system,
  p(s_c | b) proportional to exp(-beta E_c(s_c)),
  E_c(s) = -sum_k b_k s_k - sum_{k < 4 <= r} J_kr s_k s_r,
with b_k = h_k + sum_{j outside the cell} J_kj s_j (cost function of
Section 1).  A heat-bath move needs no acceptance test.

The cell is bipartite (spins 0..3 couple only to spins 4..7), so the draw
takes two stages:
  1. the left half l = (s_0..s_3) from its marginal
       p(l) proportional to exp(beta sum_{k<4} b_k s_k) prod_{r>=4} 2 cosh(beta h_r(l)),
       h_r(l) = b_r + sum_{k<4} J_kr s_k;
  2. each right spin on its own, P(s_r = +1 | l) = sigmoid(2 beta h_r(l)).
Uniforms: Philox4x32-10, key (key mod 2^32, key div 2^32), counters
(cell, walker, pass, j) for blocks j = 0, 1.  Word 0 picks the left state:
the first of the 16 left states (index bit k = spin k is +1) whose cumulative
weight exceeds u 2^-32 times the total.  Words 1..4 draw the right spins
4..7: spin r is +1 iff u 2^-32 < sigmoid(2 beta h_r).
"""
from __future__ import annotations

import numpy as np

from .learned import CellModel, cell_colour, n_colours, philox4x32  # noqa: F401

_MASK = (1 << 32) - 1


def uniforms(key_base, walker, pass_index, cell):
    """Words 0..4 of a cell's heat-bath draw (32-bit integers)."""
    key = (key_base & _MASK, (key_base >> 32) & _MASK)
    w = philox4x32((cell, walker, pass_index, 0), key) + philox4x32((cell, walker, pass_index, 1), key)
    return w[:5]


def cell_couplings(model, idx):
    """J[k][i] between left spin k (0..3) and right spin 4 + i of the cell `idx`."""
    pos = {q: t for t, q in enumerate(idx)}
    J = np.zeros((4, 4), np.int64)
    for k in range(4):
        for q, j in model.nbr[idx[k]]:
            if q in pos and pos[q] >= 4:
                J[k, pos[q] - 4] += j
    return J


def _spins_of(index, nbits):
    return np.array([1 if (index >> k) & 1 else -1 for k in range(nbits)], np.int64)


def left_log_weights(b, J, beta):
    """log p(l) up to a constant, for the 16 left states (index bit k = spin k is +1)."""
    out = np.zeros(16)
    for i in range(16):
        s = _spins_of(i, 4)
        hr = b[4:] + s @ J  # h_r for r = 4..7
        x = beta * hr
        out[i] = beta * float(b[:4] @ s) + float(np.sum(np.logaddexp(x, -x)))
    return out


def right_fields(b, J, left_index):
    return b[4:] + _spins_of(left_index, 4) @ J


def sigmoid(x):
    return np.exp(-np.logaddexp(0.0, -np.asarray(x, np.float64)))


def two_stage_law(b, J, beta):
    """Probability of each of the 256 cell states (byte bit k = spin k is +1) under the
    two-stage draw."""
    lw = left_log_weights(b, J, beta)
    pl = np.exp(lw - lw.max())
    pl /= pl.sum()
    out = np.zeros(256)
    for i in range(16):
        x = 2.0 * beta * right_fields(b, J, i)
        pp, pm = sigmoid(x), sigmoid(-x)
        for r in range(16):
            pt = 1.0
            for t in range(4):
                pt *= pp[t] if (r >> t) & 1 else pm[t]
            out[i | (r << 4)] = pl[i] * pt
    return out


def draw(b, J, beta, u):
    """The new cell byte from the 5 uniform words u."""
    lw = left_log_weights(b, J, beta)
    wgt = np.exp(lw - lw.max())
    cum = np.cumsum(wgt)
    target = u[0] * 2.0 ** -32 * cum[-1]
    left = int(np.argmax(cum > target))
    pr = sigmoid(2.0 * beta * right_fields(b, J, left))
    right = sum(1 << t for t in range(4) if u[1 + t] * 2.0 ** -32 < pr[t])
    return left | (right << 4)


def heatbath_pass(model, spins, energy, betas, key_base, walker_ids, pass_index):
    """One pass of heat-bath cell moves over every walker of one system (colours in
    order).  spins [K, N] (+-1, modified), energy [K] (modified).  Returns the number of
    cells whose spins changed, per walker."""
    sysm = model.system
    changed = np.zeros(len(spins), np.int64)
    for colour in range(n_colours(sysm)):
        for w in range(len(spins)):
            s = spins[w]
            beta = float(betas[w])
            for ci, (m, y, x) in enumerate(model.cells):
                if cell_colour(sysm, m, y, x) != colour:
                    continue
                idx = model.cell_spins(m, y, x)
                b = model.boundary(s, idx)
                J = cell_couplings(model, idx)
                byte = draw(b, J, beta, uniforms(key_base, walker_ids[w], pass_index, ci))
                new = _spins_of(byte, 8)
                old = np.array([s[i] for i in idx], np.int64)
                dE = model.cell_energy(idx, b, new) - model.cell_energy(idx, b, old)
                if np.any(new != old):
                    changed[w] += 1
                for t, i in enumerate(idx):
                    s[i] = new[t]
                energy[w] += dE
    return changed
