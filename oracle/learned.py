"""Oracle of the learned cell proposal -- TEST INFRASTRUCTURE ONLY.

Plain numpy, FP64 unless stated.  Only tests/, the smoke check and bench.py's
CPU baseline may import it.

Model (a reading of the learned-proposal extension; the 2010 paper has no
learned part): a unit cell of 8 spins (one K4,4 cell of one slice) is
re-proposed jointly from its boundary fields b_k = h_k + sum_{j outside the
cell} J_kj s_j and the walker's inverse temperature:
  x = [0]*8 ++ b/8 ++ [beta]            (17 inputs; the 8 current-spin slots
                                         stay zero: an independence proposal
                                         given the boundary)
  H1 = relu(W1 x + b1), H2 = relu(W2 H1 + b2), l = W3 H2 + b3
  q(s'|b, beta) = prod_k sigmoid(l_k)^[s'_k=+1] sigmoid(-l_k)^[s'_k=-1]
and accepted with the exact Metropolis-Hastings probability
  min(1, exp(-beta dE) q(s) / q(s'))    (cost function of Section 1),
dE = E_c(s') - E_c(s), E_c(s) = -sum_k b_k s_k - sum_{in-cell edges} J s s.
Training minimises the mean of -log q(s_cell | b, beta) over cells drawn from
the plain chain.  Uniforms come from Philox4x32-10 (Salmon et al., SC'11):
key (key mod 2^32, key div 2^32), counters (cell, walker, pass, j) for blocks
j = 0, 1, 2; the words of blocks 0 and 1 are the 8 proposal uniforms, word 0
of block 2 the acceptance uniform.
"""
from __future__ import annotations

import numpy as np

from gen.mlp import SHAPES

# ----------------------------------------------------------------- Philox4x32
_M0, _M1 = 0xD2511F53, 0xCD9E8D57          # round multipliers
_W0, _W1 = 0x9E3779B9, 0xBB67AE85          # key schedule (Weyl) increments
_MASK = (1 << 32) - 1


def philox4x32(counter, key, rounds=10):
    """One Philox4x32 block: four 32-bit words for a 128-bit counter and a 64-bit key.
    A round multiplies words 0 and 2 by the two constants (full 64-bit products),
    then the new words are (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key
    advances by the Weyl increments between rounds."""
    x = [int(c) & _MASK for c in counter]
    k0, k1 = int(key[0]) & _MASK, int(key[1]) & _MASK
    for r in range(rounds):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0, p1 = _M0 * x[0], _M1 * x[2]
        x = [(p1 >> 32) ^ x[1] ^ k0, p1 & _MASK, (p0 >> 32) ^ x[3] ^ k1, p0 & _MASK]
    return x


def cell_uniforms(key_base, walker, pass_index, cell):
    """The 9 uniforms of one cell proposal: u[0..7] for the proposed spins, u[8] for
    the acceptance; 32-bit integers (uniform = u * 2^-32)."""
    key = (key_base & _MASK, (key_base >> 32) & _MASK)
    w = []
    for j in range(3):
        w += philox4x32((cell, walker, pass_index, j), key)
    return w[:9]


# ----------------------------------------------------------------- MLP
def unpack(flat):
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(flat[o:o + n], np.float64).reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SHAPES])


def features(b, beta):
    """Inputs [n, 17] from boundary fields b [n, 8] and inverse temperatures [n]."""
    b = np.asarray(b, np.float64)
    n = b.shape[0]
    x = np.zeros((n, 17))
    x[:, 8:16] = b / 8.0
    x[:, 16] = beta
    return x


def forward(p, x):
    """FP64 forward: returns logits and the activations for backward."""
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    logits = h2 @ p["W3"].T + p["b3"]
    return logits, (x, z1, h1, z2, h2)


def log_sigmoid(v):
    return -np.logaddexp(0.0, -v)


def nll(logits, y):
    """Mean over rows of -log q(y), y [n, 8] in {0, 1} (1 means spin +1)."""
    lq = y * log_sigmoid(logits) + (1 - y) * log_sigmoid(-logits)
    return -lq.sum(1).mean()


def backward(p, cache, logits, y):
    """Gradient of `nll` with respect to every parameter (FP64)."""
    x, z1, h1, z2, h2 = cache
    n = x.shape[0]
    dl = (1.0 / (1.0 + np.exp(-logits)) - y) / n
    g = {"W3": dl.T @ h2, "b3": dl.sum(0)}
    dh2 = dl @ p["W3"]
    dz2 = dh2 * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (z1 > 0)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(0)
    return g


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a32 = np.asarray(a, np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(p, x):
    """Mirror of the GPU arithmetic: bf16 inputs, weights and activations, fp32 sums."""
    f32 = np.float32
    X = bf16(x).astype(f32)
    z1 = X @ bf16(p["W1"]).astype(f32).T + p["b1"].astype(f32)
    h1 = bf16(np.maximum(z1, 0)).astype(f32)
    z2 = h1 @ bf16(p["W2"]).astype(f32).T + p["b2"].astype(f32)
    h2 = bf16(np.maximum(z2, 0)).astype(f32)
    logits = h2 @ bf16(p["W3"]).astype(f32).T + p["b3"].astype(f32)
    return logits.astype(np.float64), (X, z1, h1, z2, h2)


def backward_bf16(p, cache, logits, y):
    """Mirror of the GPU backward: bf16 operands of every product, fp32 sums."""
    f32 = np.float32
    X, z1, h1, z2, h2 = cache
    n = X.shape[0]
    dl = ((1.0 / (1.0 + np.exp(-logits)) - y) / n).astype(f32)
    dlb = bf16(dl).astype(f32)
    g = {"W3": dlb.T @ h2, "b3": dl.sum(0)}
    dz2 = bf16((dlb @ bf16(p["W3"]).astype(f32)) * (z2 > 0)).astype(f32)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dz1 = bf16((dz2 @ bf16(p["W2"]).astype(f32)) * (z1 > 0)).astype(f32)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(0)
    return {k: v.astype(np.float64) for k, v in g.items()}


class Adam:
    """Adam (Kingma & Ba 2015) with bias correction."""

    def __init__(self, flat, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.w = np.asarray(flat, np.float64).copy()
        self.m = np.zeros_like(self.w)
        self.v = np.zeros_like(self.w)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, grad_flat):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * grad_flat
        self.v = self.b2 * self.v + (1 - self.b2) * grad_flat ** 2
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        self.w = self.w - self.lr * mh / (np.sqrt(vh) + self.eps)
        return self.w


# ----------------------------------------------------------------- cells
def cell_colour(system, m, y, x):
    """Cells of one colour share no edge: (y + x + m) mod 2, except that on a ring of
    odd length the last slice takes colours 2 and 3."""
    if system.ring and system.M % 2 == 1 and m == system.M - 1:
        return 2 + (y + x) % 2
    return (y + x + m) % 2


def n_colours(system):
    return 4 if (system.ring and system.M % 2 == 1) else 2


class CellModel:
    """Per-spin neighbour lists of a Chimera system (full graph), for cell moves."""

    def __init__(self, system):
        assert system.L > 0, "cell moves need a Chimera template"
        self.system = system
        N, u, v, J, h = system.expand()
        self.N, self.h = N, h.astype(np.int64)
        self.nbr = [[] for _ in range(N)]
        for a, b, j in zip(u, v, J):
            self.nbr[a].append((int(b), int(j)))
            self.nbr[b].append((int(a), int(j)))
        L = system.L
        self.cells = [(m, y, x) for m in range(system.M) for y in range(L) for x in range(L)]

    def cell_spins(self, m, y, x):
        S, L = self.system.S, self.system.L
        base = m * S + (y * L + x) * 8
        return list(range(base, base + 8))

    def boundary(self, s, idx):
        inside = set(idx)
        b = []
        for i in idx:
            b.append(self.h[i] + sum(j * s[k] for k, j in self.nbr[i] if k not in inside))
        return np.array(b, np.int64)

    def cell_energy(self, idx, b, sc):
        """E_c = -sum b_k s_k - sum over in-cell edges J s s, for cell spins sc (+-1)."""
        pos = {i: t for t, i in enumerate(idx)}
        e = -int(np.dot(b, sc))
        for t, i in enumerate(idx):
            for k, j in self.nbr[i]:
                if k in pos and k > i:
                    e -= j * sc[t] * sc[pos[k]]
        return e


def learned_pass(model, spins, energy, betas, params, key_base, walker_ids, pass_index, forward_fn=None):
    """One pass of cell proposals over every walker of one system (FP64).

    spins [K, N] (+-1, modified in place), energy [K] (modified), betas [K] (each
    walker's current inverse temperature).  Colours in order; inside a colour the
    cells are independent.  Returns accepted moves per walker."""
    p = unpack(params) if not isinstance(params, dict) else params
    fwd = forward if forward_fn is None else forward_fn
    sysm = model.system
    L = sysm.L
    acc = np.zeros(len(spins), np.int64)
    for colour in range(n_colours(sysm)):
        for w in range(len(spins)):
            s = spins[w]
            beta = float(betas[w])
            for ci, (m, y, x) in enumerate(model.cells):
                if cell_colour(sysm, m, y, x) != colour:
                    continue
                idx = model.cell_spins(m, y, x)
                b = model.boundary(s, idx)
                logits, _ = fwd(p, features(b[None, :], [beta]))
                logits = logits[0]
                u = cell_uniforms(key_base, walker_ids[w], pass_index, ci)
                prob = 1.0 / (1.0 + np.exp(-logits))
                new = np.array([1 if u[k] * 2.0 ** -32 < prob[k] else -1 for k in range(8)], np.int64)
                old = np.array([s[i] for i in idx], np.int64)
                lq = lambda sc: float(sum(log_sigmoid(logits[k] if sc[k] > 0 else -logits[k])  # noqa: E731
                                          for k in range(8)))
                dE = model.cell_energy(idx, b, new) - model.cell_energy(idx, b, old)
                log_alpha = -beta * dE + lq(old) - lq(new)
                if log_alpha >= 0 or u[8] * 2.0 ** -32 < np.exp(log_alpha):
                    for t, i in enumerate(idx):
                        s[i] = new[t]
                    energy[w] += dE
                    acc[w] += 1
    return acc


def collect(model, spins, betas, cells_per_walker=None, rng=None):
    """Training rows (x [n,17], y [n,8]) from walkers' current spins."""
    xs, ys = [], []
    for w in range(len(spins)):
        chosen = model.cells if cells_per_walker is None else \
            [model.cells[i] for i in rng.choice(len(model.cells), cells_per_walker, replace=False)]
        for (m, y_, x_) in chosen:
            idx = model.cell_spins(m, y_, x_)
            b = model.boundary(spins[w], idx)
            xs.append(features(b[None, :], [betas[w]])[0])
            ys.append([(1 if spins[w][i] > 0 else 0) for i in idx])
    return np.array(xs), np.array(ys, np.float64)
