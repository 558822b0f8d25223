"""Seeded initial weights of the learned cell proposal (an input, like the couplings).

Layout of the flat float32 parameter vector (19,848 values), in this order:
  W1 [128][17], b1 [128], W2 [128][128], b2 [128], W3 [8][128], b3 [8]
Weights are uniform in +-1/sqrt(fan_in), biases 0.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 17, 128, 8
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def initial_params(seed: int = 12345) -> np.ndarray:
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in SHAPES:
        if name.startswith("W"):
            bound = 1.0 / np.sqrt(shape[1])
            parts.append(rng.uniform(-bound, bound, size=shape).ravel())
        else:
            parts.append(np.zeros(shape).ravel())
    return np.concatenate(parts).astype(np.float32)


def unpack(flat):
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(flat[o:o + n]).reshape(shape)
        o += n
    return out
