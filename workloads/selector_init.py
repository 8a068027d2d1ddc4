"""Seeded initial weights of the point-scoring network: random inputs of its
training, shared by the library's trainer and the FP64 reference (no method
arithmetic here).

Packed layout (ISDF_MLP_NPARAM = 5313 values): W1[64][16], b1[64],
W2[64][64], b2[64], w3[64], b3.  Weights He-normal (standard deviation
sqrt(2 / fan_in)), biases zero.
"""
from __future__ import annotations

import numpy as np

_NF, _NH = 16, 64


def initial_weights(seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    w1 = _NH * _NF
    w2 = _NH * _NH
    th = np.zeros(w1 + _NH + w2 + _NH + _NH + 1)
    th[0:w1] = rng.standard_normal(w1) * np.sqrt(2.0 / _NF)
    o2 = w1 + _NH
    th[o2:o2 + w2] = rng.standard_normal(w2) * np.sqrt(2.0 / _NH)
    o3 = o2 + w2 + _NH
    th[o3:o3 + _NH] = rng.standard_normal(_NH) * np.sqrt(2.0 / _NH)
    return th
