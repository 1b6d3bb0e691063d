"""Inputs of the learned warm start's network on which every operation is
exact (test data only, no kernel arithmetic here).

Sparse weights of a few signed powers of two, features in {-1, 0, 1} and
targets chosen so that the loss gradient is a small multiple of 2^-8: every
product and sum stays a short dyadic fraction, so each BF16 rounding point
and each FP32 sum, in any order, is exact.  On such inputs a correct GPU
forward and backward pass must reproduce the oracle element by element
(the bias gradient of the output layer sums the unrounded dY, whose FP32
scaling by 2/(3n) may differ in the last bits)."""
from __future__ import annotations

import numpy as np

from oracle import learn as OL


def exact_case(rows: int, seed: int):
    """(theta float32 [param_count], feature BF16 bits [rows][128], T float32
    [rows][3]); rows must be even."""
    assert rows % 2 == 0
    rng = np.random.default_rng(seed)
    F, H, O = OL.FEATURES, OL.HIDDEN, OL.OUT_PAD
    X = np.zeros((rows, F))
    for r in range(rows):
        cols = rng.choice(F, size=8, replace=False)
        X[r, cols] = rng.choice([-1.0, 1.0], size=8)
    W1 = np.zeros((F, H))
    for h in range(H):
        W1[rng.choice(F, size=3, replace=False), h] = rng.choice([-0.5, -0.25, 0.25, 0.5], size=3)
    b1 = rng.choice([-0.25, 0.0, 0.25, 0.5], size=H)
    p1, p2 = rng.permutation(H), rng.permutation(H)
    while np.any(p1 == p2):
        p2 = rng.permutation(H)
    W2 = np.zeros((H, H))
    W2[np.arange(H), p1] = rng.choice([-0.5, 0.5, 1.0], size=H)
    W2[np.arange(H), p2] = rng.choice([-1.0, -0.5, 0.5], size=H)
    b2 = rng.choice([-0.125, 0.0, 0.125, 0.25], size=H)
    W3 = np.zeros((H, O))
    for c in range(O):
        W3[rng.choice(H, size=4, replace=False), c] = rng.choice([-1.0, -0.5, 0.5, 1.0], size=4)
    b3 = rng.choice([-0.0625, 0.0, 0.0625], size=O)
    theta = OL.pack(dict(W1=W1, b1=b1, W2=W2, b2=b2, W3=W3, b3=b3))
    Y, _ = OL.forward(theta, X, emulate=False)
    m = rng.integers(-8, 9, size=(rows, 3))
    # E = Y - T = (3 rows / 2) m 2^-8, so that dY = 2 E / (3 rows) = m 2^-8
    T = Y[:, :3] - (1.5 * rows) * m * 2.0 ** -8
    return theta.astype(np.float32), OL.bf16_bits(X), T.astype(np.float32)
