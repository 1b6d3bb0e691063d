"""Oracle of the learned warm start (test infrastructure only).

Plain numpy, FP64 unless a step is defined in a narrower type.  This part is
not in the paper: it is the project's own definition of a per-atom network
that predicts a displacement before L-BFGS, written out so that the GPU
kernels can be checked against it.  Definitions:

* BF16: the upper 16 bits of an FP32 pattern after rounding to nearest, ties
  to even (a value that is already FP32 is rounded once; an FP64 value is
  first rounded to FP32).
* Features of atom i: its 16 nearest other atoms j of the same system by FP64
  squared distance ((dx*dx + dy*dy) + dz*dz, each operation rounded; ties to
  the lower index); the row is q_i, sigma_i - 3.5, 10 eps_i followed, per
  neighbour, by (x_j - x_i)/4, (y_j - y_i)/4, (z_j - z_i)/4, sqrt(d2)/4, q_j,
  sigma_j - 3.5, 10 eps_j (zeros for missing neighbours), then the atom's
  offset from the centroid c of its system, (x_i - c)/16 and |x_i - c|/16,
  and the system size n/4096 (c: coordinates summed one by one in atom
  order, divided by n); zeros up to 128 columns; every value rounded to BF16.
* Network: H1 = relu(X W1 + b1), H2 = relu(H1 W2 + b2), Y = H2 W3 + b3 with
  128 features, 128 hidden units and 16 outputs of which 0..2 are the
  displacement.  In "emulated" mode the operands of every product are
  BF16-rounded (weights, H1, H2, and in the backward pass dY, dH2, dH1), as
  the GPU does; otherwise everything is FP64 and the gradient is the exact
  derivative of the loss.
* Loss: mean over rows and the three used columns of (Y - T)^2.
* Adam: Kingma and Ba (2015), with bias correction.

Parameters are packed W1, b1, W2, b2, W3, b3 (row-major) in one vector.
"""
from __future__ import annotations

import numpy as np

NEIGHBORS = 16
FEATURES = 128
HIDDEN = 128
OUT_PAD = 16
SHAPES = (("W1", (FEATURES, HIDDEN)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
          ("W3", (HIDDEN, OUT_PAD)), ("b3", (OUT_PAD,)))
PARAM_COUNT = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    """Split the packed vector into a dict of arrays (views)."""
    out, off = {}, 0
    theta = np.asarray(theta)
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = theta[off:off + k].reshape(shape)
        off += k
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


# ------------------------------------------------------------------ BF16
def bf16_bits(x) -> np.ndarray:
    """BF16 bit patterns (uint16) of x (rounded to FP32 first), nearest-even."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    return ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)).astype(np.uint16)


def bf16_value(bits) -> np.ndarray:
    """FP64 value of BF16 bit patterns."""
    b = np.ascontiguousarray(np.asarray(bits, dtype=np.uint16)).astype(np.uint32) << np.uint32(16)
    return b.view(np.float32).astype(np.float64)


def bf16(x) -> np.ndarray:
    """x rounded to BF16, as FP64."""
    return bf16_value(bf16_bits(x))


# ------------------------------------------------------------- features
def neighbors_of(xyz, i: int, lo: int, hi: int) -> np.ndarray:
    """The (up to) 16 nearest atoms j != i in [lo, hi) by FP64 squared
    distance, ties to the lower index, as an index array, and their d2."""
    j = np.arange(lo, hi)
    j = j[j != i]
    d = xyz[j] - xyz[i]
    d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    order = np.lexsort((j, d2))[:NEIGHBORS]
    return j[order], d2[order]


def feature_row(xyz, q, sigma, eps, i: int, lo: int, hi: int):
    """(BF16 bit row [FEATURES], neighbour indices [NEIGHBORS] with -1 padding)."""
    js, d2 = neighbors_of(xyz, i, lo, hi)
    row = np.zeros(FEATURES)
    row[0], row[1], row[2] = q[i], sigma[i] - 3.5, 10.0 * eps[i]
    for k, (j, dd) in enumerate(zip(js, d2)):
        base = 3 + 7 * k
        row[base:base + 3] = (xyz[j] - xyz[i]) / 4.0
        row[base + 3] = np.sqrt(dd) / 4.0
        row[base + 4], row[base + 5], row[base + 6] = q[j], sigma[j] - 3.5, 10.0 * eps[j]
    n = hi - lo
    # a running sum in atom order (not numpy's pairwise reduction)
    c = np.array([np.add.accumulate(xyz[lo:hi, a])[-1] for a in range(3)]) / n
    off = xyz[i] - c
    base = 3 + 7 * NEIGHBORS
    row[base:base + 3] = off / 16.0
    row[base + 3] = np.sqrt((off[0] * off[0] + off[1] * off[1]) + off[2] * off[2]) / 16.0
    row[base + 4] = n / 4096.0
    nbr = np.full(NEIGHBORS, -1, dtype=np.int64)
    nbr[:len(js)] = js
    return bf16_bits(row), nbr


def features(xyz, q, sigma, eps, sys_first, rows=None):
    """Feature rows (BF16 bits [len(rows)][FEATURES]) and neighbour lists of
    the atoms ``rows`` (default: all) of concatenated systems."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    sys_first = np.asarray(sys_first)
    rows = np.arange(xyz.shape[0]) if rows is None else np.asarray(rows)
    fb = np.zeros((len(rows), FEATURES), dtype=np.uint16)
    nb = np.zeros((len(rows), NEIGHBORS), dtype=np.int64)
    for r, i in enumerate(rows):
        s = int(np.searchsorted(sys_first, i, side="right")) - 1
        fb[r], nb[r] = feature_row(xyz, q, sigma, eps, int(i), int(sys_first[s]), int(sys_first[s + 1]))
    return fb, nb


# -------------------------------------------------------------- network
def forward(theta, X, emulate: bool = True):
    """(Y [n][OUT_PAD], cache) of the network at feature values X [n][FEATURES]
    (FP64 values, e.g. bf16_value of the feature bits)."""
    p = unpack(theta)
    rnd = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    W1, W2, W3 = rnd(p["W1"]), rnd(p["W2"]), rnd(p["W3"])
    H1 = np.maximum(X @ W1 + p["b1"], 0.0)
    H1r = rnd(H1)
    H2 = np.maximum(H1r @ W2 + p["b2"], 0.0)
    H2r = rnd(H2)
    Y = H2r @ W3 + p["b3"]
    return Y, dict(X=X, W1=W1, W2=W2, W3=W3, H1=H1, H1r=H1r, H2=H2, H2r=H2r, Y=Y)


def loss(theta, X, T, emulate: bool = True) -> float:
    Y, _ = forward(theta, X, emulate)
    return float(np.mean((Y[:, :3] - T) ** 2))


def loss_grad(theta, X, T, emulate: bool = True):
    """(loss, packed gradient) for targets T [n][3]; backward through the
    three layers in reverse order with the BF16 rounding points listed in
    the module docstring."""
    Y, c = forward(theta, X, emulate)
    rnd = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    n = X.shape[0]
    E = Y[:, :3] - T
    L = float(np.mean(E ** 2))
    dY = np.zeros_like(Y)
    dY[:, :3] = 2.0 * E / (3.0 * n)
    dYr = rnd(dY)
    g = {"W3": c["H2r"].T @ dYr, "b3": dY.sum(axis=0)}
    dH2 = (dYr @ c["W3"].T) * (c["H2"] > 0)
    dH2r = rnd(dH2)
    g["W2"], g["b2"] = c["H1r"].T @ dH2r, dH2.sum(axis=0)
    dH1 = (dH2r @ c["W2"].T) * (c["H1"] > 0)
    dH1r = rnd(dH1)
    g["W1"], g["b1"] = X.T @ dH1r, dH1.sum(axis=0)
    return L, pack(g)


def adam(theta, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One bias-corrected Adam step; returns (theta, m, v) new arrays."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
