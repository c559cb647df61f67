"""Rank model and sketch generator of the oracle (FP64 / NumPy).

TEST INFRASTRUCTURE.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import or run this module.

Two pieces that the learned-rank variant of the shared-basis step needs:

* A counter-based Gaussian generator: SplitMix64 (Steele, Lea and Flood,
  "Fast splittable pseudorandom number generators", OOPSLA 2014) read at an
  arbitrary position of its sequence, two outputs turned into one normal
  deviate by the Box-Muller transform (Box and Muller, 1958, cosine branch).
  The sketch rows of a point p at level l come from one of two streams (far-field
  columns, fill-in columns) keyed by (seed, l, stream): entry (p, c) is deviate
  number c * N + p, so a point's rows do not depend on the box being sketched.

* The multilayer perceptron that predicts a box's rank: 16 features -> three
  hidden layers of width 64 with ReLU -> one linear output, trained with the
  mean squared error against log2(1 + k) by Adam (Kingma and Ba, "Adam: a method
  for stochastic optimization", ICLR 2015, Algorithm 1).  Parameters are one flat
  array in the order W1 (64 x 16, row-major), b1, W2 (64 x 64), b2, W3, b3,
  w4 (64), b4.  Forward, gradient and update are written out from the chain
  rule; the gradient is pinned by finite differences in the tests.
"""
from __future__ import annotations

import math

import numpy as np

NFEAT = 16
WIDTH = 64
SHAPES = [("W1", (WIDTH, NFEAT)), ("b1", (WIDTH,)), ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
          ("W3", (WIDTH, WIDTH)), ("b3", (WIDTH,)), ("w4", (WIDTH,)), ("b4", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)
ADAM_BETA1 = 0.9
ADAM_BETA2 = 0.999
ADAM_EPS = 1e-8

# ---------------------------------------------------------------------------
# SplitMix64 read at a position of its sequence, and Box-Muller deviates
# ---------------------------------------------------------------------------
GAMMA = 0x9E3779B97F4A7C15
MASK = (1 << 64) - 1


def mix64(z):
    """SplitMix64 output function (uint64 in, uint64 out; numpy arrays or int)."""
    if isinstance(z, (int, np.integer)):
        z = int(z) & MASK
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        return z ^ (z >> 31)
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def splitmix64_at(key, c):
    """Output number c (0-based) of the SplitMix64 stream whose state starts at
    ``key``: the state after c + 1 increments by GAMMA, passed through mix64."""
    if isinstance(c, (int, np.integer)):
        return mix64((int(key) + (int(c) + 1) * GAMMA) & MASK)
    c = np.asarray(c, dtype=np.uint64)
    with np.errstate(over="ignore"):
        s = np.uint64(int(key) & MASK) + (c + np.uint64(1)) * np.uint64(GAMMA)
    return mix64(s)


def box_key(seed: int, lev: int, box: int) -> int:
    """Key of the sketch of box ``box`` at level ``lev``."""
    return splitmix64_at(seed, (lev << 40) | box)


def gaussian(key: int, idx) -> np.ndarray:
    """Normal deviates number idx of a key: Box-Muller from outputs 2 idx
    (u1 in (0, 1]) and 2 idx + 1 (u2 in [0, 1))."""
    idx = np.asarray(idx, dtype=np.uint64)
    x1 = splitmix64_at(key, idx * np.uint64(2))
    x2 = splitmix64_at(key, idx * np.uint64(2) + np.uint64(1))
    u1 = ((x1 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (x2 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


STREAM_FAR = 0     # sketch rows of far-field columns
STREAM_FILL = 1    # sketch rows of fill-in columns
STREAM_BASE = 1 << 39


def point_rows(seed: int, lev: int, stream: int, points, npts: int, cols: int) -> np.ndarray:
    """Sketch rows of the given points (len(points) x cols): entry (r, c) is deviate
    number c * npts + points[r] of the key of (seed, level, stream).  The rows of a
    point do not depend on the box whose basis is sketched."""
    points = np.asarray(points, dtype=np.int64)
    if points.size == 0 or cols == 0:
        return np.zeros((points.size, cols))
    key = box_key(seed, lev, STREAM_BASE + stream)
    c = np.arange(cols, dtype=np.uint64)[None, :]
    idx = c * np.uint64(npts) + points.astype(np.uint64)[:, None]
    return gaussian(key, idx.reshape(-1)).reshape(points.size, cols)


# ---------------------------------------------------------------------------
# Multilayer perceptron
# ---------------------------------------------------------------------------
def unpack(theta: np.ndarray) -> dict:
    out, off = {}, 0
    for name, shp in SHAPES:
        sz = int(np.prod(shp))
        out[name] = theta[off:off + sz].reshape(shp)
        off += sz
    return out


def pack(parts: dict) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1)
                           for name, _ in SHAPES])


def init_weights(seed: int) -> np.ndarray:
    """He-normal hidden weights, N(0, 1/64) output weights, zero biases, from
    the Gaussian generator keyed by (seed, 0, 0)."""
    z = gaussian(box_key(seed, 0, 0), np.arange(NPARAM, dtype=np.uint64))
    parts, off = {}, 0
    for name, shp in SHAPES:
        sz = int(np.prod(shp))
        if name.startswith("b"):
            parts[name] = np.zeros(shp)
        else:
            fan_in = shp[1] if len(shp) == 2 else shp[0]
            gain = 2.0 if name != "w4" else 1.0
            parts[name] = (z[off:off + sz] * math.sqrt(gain / fan_in)).reshape(shp)
        off += sz
    return pack(parts)


def forward(theta: np.ndarray, X: np.ndarray, dtype=np.float64):
    """Outputs y (n,) and the hidden activations (for the gradient)."""
    p = {k: v.astype(dtype) for k, v in unpack(np.asarray(theta)).items()}
    a0 = np.asarray(X, dtype=dtype)
    z1 = a0 @ p["W1"].T + p["b1"]
    a1 = np.maximum(z1, 0)
    z2 = a1 @ p["W2"].T + p["b2"]
    a2 = np.maximum(z2, 0)
    z3 = a2 @ p["W3"].T + p["b3"]
    a3 = np.maximum(z3, 0)
    y = a3 @ p["w4"] + p["b4"][0]
    return y, (a0, a1, a2, a3)


def loss_and_grad(theta: np.ndarray, X: np.ndarray, t: np.ndarray):
    """L = mean (y - t)^2 and dL/dtheta, by the chain rule through the layers."""
    p = unpack(theta)
    y, (a0, a1, a2, a3) = forward(theta, X)
    n = y.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / n                      # dL/dy
    g = {"w4": a3.T @ dy, "b4": np.array([dy.sum()])}
    d3 = np.outer(dy, p["w4"]) * (a3 > 0)  # dL/dz3
    g["W3"] = d3.T @ a2
    g["b3"] = d3.sum(axis=0)
    d2 = (d3 @ p["W3"]) * (a2 > 0)
    g["W2"] = d2.T @ a1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"]) * (a1 > 0)
    g["W1"] = d1.T @ a0
    g["b1"] = d1.sum(axis=0)
    return loss, pack(g)


def adam_step(theta, m, v, g, step: int, lr: float):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = ADAM_BETA1 * m + (1.0 - ADAM_BETA1) * g
    v = ADAM_BETA2 * v + (1.0 - ADAM_BETA2) * g * g
    mhat = m / (1.0 - ADAM_BETA1 ** step)
    vhat = v / (1.0 - ADAM_BETA2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + ADAM_EPS), m, v


def train(theta, X, t, steps: int, lr: float):
    """Full-batch Adam; returns (theta, loss history)."""
    theta = np.array(theta, dtype=np.float64, copy=True)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    hist = []
    for s in range(1, steps + 1):
        loss, g = loss_and_grad(theta, X, t)
        hist.append(loss)
        theta, m, v = adam_step(theta, m, v, g, s, lr)
    return theta, hist


def predicted_rank(y: float) -> int:
    """k-hat from the output y ~ log2(1 + k): round(2^y - 1), at least 0."""
    return max(0, int(math.floor(2.0 ** float(y) - 1.0 + 0.5)))


def sketch_size(khat: int, oversample: int) -> int:
    """Columns of the sketch for a predicted rank: ceil(1.25 khat) + oversample."""
    return (5 * khat + 3) // 4 + oversample
