"""Cost-model MLP -- oracle side, TEST INFRASTRUCTURE ONLY.

The paper estimates predicate costs with a shallow feed-forward network
trained offline on logs (Section 4.2, "Shallow NNs" and "Estimated cost";
the defaults in Section 6 use ReLU and Adam).  The learned part here is a
16 -> 64 -> 64 -> 2 network (ReLU after both hidden layers, linear output)
over per-(block, predicate) features, predicting (pass rate, cost).

This module is the plain fp64 reference the GPU kernels are checked
against:
  * forward and backward written out layer by layer (no autograd);
  * loss = mean over rows and outputs of (y - t)^2;
  * Adam (Kingma and Ba, ICLR 2015): m = b1 m + (1-b1) g,
    v = b2 v + (1-b2) g^2, w -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps);
  * bf16 round-to-nearest-even of float32 values, done with exact
    arithmetic on the two neighbouring bf16 values (not a bit trick).
Weights are (W1 [16x64], b1 [64], W2 [64x64], b2 [64], W3 [64x2], b3 [2]),
row-major, used as x @ W + b.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Dict, List, Tuple

import numpy as np

SHAPES = [("W1", (16, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64, 2)), ("b3", (2,))]


def init_params(seed: int) -> Dict[str, np.ndarray]:
    """He-uniform weights, zero biases (fp64)."""
    r = np.random.default_rng(seed)
    p = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            lim = math.sqrt(6.0 / shape[0])
            p[name] = r.uniform(-lim, lim, size=shape)
        else:
            p[name] = np.zeros(shape)
    return p


def forward(p, x):
    """Returns (y, cache) with every intermediate, in fp64."""
    z1 = x @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["W3"] + p["b3"]
    return y, (x, z1, h1, z2, h2)


def loss(y, t) -> float:
    return float(np.mean((y - t) ** 2))


def backward(p, y, t, cache):
    """Gradients of the mean squared error with respect to every parameter."""
    x, z1, h1, z2, h2 = cache
    n = y.shape[0]
    dy = 2.0 * (y - t) / (n * y.shape[1])
    g = {}
    g["W3"] = h2.T @ dy
    g["b3"] = dy.sum(axis=0)
    dh2 = dy @ p["W3"].T
    dz2 = dh2 * (z2 > 0)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"].T
    dz1 = dh1 * (z1 > 0)
    g["W1"] = x.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return g


def adam_step(p, g, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; state holds m, v and the step count t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for name, _ in SHAPES:
        m = state.setdefault("m_" + name, np.zeros_like(p[name]))
        v = state.setdefault("v_" + name, np.zeros_like(p[name]))
        m[...] = b1 * m + (1 - b1) * g[name]
        v[...] = b2 * v + (1 - b2) * g[name] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[name] -= lr * mh / (np.sqrt(vh) + eps)


# ------------------------------------------------------------------ bf16

def _f32_bits(x: float) -> int:
    return int(np.array([x], dtype=np.float32).view(np.uint32)[0])


def _bits_f32(b: int) -> float:
    return float(np.array([b], dtype=np.uint32).view(np.float32)[0])


def bf16_round_scalar(x: float) -> float:
    """Nearest bf16 value of a float32, ties to the even mantissa, chosen by
    comparing exact distances to the two bf16 neighbours (as if the exponent
    were unbounded; a result beyond the largest bf16 overflows to inf)."""
    xf = float(np.float32(x))
    if math.isnan(xf) or math.isinf(xf):
        return xf
    bits = _f32_bits(xf)
    lo_bits = bits & 0xFFFF0000           # truncation toward zero
    lo = _bits_f32(lo_bits)
    if lo_bits == bits:
        return lo
    hi_bits = lo_bits + 0x10000           # next bf16 away from zero
    if (hi_bits & 0x7FFFFFFF) == 0x7F800000:
        hi_exact = Fraction(2) ** 128 * (1 if xf > 0 else -1)
        hi = math.copysign(math.inf, xf)
    else:
        hi = _bits_f32(hi_bits)
        hi_exact = Fraction(hi)
    ex = Fraction(xf)
    dl, dh = abs(ex - Fraction(lo)), abs(hi_exact - ex)
    if dl < dh:
        return lo
    if dh < dl:
        return hi
    return lo if ((lo_bits >> 16) & 1) == 0 else hi


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Elementwise bf16 rounding (as float64 values)."""
    flat = np.asarray(a, dtype=np.float64).ravel()
    out = np.array([bf16_round_scalar(float(v)) for v in flat])
    return out.reshape(np.shape(a))
