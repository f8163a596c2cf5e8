"""Pins of the cost-model MLP oracle (CPU): gradients against central finite
differences, Adam against its closed form, bf16 rounding against the bit
formulation of round-to-nearest-even and known values."""
import math

import numpy as np
import pytest

from oracle import mlp


def _data(seed, n=37):
    r = np.random.default_rng(seed)
    x = r.normal(size=(n, 16))
    t = r.normal(size=(n, 2))
    return x, t


@pytest.mark.parametrize("seed", range(3))
def test_gradients_match_central_differences(seed):
    p = mlp.init_params(seed)
    x, t = _data(seed)
    y, cache = mlp.forward(p, x)
    g = mlp.backward(p, y, t, cache)
    r = np.random.default_rng(100 + seed)
    h = 1e-6
    for name, shape in mlp.SHAPES:
        for _ in range(12):
            idx = tuple(int(r.integers(0, s)) for s in shape)
            old = p[name][idx]
            p[name][idx] = old + h
            lp = mlp.loss(mlp.forward(p, x)[0], t)
            p[name][idx] = old - h
            lm = mlp.loss(mlp.forward(p, x)[0], t)
            p[name][idx] = old
            num = (lp - lm) / (2 * h)
            assert abs(num - g[name][idx]) <= 1e-6 * max(1.0, abs(num)), (name, idx, num, g[name][idx])


def test_relu_masks_and_shapes():
    p = mlp.init_params(0)
    x, t = _data(0, n=5)
    y, (x0, z1, h1, z2, h2) = mlp.forward(p, x)
    assert y.shape == (5, 2) and h1.shape == (5, 64) and h2.shape == (5, 64)
    assert np.all(h1 >= 0) and np.all((h1 == 0) == (z1 <= 0))


def test_adam_first_step_closed_form():
    # after one step from zero state, m_hat = g and v_hat = g^2, so each
    # weight moves by -lr * g / (|g| + eps)
    p = mlp.init_params(1)
    x, t = _data(1)
    y, cache = mlp.forward(p, x)
    g = mlp.backward(p, y, t, cache)
    before = {k: v.copy() for k, v in p.items()}
    st = {}
    mlp.adam_step(p, g, st, lr=1e-3)
    for name, _ in mlp.SHAPES:
        want = before[name] - 1e-3 * g[name] / (np.abs(g[name]) + 1e-8)
        assert np.allclose(p[name], want, rtol=0, atol=1e-15)


def test_adam_constant_gradient_moves_lr_per_step():
    # with a constant gradient, m_hat = g and v_hat = g^2 at every step
    p = {k: np.zeros(s) for k, s in mlp.SHAPES}
    g = {k: np.full(s, 0.5) for k, s in mlp.SHAPES}
    st = {}
    for _ in range(5):
        mlp.adam_step(p, g, st, lr=0.01)
    for name, _ in mlp.SHAPES:
        assert np.allclose(p[name], -5 * 0.01 * 0.5 / (0.5 + 1e-8))


def test_training_reduces_loss():
    r = np.random.default_rng(5)
    x = r.normal(size=(256, 16))
    w = r.normal(size=(16, 2))
    t = np.tanh(x @ w)
    p = mlp.init_params(7)
    st = {}
    l0 = mlp.loss(mlp.forward(p, x)[0], t)
    for _ in range(200):
        y, c = mlp.forward(p, x)
        mlp.adam_step(p, mlp.backward(p, y, t, c), st, lr=3e-3)
    assert mlp.loss(mlp.forward(p, x)[0], t) < 0.25 * l0


def _rne_bits(x32: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even by the bit formulation: add 0x7FFF plus the
    lowest kept bit, then truncate (finite inputs)."""
    b = x32.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    return (((b + 0x7FFF + lsb) >> 16) << 16).astype(np.uint32).view(np.float32)


def test_bf16_known_values():
    assert mlp.bf16_round_scalar(1.0) == 1.0
    assert mlp.bf16_round_scalar(1.0 + 2 ** -8) == 1.0                  # tie -> even (down)
    assert mlp.bf16_round_scalar(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6    # tie -> even (up)
    assert mlp.bf16_round_scalar(1.0 + 1.5 * 2 ** -8) == 1.0 + 2 ** -7
    assert mlp.bf16_round_scalar(-(1.0 + 2 ** -8)) == -1.0
    assert mlp.bf16_round_scalar(float(np.finfo(np.float32).max)) == math.inf
    assert mlp.bf16_round_scalar(0.0) == 0.0


def test_bf16_matches_bit_formulation_on_sample():
    r = np.random.default_rng(11)
    bits = r.integers(0, 2 ** 32, size=20000, dtype=np.uint64).astype(np.uint32)
    # keep finite values; add every exponent's exact ties and near-ties
    ties = (np.arange(0, 255, dtype=np.uint32) << 23) | 0x8000
    bits = np.concatenate([bits, ties, ties | 0x10000, ties + 1, ties - 1])
    x = bits.view(np.float32)
    x = x[np.isfinite(x)]
    want = _rne_bits(x.copy())
    got = np.array([mlp.bf16_round_scalar(float(v)) for v in x], dtype=np.float64)
    fin = np.isfinite(want)
    assert np.array_equal(got[fin], want[fin].astype(np.float64))
    assert np.all(np.isinf(got[~fin]))
