"""Pins of the FP64 network reference (finite differences, closed forms)."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp


def rand_w(seed, scale=0.3):
    return np.random.default_rng(seed).standard_normal(mlp.PARAMS) * scale


def test_param_count_and_layout():
    assert mlp.PARAMS == 20865
    w = np.arange(mlp.PARAMS, dtype=np.float64)
    p = mlp.unpack(w)
    assert p["W1"][1, 0] == 32 and p["b1"][0] == 4096 and p["W2"][0, 0] == 4224
    assert np.array_equal(mlp.pack(p), w)


def test_gradient_matches_central_differences():
    g = np.random.default_rng(1)
    x = g.standard_normal((7, 32))
    y = (g.random(7) < 0.5).astype(float)
    w = rand_w(2)
    ga = mlp.grad(x, y, w)
    idx = np.concatenate([g.choice(mlp.PARAMS, 300, replace=False), [mlp.PARAMS - 1, 4096, 20736]])
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (mlp.loss(x, y, wp) - mlp.loss(x, y, wm)) / (2 * h)
        assert ga[i] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_closed_forms():
    w = np.zeros(mlp.PARAMS)
    w[-1] = 0.7  # only the output bias
    x = np.ones((4, 32))
    y = np.array([1.0, 0.0, 1.0, 1.0])
    z, h1, h2 = mlp.forward(x, w)
    assert np.all(z == 0.7) and not h1.any() and not h2.any()
    assert mlp.loss(x, y, w) == pytest.approx(math.log1p(math.exp(0.7)) - 0.75 * 0.7, rel=1e-14)
    gr = mlp.grad(x, y, w)
    assert gr[-1] == pytest.approx(1 / (1 + math.exp(-0.7)) - 0.75, rel=1e-14)
    assert not gr[:-1].any()  # dead ReLUs pass no gradient
    assert mlp.loss(x, np.full(4, 0.3), np.zeros(mlp.PARAMS)) == pytest.approx(math.log(2), rel=1e-14)


def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -0.01, 0.0, 2e-5])
    w, m, v = mlp.adam(np.zeros(4), np.zeros(4), np.zeros(4), g, lr=0.1, t=1)
    np.testing.assert_allclose(w[[0, 1]], [-0.1, 0.1], rtol=1e-6)
    assert w[2] == 0.0
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_bf16_rounding_reference():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -9, -2.5, 3.0e-3], dtype=np.float32)
    got = mlp.bf16_round(vals)
    # ties to even: 1 + 2^-8 -> 1, 1 + 3 2^-8 -> 1 + 2^-6... (8-bit significand)
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == 1 + 2 ** -6 and got[3] == 1.0 and got[4] == -2.5
    assert abs(got[5] - 3.0e-3) <= 3.0e-3 * 2 ** -8


def test_features_reference_small_case():
    J = np.array([[0, 1], [1, 0]], dtype=np.int8)
    x = np.zeros((2, 2, 2))
    x[0, 0] = [3.0, 4.0]
    x[1, 0] = [-1.0, 0.0]
    x[:, 1, 0] = [0.5, 0.5]
    prev = np.array([[1, 1], [1, -1]], dtype=np.int8)
    f, sig = mlp.features(J, x, prev)
    # replica 0: u0 = (0.6, 0.8), u1 = (-1, 0): E_hs = -2 (-0.6) = 1.2; signs (+, -): E = 2
    np.testing.assert_allclose(f[0], [0.6, 1.0, 3.0, 0.5])
    np.testing.assert_allclose(f[1], [-1.0, -1.0, 0.5, 0.5])
    np.testing.assert_array_equal(sig, [[1, -1], [1, 1]])
