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
    # replica 0: x_1 = (3, -1): x_1^T J x_1 = 2 * 3 * (-1) = -6, |x_1|^2 = 10, so the Rayleigh
    # quotient per spin is 6 / 20; signs (+, -): E = 2, E / n = 1; share 10 / (9 + 16 + 1); one flip of two
    np.testing.assert_allclose(f[0], [0.3, 1.0, 10.0 / 26.0, 0.5])
    # replica 1: x_1 = (0.5, 0.5): quadratic form 0.5, |x_1|^2 0.5 -> -0.5; signs (+, +): E = -2; share 1
    np.testing.assert_allclose(f[1], [-0.5, -1.0, 1.0, 0.5])
    np.testing.assert_array_equal(sig, [[1, -1], [1, 1]])
    # a zero state: quotient and share are 0 by definition, every sign reads +1
    z, sz = mlp.features(J, np.zeros((2, 1, 2)), np.array([[1, 1]], dtype=np.int8))
    np.testing.assert_array_equal(z[0], [0.0, -1.0, 0.0, 0.0])


def test_features_rayleigh_quotient_bounds():
    """The quotient lies in [-lambda_max, -lambda_min] / n, with the ends at
    the eigenvectors (placed in the first component)."""
    J = np.array([[0, 1, -1], [1, 0, 1], [-1, 1, 0]], dtype=np.float64)
    w, V = np.linalg.eigh(J)
    g = np.random.default_rng(5)
    x = g.standard_normal((3, 50, 3))
    x[:, 0, 0], x[:, 1, 0] = V[:, -1], V[:, 0]
    f, _ = mlp.features(J, x, np.ones((50, 3), dtype=np.int8))
    assert np.all(f[:, 0] >= -w[-1] / 3 - 1e-12) and np.all(f[:, 0] <= -w[0] / 3 + 1e-12)
    assert f[0, 0] == pytest.approx(-w[-1] / 3) and f[1, 0] == pytest.approx(-w[0] / 3)
    assert np.all((f[:, 2] >= 0) & (f[:, 2] <= 1))


def test_standardize_reference():
    g = np.random.default_rng(6)
    F = g.standard_normal((12, 5)) * 3 + 7
    F[4:8, 2] = 1.5  # a constant column in the second group standardizes to 0
    S = mlp.standardize(F, 4)
    for k in range(3):
        blk = S[4 * k:4 * k + 4]
        np.testing.assert_allclose(blk.mean(axis=0), 0.0, atol=1e-12)
        sd = blk.std(axis=0)
        assert np.all((np.abs(sd - 1) < 1e-12) | (sd == 0))
    assert not S[4:8, 2].any()
    # invariant under a shift and a positive scale of the group's values
    np.testing.assert_allclose(mlp.standardize(F * 2.5 - 4, 4), S, atol=1e-12)


def test_select_top_reference_against_brute_force():
    g = np.random.default_rng(7)
    s = np.round(g.standard_normal(40), 1)  # many ties
    s[3] = np.nan
    idx = mlp.select_top(s, 10, 4)
    for grp in range(4):
        blk = s[grp * 10:(grp + 1) * 10]
        key = np.where(np.isnan(blk), -np.inf, blk)
        chosen = set(idx[grp] - grp * 10)
        assert len(chosen) == 4 and list(idx[grp]) == sorted(idx[grp])
        # every chosen score beats every other, and among equal scores the lower index is chosen
        for i in chosen:
            for j in set(range(10)) - chosen:
                assert key[i] > key[j] or (key[i] == key[j] and i < j)


def test_bf16_network_reduces_to_exact_one_on_representable_values():
    # small integers everywhere: every layer input and activation is a bf16
    # value (integers up to 256), so the rounded network is the exact one
    g = np.random.default_rng(5)
    p = {"W1": g.integers(-1, 2, (128, 32)), "b1": g.integers(-2, 3, 128),
         "W2": g.integers(-1, 2, (128, 128)) / 8.0, "b2": g.standard_normal(128),
         "w3": g.standard_normal(128) * 0.1, "b3": np.array([0.3])}
    w = mlp.pack(p)
    x = g.integers(-3, 4, (9, 32)).astype(float)
    y = (g.random(9) < 0.5).astype(float)
    assert np.abs(x @ p["W1"].T + p["b1"]).max() <= 256
    for a, b in zip(mlp.forward_bf16(x, w), mlp.forward(x, w)):
        assert np.array_equal(a, b)
    assert np.array_equal(mlp.grad_bf16(x, y, w), mlp.grad(x, y, w))
    assert mlp.loss_bf16(x, y, w) == mlp.loss(x, y, w)


def test_bf16_network_hand_rounded_case():
    # one path x_0 -> h1_0 -> h2_0 -> z with unit weights:
    # x_0 = 1 + 2^-9 rounds to 1 (half an ulp, ties to even);
    # h1_0 = 1 + 2^-8 + 2^-10 rounds to 1 + 2^-7 (five eighths of an ulp up)
    p = {name: np.zeros(shp) for name, shp in mlp.SHAPES}
    p["W1"][0, 0] = 1.0
    p["b1"][0] = 2.0 ** -8 + 2.0 ** -10
    p["W2"][0, 0] = 1.0
    p["w3"][0] = 1.0
    w = mlp.pack(p)
    x = np.zeros((1, 32))
    x[0, 0] = 1 + 2.0 ** -9
    z, h1, h2 = mlp.forward_bf16(x, w)
    assert h1[0, 0] == 1 + 2.0 ** -7 and h2[0, 0] == 1 + 2.0 ** -7 and z[0] == 1 + 2.0 ** -7
    assert mlp.forward(x, w)[0][0] == 1 + 2.0 ** -9 + 2.0 ** -8 + 2.0 ** -10
    y = np.array([1.0])
    gr = mlp.unpack(mlp.grad_bf16(x, y, w))
    dz = 1 / (1 + math.exp(-(1 + 2.0 ** -7))) - 1
    assert gr["b3"][0] == pytest.approx(dz, rel=1e-15)
    assert gr["w3"][0] == pytest.approx(dz * (1 + 2.0 ** -7), rel=1e-15)
    assert gr["W2"][0, 0] == pytest.approx(dz * (1 + 2.0 ** -7), rel=1e-15)  # the rounded h1
    assert gr["W1"][0, 0] == pytest.approx(dz, rel=1e-15)  # the rounded x: 1, not 1 + 2^-9
    assert gr["b1"][0] == pytest.approx(dz, rel=1e-15) and gr["b2"][0] == pytest.approx(dz, rel=1e-15)
    assert np.count_nonzero(mlp.grad_bf16(x, y, w)) == 6
