"""Host side of the XY-machine check (Fig. 2, parameter paragraph): the
continuous ground-state minimizer against closed forms, a brute-force grid,
the spectral bound, the Ising ground state, and first- and second-order
optimality; the machine's inputs against the thresholds they encode."""
import math

import numpy as np
import pytest

import oracle
from paper_2308_02329_amd import stats, synth, xy


def test_closed_forms():
    n = 9
    ferro = np.ones((n, n)) - np.eye(n)
    assert xy.xy_ground(ferro, starts=8)[0] == pytest.approx(-n * (n - 1), abs=1e-9)
    # frustrated antiferromagnetic triangle: 120-degree state, 6 cos(2 pi / 3) = -3 (Ising: -2)
    tri = -(np.ones((3, 3)) - np.eye(3))
    e, th = xy.xy_ground(tri, starts=8)
    assert e == pytest.approx(-3.0, abs=1e-9)
    d = np.mod(np.diff(np.r_[th, th[0]]), 2 * math.pi)
    np.testing.assert_allclose(np.minimum(d, 2 * math.pi - d), 2 * math.pi / 3, atol=1e-5)
    # two spins: -2 |J|
    assert xy.xy_ground(np.array([[0.0, -1.5], [-1.5, 0.0]]), starts=4)[0] == pytest.approx(-3.0, abs=1e-9)
    # unfrustrated (bipartite) graph: the XY ground state is collinear, equal to the Ising one
    ring = np.zeros((6, 6))
    for p in range(6):
        ring[p, (p + 1) % 6] = ring[(p + 1) % 6, p] = -1.0
    assert xy.xy_ground(ring, starts=8)[0] == pytest.approx(oracle.bruteforce_gs(ring)[0], abs=1e-9)


def test_three_spins_against_a_grid():
    g = np.random.default_rng(5)
    for _ in range(3):
        J = g.normal(size=(3, 3))
        J = J + J.T
        np.fill_diagonal(J, 0.0)
        k = 2 * math.pi * np.arange(1440) / 1440  # quarter-degree grid, theta_0 = 0 (rotation invariance)
        t1, t2 = np.meshgrid(k, k, indexing="ij")
        th = np.stack([np.zeros_like(t1), t1, t2], axis=-1)
        grid = xy.xy_energy(J, th).min()
        e = xy.xy_ground(J, starts=16)[0]
        # the grid is at most (pi / 1440)^2 / 2 * sum |J| above the minimum
        assert grid - (math.pi / 1440) ** 2 * np.abs(J).sum() <= e <= grid + 1e-12


@pytest.mark.parametrize("n", [6, 10, 14])
def test_bounds_and_optimality(n):
    J = stats.graph(n, 3, 77).astype(np.float64) if n >= 10 else synth.sk_pm1(n, 77).astype(np.float64)
    e, th = xy.xy_ground(J, starts=32, seed=4)
    lam = np.linalg.eigvalsh(J)[-1]
    assert -n * lam - 1e-9 <= e <= oracle.bruteforce_gs(J)[0] + 1e-9  # spectral bound <= E_XY <= E_Ising
    # stationary: analytic gradient vanishes; and it matches finite differences
    _, gr = xy._energy_grad(th[None, :].ravel(), J, 1, n)
    assert np.abs(gr).max() < 1e-5
    t0 = synth.rng(9, n).uniform(-3, 3, n)
    _, g0 = xy._energy_grad(t0, J, 1, n)
    h = 1e-6
    fd = np.array([(xy.xy_energy(J, t0 + h * np.eye(n)[p]) - xy.xy_energy(J, t0 - h * np.eye(n)[p])) / (2 * h)
                   for p in range(n)])
    np.testing.assert_allclose(g0, fd, rtol=1e-6, atol=1e-7)
    # a minimum: the Hessian (finite differences of the gradient) has no negative direction
    H = np.array([(xy._energy_grad(th + h * np.eye(n)[p], J, 1, n)[1] -
                   xy._energy_grad(th - h * np.eye(n)[p], J, 1, n)[1]) / (2 * h) for p in range(n)])
    assert np.linalg.eigvalsh((H + H.T) / 2)[0] > -1e-5
    # global rotation leaves the energy unchanged
    assert xy.xy_energy(J, th + 0.7) == pytest.approx(e, abs=1e-9)


def test_machine_inputs():
    J = stats.graph(20, 0, 1)
    jmag, h, A0, alpha = xy.machine_inputs(J, 5, 100, (0.1, 0.5), 1, 0)
    assert h.shape == (10,) and A0.shape == (20, 10, 2) and alpha.shape == (100, 2) and np.all(alpha == 1.0)
    hth = xy.h_threshold()
    assert (1 - xy.LOSS) * (1 - xy.B) * math.exp(xy.KL * hth) == pytest.approx(1.0, rel=1e-12)
    np.testing.assert_allclose(h[::5], np.float32(hth * np.array([1.1, 1.5])))
    assert xy.KL == 1e-3 and xy.BB2 == 25.0
    with pytest.raises(ValueError, match="symmetric"):
        xy.xy_ground(np.array([[0.0, 1.0], [0.0, 0.0]]))
