"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each uses an independent
computation (exhaustive enumeration in numpy, closed forms, eigen-
decompositions, symmetries, the literal round-trip map of Eq. (2)), chosen so
that a dropped term, a wrong sign, a wrong index or a transposed operand in
the oracle fails at least one of them.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2308_02329_amd import synth


def enum_energies(J):
    """All 2^n Ising energies by dense enumeration (independent of the
    oracle's Gray-code search): E = -sigma^T J sigma."""
    n = J.shape[0]
    S = np.array(list(itertools.product([-1.0, 1.0], repeat=n)))
    return -np.einsum("ip,pq,iq->i", S, J.astype(np.float64), S), S


# ---------------------------------------------------------------- P1 energies
@pytest.mark.parametrize("n,kind,seed", [(1, "sk", 0), (2, "sk", 1), (5, "sk", 2), (8, "sk", 3),
                                         (10, "er", 4), (9, "gauss", 5), (12, "sk", 6)])
def test_bruteforce_gs_matches_enumeration(n, kind, seed):
    J = {"sk": synth.sk_pm1, "er": synth.er_pm1, "gauss": synth.gaussian_j}[kind](n, 90, seed)
    if kind == "er" and n < 2:
        pytest.skip()
    E, S = enum_energies(J)
    egs, best = oracle.bruteforce_gs(J)
    assert egs == pytest.approx(E.min(), abs=1e-9)
    # the returned configuration attains it, according to an independent formula
    bs = best.astype(np.float64)
    assert -bs @ J.astype(np.float64) @ bs == pytest.approx(egs, abs=1e-9)


def test_ising_energy_definition_and_symmetry():
    J = synth.sk_pm1(11, 91, 0)
    E, S = enum_energies(J)
    sig = S.astype(np.int8)
    Eo = oracle.ising_energy(J, sig)
    np.testing.assert_array_equal(Eo, E)
    # full double sum over (p, q): E = -2 sum_{p<q} J_pq s_p s_q
    iu = np.triu_indices(11, 1)
    half = np.array([-(2.0 * (J[iu] * s[iu[0]] * s[iu[1]]).sum()) for s in S[:64]])
    np.testing.assert_array_equal(Eo[:64], half)
    # global spin flip leaves E unchanged
    np.testing.assert_array_equal(oracle.ising_energy(J, -sig[:64]), Eo[:64])
    # +-1 couplings with the double sum: every energy is even and all energy gaps are multiples of 4
    assert np.all(Eo % 2 == 0)
    assert np.all((Eo - Eo.min()) % 4 == 0)


def test_ising_energy_nonzero_diagonal_counts_once():
    # the definition sums over all (p, q), including p = q
    J = np.array([[3.0, 1.0], [1.0, -2.0]])
    s = np.array([[1, -1]], dtype=np.int8)
    assert oracle.ising_energy(J, s)[0] == -(3.0 - 1.0 - 1.0 - 2.0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_anneal_gs_reaches_exhaustive_gs(seed):
    J = synth.sk_pm1(18, 92, seed)
    egs, _ = oracle.bruteforce_gs(J)
    esa, s = oracle.anneal_gs(J, sweeps=400, restarts=32, seed=seed)
    assert esa == egs
    assert -s.astype(float) @ J @ s.astype(float) == esa


# --------------------------------------------------------------- readout
def test_readout_sign_convention():
    x = np.zeros((4, 2, 2))
    x[:, 0, 0] = [1.0, -1e-300, 0.0, -0.0]
    x[:, 1, 0] = [np.nan, 5.0, -7.0, np.inf]
    x[:, :, 1] = 123.0  # only the first component is read
    s = oracle.readout(x)
    np.testing.assert_array_equal(s[0], [1, -1, 1, 1])
    np.testing.assert_array_equal(s[1], [-1, 1, -1, 1])


def test_extra_frac_and_diverged_cases():
    x = np.zeros((3, 3, 2))
    x[0, 0] = [3.0, 4.0]      # extra share 16/25
    x[1, 0] = [1.0, 0.0]
    x[2, 0] = [0.0, 0.0]      # zero hyperspin contributes 0
    x[:, 1, 0] = 1.0
    x[1, 2, 1] = 2e3          # |x| > 1e3 -> diverged
    f = oracle.extra_frac(x)
    assert f[0] == 16.0 / 25.0 and f[1] == 0.0
    assert f[2] == 1.0
    x[0, 1, 0] = np.nan
    dv = oracle.diverged(x)
    np.testing.assert_array_equal(dv, [0, 1, 1])


# ----------------------------------------------------- P3 uncoupled fixed point
def test_uncoupled_norm_fixed_point_nonlocal_loss():
    """eps = 0, eta = 0: |x_p|^2 -> r - 1 under the nonlocal loss, and the
    direction of every hyperspin is invariant."""
    n, r, d = 5, 3, 3
    g = np.random.default_rng(0)
    x0 = g.standard_normal((n, r, d)) * 0.3
    pump = np.array([1.5, 1.4, 2.0])
    alpha = np.ones((6000, d))
    J = synth.sk_pm1(n, 93, 0)
    x = oracle.ode_run(J, pump, x0, eps=0.0, btil=1.0, eta=0.0, dt=0.01, steps=6000, alpha=alpha)
    nrm2 = (x ** 2).sum(axis=2)
    np.testing.assert_allclose(nrm2, np.broadcast_to(pump - 1.0, (n, r)), rtol=1e-10)
    u0 = x0 / np.linalg.norm(x0, axis=2, keepdims=True)
    u = x / np.linalg.norm(x, axis=2, keepdims=True)
    np.testing.assert_allclose(u, u0, atol=1e-13)


def test_euler_map_fixed_point_is_exact():
    """On |x|^2 = r - 1 the Euler map itself is stationary (up to rounding)."""
    n, r, d = 4, 2, 2
    pump = np.array([1.5, 1.8])
    g = np.random.default_rng(1)
    v = g.standard_normal((n, r, d))
    x0 = v / np.linalg.norm(v, axis=2, keepdims=True) * np.sqrt(pump - 1.0)[None, :, None]
    J = np.zeros((n, n))
    x = oracle.ode_run(J, pump, x0, 0.0, 1.0, 0.0, 0.05, 50, np.ones((50, d)))
    np.testing.assert_allclose(x, x0, rtol=1e-13, atol=1e-15)


def test_uncoupled_local_cubic_saturates_each_component():
    """CIM nonlinearity (btil = 0, eta = 1): every component saturates on its
    own, x_mu^2 -> r - 1, so |x_p|^2 -> D (r - 1).  Mixing up the local and
    the nonlocal term fails this or the test above."""
    n, r, d = 3, 2, 2
    x0 = np.full((n, r, d), 0.01)
    x0[1, 0, 1] = -0.02
    pump = np.array([1.3, 1.7])
    x = oracle.ode_run(np.zeros((n, n)), pump, x0, 0.0, 0.0, 1.0, 0.01, 6000, np.ones((6000, d)))
    np.testing.assert_allclose(x ** 2, np.broadcast_to((pump - 1.0)[None, :, None], x.shape), rtol=1e-9)
    assert x[1, 0, 1] < 0


def test_linear_decay_below_threshold():
    """Linear regime, r < 1, eps = 0: x_k = (1 + dt (r-1))^k x_0."""
    n, r, d = 3, 2, 2
    x0 = np.random.default_rng(2).standard_normal((n, r, d)) * 1e-9
    pump = np.array([0.5, 0.9])
    k = 300
    x = oracle.ode_run(np.zeros((n, n)), pump, x0, 0.0, 1.0, 1.0, 0.01, k, np.ones((k, d)))
    fac = (1.0 + 0.01 * (pump - 1.0)) ** k
    np.testing.assert_allclose(x, x0 * fac[None, :, None], rtol=1e-12)


# --------------------------------------- P4 linear closed form (GEMM, eps, alpha)
def test_linear_closed_form_constant_alpha_per_component():
    """btil = eta = 0: x_k = (I (1 + dt (r-1)) + dt eps alpha_mu J)^k x_0 for
    every component, computed by eigendecomposition.  alpha differs per
    component, so a component/step index mix-up fails."""
    n, r, d = 7, 3, 3
    J = synth.sk_pm1(n, 94, 0).astype(np.float64)
    g = np.random.default_rng(3)
    x0 = g.standard_normal((n, r, d))
    pump = np.array([0.8, 1.0, 1.1])
    eps, dt, k = 0.07, 0.02, 250
    avec = np.array([1.0, 0.5, -0.25])
    alpha = np.tile(avec, (k, 1))
    x = oracle.ode_run(J, pump, x0, eps, 0.0, 0.0, dt, k, alpha)
    w, V = np.linalg.eigh(J)
    for i in range(r):
        for mu in range(d):
            lam = 1.0 + dt * (pump[i] - 1.0) + dt * eps * avec[mu] * w
            ref = V @ (lam ** k * (V.T @ x0[:, i, mu]))
            np.testing.assert_allclose(x[:, i, mu], ref, rtol=1e-10, atol=1e-12)


def test_linear_asymmetric_coupling_row_convention():
    """With a non-symmetric J the contraction must be sum_q J_pq x_q (row p):
    a transposed operand fails.  Reference: explicit matrix products."""
    n, r, d = 6, 2, 2
    g = np.random.default_rng(4)
    J = g.standard_normal((n, n))
    x0 = g.standard_normal((n, r, d))
    pump = np.array([0.9, 1.05])
    eps, dt, k = 0.1, 0.01, 40
    # time-varying, component-dependent alpha, started mid-table
    start = 13
    tab = np.stack([np.cos(0.1 * np.arange(start + k)), np.linspace(1, -1, start + k)], axis=1)
    x = oracle.ode_run(J, pump, x0, eps, 0.0, 0.0, dt, k, tab, start_step=start)
    for i in range(r):
        for mu in range(d):
            v = x0[:, i, mu].copy()
            for s in range(start, start + k):
                M = np.eye(n) * (1.0 + dt * (pump[i] - 1.0)) + dt * eps * tab[s, mu] * J
                v = M @ v
            np.testing.assert_allclose(x[:, i, mu], v, rtol=1e-11, atol=1e-13)


def test_split_run_equals_full_run():
    n, r, d = 6, 4, 2
    J = synth.sk_pm1(n, 95, 0)
    x0 = synth.initial_states(n, r, d, 95, 0)
    al, _ = synth.anneal_schedule(300, d)
    pump = synth.pump_grid(2, [0.8, 1.4])
    kw = dict(eps=0.2, btil=1.0, eta=2e-4, dt=0.01)
    full = oracle.ode_run(J, pump, x0, steps=300, alpha=al, **kw)
    a = oracle.ode_run(J, pump, x0, steps=120, alpha=al, **kw)
    b = oracle.ode_run(J, pump, a, steps=180, alpha=al, start_step=120, **kw)
    np.testing.assert_array_equal(full, b)


# ----------------------------------------------- P2 D = 1 reduces to the CIM
def test_d1_nonlocal_equals_local_bit_exact():
    """For D = 1 the nonlocal loss x S and the local cubic x^3 coincide, so
    (btil, eta) = (1, 0) and (0, 1) give identical trajectories."""
    n, r = 12, 8
    J = synth.sk_pm1(n, 96, 0)
    x0 = synth.initial_states(n, r, 1, 96, 0)
    pump = synth.pump_grid(2, [0.7, 1.1, 1.4, 1.9])
    al = synth.constant_schedule(1500, 1)
    eps = synth.default_eps(J)
    a = oracle.ode_run(J, pump, x0, eps, 1.0, 0.0, 0.01, 1500, al)
    b = oracle.ode_run(J, pump, x0, eps, 0.0, 1.0, 0.01, 1500, al)
    assert np.array_equal(a, b)
    assert np.abs(a).max() > 0.1  # left the linear regime


def test_d1_matches_textbook_cim_loop():
    """Against a separately written CIM integrator:
    dx/dt = (r - 1) x + eps sum_q J x_q - x^3."""
    n, r = 10, 6
    J = synth.sk_pm1(n, 97, 0).astype(np.float64)
    x0 = synth.initial_states(n, r, 1, 97, 0).astype(np.float64)[:, :, 0]
    pump = np.linspace(0.6, 1.8, r)
    eps, dt, k = synth.default_eps(J), 0.01, 1200
    x = oracle.ode_run(J, pump, x0[:, :, None], eps, 0.0, 1.0, dt, k, np.ones((k, 1)))[:, :, 0]
    y = x0.copy()
    for _ in range(k):
        y = y + dt * ((pump[None, :] - 1.0) * y + eps * (J @ y) - y ** 3)
    np.testing.assert_allclose(x, y, rtol=1e-10, atol=1e-12)


# ------------------------------------------------------- P5 / P6 / P7 symmetries
def test_gauge_covariance_bit_exact():
    n, r, d = 14, 6, 2
    J = synth.sk_pm1(n, 98, 0)
    x0 = synth.initial_states(n, r, d, 98, 0)
    al, _ = synth.anneal_schedule(800, d)
    pump = synth.pump_grid(3, [0.9, 1.5])
    s = np.where(np.random.default_rng(5).random(n) < 0.5, -1, 1).astype(np.int8)
    Jg = (s[:, None] * J * s[None, :]).astype(np.int8)
    x0g = x0 * s[:, None, None]
    kw = dict(eps=synth.default_eps(J), btil=1.0, eta=2e-4, dt=0.01, steps=800, alpha=al)
    x = oracle.ode_run(J, pump, x0, **kw)
    xg = oracle.ode_run(Jg, pump, x0g, **kw)
    assert np.array_equal(xg, x * s[:, None, None])
    sig, sigg = oracle.readout(x), oracle.readout(xg)
    nz = (x[:, :, 0] != 0).T
    assert np.array_equal((sigg * s[None, :])[nz], sig[nz])
    np.testing.assert_array_equal(oracle.ising_energy(Jg, sigg), oracle.ising_energy(J, sig))


def test_z2_symmetry_bit_exact():
    n, r, d = 9, 5, 3
    J = synth.sk_pm1(n, 99, 0)
    x0 = synth.initial_states(n, r, d, 99, 0)
    al, _ = synth.anneal_schedule(600, d)
    pump = np.linspace(0.6, 1.9, r)
    kw = dict(eps=synth.default_eps(J), btil=1.0, eta=0.3, dt=0.01, steps=600, alpha=al)
    assert np.array_equal(oracle.ode_run(J, pump, -x0, **kw), -oracle.ode_run(J, pump, x0, **kw))


def test_rotation_covariance_before_annealing():
    """With equal alpha for all components and no local cubic term the
    equations are O(D) covariant: rotating every hyperspin rotates the
    trajectory."""
    n, r, d = 8, 3, 3
    J = synth.sk_pm1(n, 100, 0)
    g = np.random.default_rng(6)
    x0 = g.standard_normal((n, r, d)) * 0.05
    Q, _ = np.linalg.qr(g.standard_normal((d, d)))
    pump = np.array([0.8, 1.2, 1.6])
    kw = dict(eps=synth.default_eps(J), btil=1.0, eta=0.0, dt=0.01, steps=700, alpha=np.ones((700, d)))
    x = oracle.ode_run(J, pump, x0, **kw)
    xr = oracle.ode_run(J, pump, x0 @ Q, **kw)
    np.testing.assert_allclose(xr, x @ Q, atol=1e-12)
    # the local cubic term breaks it (guards against eta being dropped)
    kw["eta"] = 0.5
    x = oracle.ode_run(J, pump, x0, **kw)
    xr = oracle.ode_run(J, pump, x0 @ Q, **kw)
    assert np.abs(xr - x @ Q).max() > 1e-6


# ----------------------------------------------------------- P8 E_hs
def test_hs_energy_d1_equals_ising_energy():
    n, r = 13, 7
    J = synth.sk_pm1(n, 101, 0)
    x = np.random.default_rng(7).standard_normal((n, r, 1))
    np.testing.assert_array_equal(oracle.hs_energy(J, x), oracle.ising_energy(J, oracle.readout(x)))


def test_hs_energy_two_spin_closed_form():
    th = np.linspace(0, 2 * np.pi, 9)
    x = np.zeros((2, len(th), 2))
    x[0, :, 0] = 2.0
    x[1, :, 0] = 0.5 * np.cos(th)
    x[1, :, 1] = 0.5 * np.sin(th)
    J = np.array([[0.0, -1.5], [-1.5, 0.0]])
    np.testing.assert_allclose(oracle.hs_energy(J, x), 3.0 * np.cos(th), atol=1e-14)


def test_hs_energy_bounds_and_rotation():
    n, r, d = 20, 16, 3
    J = synth.gaussian_j(n, 102, 0)
    g = np.random.default_rng(8)
    x = g.standard_normal((n, r, d))
    e = oracle.hs_energy(J, x)
    lam = np.linalg.eigvalsh(J.astype(np.float64))
    assert np.all(e >= -n * lam[-1] - 1e-9) and np.all(e <= -n * lam[0] + 1e-9)
    Q, _ = np.linalg.qr(g.standard_normal((d, d)))
    np.testing.assert_allclose(oracle.hs_energy(J, x @ Q), e, atol=1e-11)
    # zero hyperspins contribute nothing
    x[3] = 0.0
    xs = np.delete(x, 3, axis=0)
    Js = np.delete(np.delete(J, 3, 0), 3, 1)
    np.testing.assert_allclose(oracle.hs_energy(J, x), oracle.hs_energy(Js, xs), atol=1e-11)


# --------------------------------------------- P9 the paper's qualitative claim
def test_hyperspin_steady_state_below_ising_gs():
    """Before annealing, the D = 2 steady state reaches a hyperspin energy
    below the Ising ground state (main text, discussion of Fig. 2)."""
    n = 16
    J = synth.sk_pm1(n, 0, 0)
    egs, _ = oracle.bruteforce_gs(J)
    r, d = 64, 2
    x0 = synth.initial_states(n, r, d, 0, 0)
    pump = synth.pump_grid(16, [0.6, 0.9, 1.2, 1.5])
    x = oracle.ode_run(J, pump, x0, synth.default_eps(J), 1.0, 2e-4, 0.01, 800, np.ones((800, d)))
    assert oracle.hs_energy(J, x).min() < egs


# ------------------------------------------- P10 the ODE is the limit of Eq. (2)
def _rk4_coupled_mode(a, h, kl, m=4000):
    def f(v):
        s, p = v
        return np.array([p * s, -s * s])
    v = np.array([a, h], dtype=np.float64)
    dz = kl / m
    for _ in range(m):
        k1 = f(v); k2 = f(v + 0.5 * dz * k1); k3 = f(v + 0.5 * dz * k2); k4 = f(v + dz * k3)
        v = v + dz / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return v[0] / a


@pytest.mark.parametrize("a,h,kl", [(0.3, 0.8, 0.5), (-1.2, 0.3, 1.0), (0.01, 2.0, 0.1), (2.5, 0.0, 0.7)])
def test_nlm_gain_solves_coupled_mode_equations(a, h, kl):
    assert oracle.nlm_gain(a, h, kl) == pytest.approx(_rk4_coupled_mode(a, h, kl), rel=1e-11)


def test_nlm_gain_small_signal_and_depletion():
    for h, kl in [(0.5, 0.1), (2.0, 0.3)]:
        assert oracle.nlm_gain(0.0, h, kl) == pytest.approx(math.exp(kl * h), rel=1e-14)
        # first order in A^2: K ~ exp(kl h) (1 - (kl A)^2 / 2) for small kl h
    a, h, kl = 1e-3, 1e-3, 1e-2
    k = oracle.nlm_gain(a, h, kl)
    assert k == pytest.approx(math.exp(kl * h) * (1 - (kl * a) ** 2 / 2), rel=1e-9)


def _map_vs_ode_error(gamma, T=6.0):
    n, r, d = 8, 3, 2
    J = synth.sk_pm1(n, 103, 0).astype(np.float64)
    bb2 = 25.0           # beta b^2 of the paper
    eta = 0.02
    kl = math.sqrt(2.0 * bb2 * eta)
    b = dd = gamma / 2.0
    beta = bb2 / (b * b)
    eps = 0.5 / synth.lambda_max(J)
    jmag = eps * gamma / b
    rr = np.array([1.2, 1.5, 2.0])
    hth = -math.log((1 - b) * (1 - dd)) / kl
    x0 = np.random.default_rng(9).standard_normal((n, r, d)) * 0.1
    scale = math.sqrt(gamma / bb2)
    steps = int(round(T / gamma))
    A = oracle.map_run(jmag * J, rr * hth, x0 * scale, b, dd, kl, beta, steps, np.ones((steps, d)))
    # fine-step reference of the ODE
    fine = 20000
    x = oracle.ode_run(J, rr, x0, eps, 1.0, eta, T / fine, fine, np.ones((fine, d)))
    return np.abs(A / scale - x).max()


def test_map_converges_to_ode_first_order():
    errs = [_map_vs_ode_error(g) for g in (0.04, 0.02, 0.01)]
    assert errs[2] < 0.03
    for e1, e2 in zip(errs, errs[1:]):
        assert 1.6 < e1 / e2 < 2.5


# ------------------------- the map's annealing weight C_jl -> alpha_{mu,tau} C_jl
def _small_signal_map_matrix(J, h, b, dd, kl, a_mu):
    """Eq. (2) linearised at vanishing amplitude with beta = 0: the medium
    multiplies by its small-signal gain exp(kL h), the coupler mixes
    (1-b) B + b alpha_mu J B, the loss keeps (1-d).  Written from the
    equation, not from the oracle."""
    n = J.shape[0]
    return (1.0 - dd) * math.exp(kl * h) * ((1.0 - b) * np.eye(n) + b * a_mu * J)


def test_map_linear_closed_form_alpha_per_component():
    """beta = 0 and amplitudes <= 1e-8, so K = exp(kL h) to first order
    (the depletion term is (kL A)^2 / 2 ~ 1e-18 relative): the map is then
    linear per component, A_k = M_mu^k A_0 with a different alpha for every
    component, computed by eigendecomposition of the symmetric J.  A wrong
    component or step index of alpha, a dropped (1-b) or (1-d), or the
    coupling applied to A instead of B = K A fails."""
    n, r, d = 9, 3, 3
    J = synth.sk_pm1(n, 104, 0).astype(np.float64) * 0.3
    g = np.random.default_rng(11)
    A0 = g.standard_normal((n, r, d)) * 1e-9
    b, dd, kl = 0.02, 0.01, 0.1
    h = np.array([0.05, 0.2, 0.31])        # below and near the uncoupled threshold
    avec = np.array([1.0, 0.6, -0.35])
    k = 120
    A = oracle.map_run(J, h, A0, b, dd, kl, 7.0, k, np.tile(avec, (k, 1)))
    # beta enters only through B S(B) ~ 1e-18 relative at these amplitudes
    assert np.abs(A).max() < 1e-7
    w, V = np.linalg.eigh(J)
    for i in range(r):
        for mu in range(d):
            lam = (1.0 - dd) * math.exp(kl * h[i]) * ((1.0 - b) + b * avec[mu] * w)
            ref = V @ (lam ** k * (V.T @ A0[:, i, mu]))
            np.testing.assert_allclose(A[:, i, mu], ref, rtol=1e-10, atol=1e-22)


def test_map_asymmetric_coupling_time_varying_alpha():
    """Non-symmetric couplings and an alpha that changes with the round trip
    and the component, started in the middle of the table: the coupling must
    be sum_l J_pl B_l (row p) and round trip tau must use alpha row tau.
    Reference: explicit products of the small-signal map matrices."""
    n, r, d = 7, 2, 2
    g = np.random.default_rng(12)
    J = g.standard_normal((n, n)) * 0.4
    A0 = g.standard_normal((n, r, d)) * 1e-9
    b, dd, kl = 0.03, 0.02, 0.1
    h = np.array([0.1, 0.45])
    start, k = 17, 60
    tab = np.stack([np.cos(0.07 * np.arange(start + k)), np.linspace(1.0, -0.5, start + k)], axis=1)
    A = oracle.map_run(J, h, A0, b, dd, kl, 0.0, k, tab, start_step=start)
    for i in range(r):
        for mu in range(d):
            v = A0[:, i, mu].copy()
            for s in range(start, start + k):
                v = _small_signal_map_matrix(J, h[i], b, dd, kl, tab[s, mu]) @ v
            np.testing.assert_allclose(A[:, i, mu], v, rtol=1e-10, atol=1e-22)


def test_map_split_run_with_alpha_table_equals_full_run():
    """The round trips of one call equal those of two calls that resume at
    start_step, with an annealing table that changes every round trip."""
    n, r, d = 6, 3, 3
    J = synth.sk_pm1(n, 105, 0).astype(np.float64) * 0.05
    A0 = np.random.default_rng(13).standard_normal((n, r, d)) * 0.05
    steps = 90
    tab, _ = synth.anneal_schedule(steps, d)
    h = np.array([0.3, 0.5, 0.9])
    full = oracle.map_run(J, h, A0, 0.01, 0.01, 0.1, 25.0 / 0.01 ** 2, steps, tab)
    half = oracle.map_run(J, h, A0, 0.01, 0.01, 0.1, 25.0 / 0.01 ** 2, 40, tab)
    rest = oracle.map_run(J, h, half, 0.01, 0.01, 0.1, 25.0 / 0.01 ** 2, 50, tab, start_step=40)
    np.testing.assert_array_equal(rest, full)
    # the table's last rows are zero for the extra components: the anneal acted
    assert tab[-1, 1:].max() == 0.0 and tab[0].min() == 1.0
