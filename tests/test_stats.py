"""Host logic of the statistical harness (statistics paragraph, Figs. 3-4):
the figures of merit on hand-worked energy tables, the exponential fit, the
exhaustive ground state against the oracle's brute force and closed forms,
and the map parameters against the thresholds they are derived from."""
import math

import numpy as np
import pytest

import oracle
from paper_2308_02329_amd import stats, synth


def test_figures_hand_worked():
    # 3 pumps x 4 runs, E_GS = -10 (gaps of 4, as for +-1 couplings)
    e = np.array([[-10, -10, -6, -2], [-6, -6, -6, -6], [-10, -6, -6, -6]]).ravel()
    f = stats.figures(e, -10, 3, 4, n=8)
    assert f["P"] == [0.5, 0.0, 0.25]
    assert f["P_max"] == 0.5
    assert f["W"] == pytest.approx((0.5 + 0.25) / 2)       # mean over the pumps where P > 0
    assert f["W_scan"] == pytest.approx((0.5 + 0.25) / 3)  # mean over the whole scan
    assert f["dE"] == pytest.approx((0 + 0 + 4 + 8 + 16 + 0 + 12) / 12)
    assert f["dE_per_n"] == pytest.approx(f["dE"] / 8)
    # every run at the ground state: P = 1 everywhere, dE = 0
    g = stats.figures(np.full(6, -3), -3, 2, 3, n=3)
    assert g["P_max"] == g["W"] == g["W_scan"] == 1.0 and g["dE"] == 0.0
    # never at the ground state: W = 0 (empty support)
    h = stats.figures(np.full(6, 1), -3, 2, 3, n=3)
    assert h["P_max"] == h["W"] == 0.0 and h["dE"] == 4.0
    with pytest.raises(ValueError, match="below"):
        stats.figures(np.array([-12, -10]), -10, 1, 2, n=2)


def test_histogram_and_summary():
    hist = stats.histogram([-10, -6, -6, -2, -10, -10], -10)
    assert hist == {0: 0.5, 4: pytest.approx(1 / 3), 8: pytest.approx(1 / 6)}
    assert sum(hist.values()) == pytest.approx(1.0)
    # dE is the histogram's mean deviation
    assert sum(k * v for k, v in hist.items()) == pytest.approx(stats.figures(
        [-10, -6, -6, -2, -10, -10], -10, 1, 6, n=1)["dE"])
    s = stats.summary([1, 2, 3, 4, 5])
    assert s == {"mean": 3.0, "q25": 2.0, "q75": 4.0}


def test_exponential_fit():
    ns = np.arange(10, 101, 10)
    for a, b in ((18e-3, 0.9), (8e-3, 1.3)):
        fa, fb = stats.fit_exponential(ns, b * np.exp(-a * ns))
        assert fa == pytest.approx(a, rel=1e-10) and fb == pytest.approx(b, rel=1e-10)
    # zeros are left out of the log fit
    v = 0.5 * np.exp(-0.01 * ns)
    v[3] = 0.0
    assert stats.fit_exponential(ns, v)[0] == pytest.approx(0.01, rel=1e-10)
    assert all(math.isnan(x) for x in stats.fit_exponential([10, 20], [0.3, 0.0]))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 9, 12])
def test_exhaustive_ground_state(n):
    for k in range(3):
        J = synth.er_pm1(n, 91, n, k, density=0.5) if n > 2 else synth.sk_pm1(n, 91, k)
        assert stats.ground_state_exhaustive(J) == int(round(oracle.bruteforce_gs(J)[0]))


def test_exhaustive_ground_state_closed_forms():
    n = 10
    ferro = np.ones((n, n), dtype=np.int8) - np.eye(n, dtype=np.int8)
    assert stats.ground_state_exhaustive(ferro) == -n * (n - 1)  # all aligned
    # antiferromagnetic complete graph: E = (sum s)^2 - n, minimized at sum s = 0 (even n) or 1 (odd n)
    for m in (7, 8):
        af = -(np.ones((m, m), dtype=np.int8) - np.eye(m, dtype=np.int8))
        assert stats.ground_state_exhaustive(af) == (m % 2) - m


def test_map_parameters_sit_at_the_thresholds():
    J = stats.graph(30, 0, 1)
    assert np.array_equal(J, J.T) and set(np.unique(J)) <= {-1, 0, 1}
    assert 0.1 < np.count_nonzero(J) / (30 * 29) < 0.3  # 20% density
    jmag, h, A0, alpha, bb2 = stats.machine_inputs(J, 2, stats.pumps(2), 4, 100, 1, 0)
    assert stats.pumps(1).size == 51 and stats.pumps(2).size == 21
    assert h.shape == (84,) and A0.shape == (30, 84, 2) and alpha.shape == (100, 2) and bb2 == stats.BB2
    hth = stats.h_threshold()
    # uncoupled threshold: unit small-signal gain (1 - d)(1 - b) e^{kappa L h_th} per round trip
    assert (1 - stats.LOSS) * (1 - stats.B) * math.exp(stats.KL * hth) == pytest.approx(1.0, rel=1e-12)
    np.testing.assert_allclose(h[::4], (hth * (1 + stats.pumps(2))).astype(np.float32))
    # coupled threshold at delta h = -0.5: (1 - d)((1 - b) + b J lambda_max) e^{kappa L h} = 1
    lam = synth.lambda_max(J)
    g = (1 - stats.LOSS) * ((1 - stats.B) + stats.B * jmag * lam) * math.exp(stats.KL * hth * 0.5)
    assert g == pytest.approx(1.0, rel=1e-4)
    # the CIM: no nonlocal loss, no anneal
    _, _, _, a1, b1 = stats.machine_inputs(J, 1, stats.pumps(1), 2, 50, 1, 0)
    assert b1 == 0.0 and np.all(a1 == 1.0)


def test_success_report_hand_worked():
    """Two instances, 2 pumps x 4 runs each, E_GS -10 and -6."""
    e0 = [-10, -10, -6, -2, -6, -6, -6, -6]      # P = (0.5, 0), deviations 0 0 4 8 4 4 4 4
    e1 = [-2, -2, -2, -2, -6, -2, -2, -2]       # P = (0, 0.25), deviations 4 4 4 4 0 4 4 4
    rep = stats.success_report([e0, e1], [-10, -6], 2, 4, n=4, t_run_ms=2.0)
    assert rep["instances"] == 2
    assert rep["P_per_pump_mean"] == [0.25, 0.125]
    assert rep["solved_fraction"] == 1.0
    # quartiles of (0.25, 0.5) by linear interpolation
    assert rep["P_max"] == {"q25": 0.3125, "median": 0.375, "q75": 0.4375}
    assert rep["dE"]["q25"] == pytest.approx(28 / 8) and rep["dE"]["q75"] == pytest.approx(28 / 8)
    assert rep["dE_per_n"]["median"] == pytest.approx(28 / 8 / 4)
    # best-pump TTS99: 2 ms per run, p = 0.5 and 0.25
    t_a, t_b = 2.0 * math.log(0.01) / math.log(0.75), 2.0 * math.log(0.01) / math.log(0.5)
    assert rep["tts99_ms"]["median"] == pytest.approx((t_a + t_b) / 2)
    assert rep["tts99_ms"]["q25"] == pytest.approx(t_b + 0.25 * (t_a - t_b))
    # an unsolved instance has an infinite TTS99, reported as None; it does not count as solved
    rep2 = stats.success_report([e0, e1, [-2] * 8, [-2] * 8], [-10, -6, -6, -6], 2, 4, n=4, t_run_ms=2.0)
    assert rep2["solved_fraction"] == 0.5
    assert rep2["tts99_ms"]["median"] is None and rep2["tts99_ms"]["q75"] is None
    assert rep2["tts99_ms"]["q25"] == pytest.approx(t_b + 0.75 * (t_a - t_b))


def test_tts99_is_the_attempt_count_closed_form():
    assert stats.tts99(2.0, 0.0) == math.inf
    assert stats.tts99(2.0, 0.995) == 2.0
    for k in (1.5, 10.0, 1000.0):
        assert stats.tts99(3.0, 1.0 - 0.01 ** (1.0 / k)) == pytest.approx(3.0 * k, rel=1e-12)
