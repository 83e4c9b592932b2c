"""Energy traces of the three operating modes of Fig. 2 on one 20% Erdos-Renyi
graph at N = 20 (exhaustive Ising ground state): the XY machine settles at
the XY ground state of the independent minimizer, below the Ising ground
state; the annealed CHYM passes below the Ising ground state and reaches an
Ising energy from below; the CIM's hyperspin energy is its Ising energy at
every checkpoint, at or above the ground state.  The segmented runs equal
whole runs bit for bit, and the hyperspin energies equal the oracle's for
the same amplitudes."""
import numpy as np
import pytest

import oracle
from paper_2308_02329_amd import api, stats, traces, xy

torch = pytest.importorskip("torch")
from gpu_helpers import to_dev  # noqa: E402

pytestmark = pytest.mark.gpu

N, STEPS, CKPT, REP = 20, 20000, 20, 8


@pytest.fixture(scope="module")
def graph():
    J = stats.graph(N, 0, 2308)
    return J, stats.ground_state_exhaustive(J), xy.xy_ground(J, starts=64, seed=1)[0]


def test_xy_mode_settles_at_the_xy_ground_state(graph):
    J, egs, exy = graph
    taus, hs, isg = traces.trace(J, "xy", REP, STEPS, CKPT)
    assert exy < egs
    final = hs[-1].min()
    assert final < egs  # below the Ising ground state
    assert final >= exy - 1e-9 * abs(exy)  # never below the XY ground state
    assert (final - exy) / abs(exy) <= 2e-3
    assert np.all(isg >= egs)


def test_annealed_chym_reaches_the_ising_energy_from_below(graph):
    J, egs, exy = graph
    taus, hs, isg, A = traces.trace(J, "chym_annealed", REP, STEPS, CKPT, return_state=True)
    k0 = int(np.searchsorted(taus, 0.4 * STEPS))  # the anneal starts here
    assert hs[k0].min() < egs  # the hyperspins sit below the Ising ground state
    best = int(np.argmin(isg[-1]))
    assert hs[k0, best] < hs[-1, best]  # and the energy rises to the final Ising energy
    np.testing.assert_allclose(hs[-1], isg[-1], rtol=1e-3, atol=0.05)  # collinear at the end
    assert isg[-1].min() >= egs
    # the segmented run equals a whole run; E_hs equals the oracle's on the same amplitudes
    jmag, h, A0, alpha, bb2 = traces.mode_inputs(J, "chym_annealed", REP, STEPS, (0.1, 0.5, 1.0), 2308)
    Aw = to_dev(A0)
    m = traces.MODES["chym_annealed"]
    api.chym_map_integrate(to_dev(J), to_dev(h), Aw, to_dev(alpha), b=traces.B, loss=traces.LOSS, kl=m["kl"],
                           beta_b2=bb2, jmag=jmag, steps=STEPS)
    assert np.array_equal(Aw.cpu().numpy(), A)
    np.testing.assert_allclose(hs[-1], oracle.hs_energy(J, A), rtol=1e-12, atol=1e-9)


def test_cim_hyperspin_energy_is_its_ising_energy(graph):
    J, egs, exy = graph
    taus, hs, isg = traces.trace(J, "cim", REP, STEPS, CKPT)
    assert np.array_equal(hs, isg)  # D = 1: unit vectors are the signs
    assert np.all(isg >= egs)
