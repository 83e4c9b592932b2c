"""XY-machine mode on the GPU (Fig. 2 (I), parameter paragraph: D = 2, no
annealing, kappa L = 1e-3, beta b^2 = 25).

Parity: the final hyperspin energies of the batched map runs against the
oracle's literal map and its E_hs on the same inputs.  E_hs depends only on
the directions of the hyperspins (and is invariant under a global rotation,
the XY model's zero mode), so float32 amplitude errors of relative size
~1e-4 after a few thousand round trips move it by at most ~2e-4 * sum|J|;
the bar is 2e-3 of |E_hs|.

Claim: the best run's E_hs lies within 0.14% of the XY ground-state energy
of the independent minimizer, and that energy is below the Ising ground
state (exhaustive) on these frustrated graphs."""
import numpy as np
import pytest

import oracle
from paper_2308_02329_amd import stats, xy

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [12, 30])
def test_xy_runs_match_oracle(n):
    n_rep, steps, seed, dh = 8, 3000, 13, (0.1, 0.5)
    graphs = [stats.graph(n, g, seed) for g in range(2)]
    ehs, amps = xy.run_machine(graphs, n_rep, steps, dh, seed)
    for g, J in enumerate(graphs):
        jmag, h, A0, alpha = xy.machine_inputs(J, n_rep, steps, dh, seed, g)
        Ao = oracle.map_run(jmag * J.astype(np.float64), h.astype(np.float64), A0.astype(np.float64), xy.B, xy.LOSS,
                            xy.KL, xy.BB2 / xy.B ** 2, steps, alpha)
        eo = oracle.hs_energy(J, Ao)
        # the GPU's E_hs kernel on the GPU's own amplitudes equals the oracle's E_hs of them
        np.testing.assert_allclose(ehs[g], oracle.hs_energy(J, amps[g]), rtol=1e-12, atol=1e-9)
        assert np.abs(Ao).max() > 1e-3  # above threshold
        rel = np.abs(ehs[g] - eo) / np.abs(eo)
        print(f"n={n} graph {g}: max relative E_hs difference {rel.max():.2e}")
        assert rel.max() <= 2e-3


def test_xy_machine_reaches_the_xy_ground_state():
    rep = xy.report(ns=(20, 100), n_graphs=3, n_rep=50, steps=20000, dh=(0.1, 0.25, 0.5, 1.0), starts=32)
    small, big = rep["rows"]
    for row in (small, big):
        for p in row["graphs_detail"]:
            assert p["E_hs_best"] >= p["E_XY"] - 1e-6 * abs(p["E_XY"])  # no run beats the minimizer
    for p in small["graphs_detail"]:
        assert p["E_XY"] < p["E_Ising_GS"]  # the XY ground state lies below the Ising one
    for p in big["graphs_detail"]:  # N = 100, the paper's size
        assert p["best"] <= 1.4e-3, p
