"""The statistical harness on the GPU: its runs (chym_map_batch, readout and
exact energies) against the oracle's literal map on the same inputs, and a
small end-to-end report.

Final Ising energies are integers decided by float arithmetic: a run that
ends near a sign change of some amplitude can be read differently by the
float32 kernels and the float64 oracle, so the bar is that at least 98% of
the runs agree exactly and the figures of merit computed from the two agree
to within the disagreeing fraction."""
import numpy as np
import pytest

import oracle
from paper_2308_02329_amd import stats

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def oracle_energies(J, d, n_rep, steps, seed, g):
    jmag, h, A0, alpha, bb2 = stats.machine_inputs(J, d, stats.pumps(d), n_rep, steps, seed, g)
    A = oracle.map_run(jmag * J.astype(np.float64), h.astype(np.float64), A0.astype(np.float64), stats.B,
                       stats.LOSS, stats.KL, bb2 / stats.B ** 2, steps, alpha)
    return oracle.ising_energy(J, oracle.readout(A)).astype(np.int64)


@pytest.mark.parametrize("n", [10, 17])
def test_harness_runs_match_oracle(n):
    n_rep, steps, seed = 8, 3000, 11
    graphs = [stats.graph(n, g, seed) for g in range(2)]
    for d in (1, 2):
        eg = stats.run_machine(graphs, d, n_rep, steps, seed)
        for g, J in enumerate(graphs):
            eo = oracle_energies(J, d, n_rep, steps, seed, g)
            agree = np.mean(eg[g] == eo)
            print(f"n={n} d={d} graph {g}: {agree:.4f} of the runs agree")
            assert agree >= 0.98, (n, d, g, agree)
            egs = stats.ground_state_exhaustive(J)
            fg = stats.figures(eg[g], egs, stats.pumps(d).size, n_rep, n)
            fo = stats.figures(eo, egs, stats.pumps(d).size, n_rep, n)
            tol = (1 - agree) * n_rep + 1e-12  # one disagreeing run moves P by 1 / n_rep
            assert abs(fg["P_max"] - fo["P_max"]) <= tol
            assert np.abs(np.array(fg["P"]) - np.array(fo["P"])).max() <= tol


def test_harness_report():
    rep = stats.harness(ns=(8, 12, 30), n_graphs=3, n_rep=10, steps=2000, search_rep=200, search_steps=2000,
                        log=None)
    assert [r["n"] for r in rep["per_n"]] == [8, 12, 30]
    assert rep["per_n"][0]["E_GS"] == "exhaustive" and rep["per_n"][2]["E_GS"] == "best run"
    for row in rep["per_n"]:
        for m in ("D1_cim", "D2_chym"):
            s = row[m]
            assert 0.0 <= s["P_max"]["q25"] <= s["P_max"]["q75"] <= 1.0
            assert 0.0 <= s["W"]["mean"] <= s["P_max"]["mean"] + 1e-12
            assert s["W_scan"]["mean"] <= s["W"]["mean"] + 1e-12
            assert s["dE"]["mean"] >= 0.0
    ex = rep["example"]
    assert ex["n"] == 30 and len(ex["P_d1"]) == 51 and len(ex["P_d2"]) == 21
    assert sum(ex["H_E_d1"].values()) == pytest.approx(1.0) and min(ex["H_E_d2"]) >= 0
    assert set(rep["fits"]) == {"D1_cim", "D2_chym"}
