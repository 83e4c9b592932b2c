"""Energy traces of the three operating modes of Fig. 2 on one graph.

Fig. 2 shows the hyperspin energy E_hs of Eq. (3) during the round trips
for the CHYM run as (I) an XY machine (D = 2, no annealing, kappa L = 1e-3),
(II) an XY machine with dimensional annealing (D = 2 -> 1, kappa L = 0.1),
and (III) the CIM (D = 1, beta = 0, kappa L = 0.1); beta b^2 = 25 where the
nonlocal loss is on (parameter paragraph).  (I) settles at the XY ground
state, below the Ising ground state; (II) first settles near the XY ground
state and then reaches the Ising ground state from below; (III) approaches
the Ising ground state from above through Ising local minima.

The runs are the round-trip map of Eq. (2) (chym_map_integrate), split
into segments at the checkpoints (a split run is bit-identical to a whole
one); at every checkpoint chym_hs_energy gives E_hs and chym_readout with
chym_ising_energy the Ising energy of the current signs.  Couplings,
pumps and initial states follow the statistics harness (b = d = 0.01,
J = eps (b + d) / b with eps = 0.5 / lambda_max, h = h_th (1 + delta h)).

    python -m paper_2308_02329_amd.traces --out traces.json
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np
import torch

from . import api, synth

B = 0.01
LOSS = 0.01
BB2 = 25.0
MODES = {
    "xy": dict(d=2, kl=1e-3, bb2=BB2, anneal=False),
    "chym_annealed": dict(d=2, kl=0.1, bb2=BB2, anneal=True),
    "cim": dict(d=1, kl=0.1, bb2=0.0, anneal=False),
}
_X0_TAG = 8


def mode_inputs(J, mode, n_rep, steps, dh, seed):
    """Coupling magnitude, pumps h [R] (replica k * n_rep + i: dh[k]),
    amplitudes A0 [n, R, d], annealing table [steps, d] and beta b^2."""
    m = MODES[mode]
    n, d = J.shape[0], m["d"]
    jmag = float(np.float32(0.5 / synth.lambda_max(J) * (B + LOSS) / B))
    hth = -math.log((1.0 - B) * (1.0 - LOSS)) / m["kl"]
    h = synth.pump_grid(n_rep, hth * (1.0 + np.asarray(dh, dtype=np.float64)))
    A0 = synth.initial_states(n, h.size, d, seed, _X0_TAG, n, d, sigma=0.1 * math.sqrt((B + LOSS) / BB2))
    alpha = synth.anneal_schedule(steps, d)[0] if m["anneal"] else synth.constant_schedule(steps, d)
    return jmag, h, A0, alpha, m["bb2"]


def trace(J, mode, n_rep=16, steps=20000, n_ckpt=40, dh=(0.1, 0.5, 1.0), seed=2308, device="cuda",
          return_state=False):
    """Round trips tau [n_ckpt + 1] and, per checkpoint and run, the
    hyperspin energy E_hs and the Ising energy of the signs [n_ckpt + 1, R]
    (and the final amplitudes [n, R, d] when return_state)."""
    m = MODES[mode]
    dev = torch.device(device)
    n = J.shape[0]
    jmag, h, A0, alpha, bb2 = mode_inputs(J, mode, n_rep, steps, dh, seed)
    Jd = torch.from_numpy(J).to(dev)
    hd = torch.from_numpy(h).to(dev)
    A = torch.from_numpy(A0).to(dev)
    al = torch.from_numpy(alpha).to(dev)
    R = h.size
    spins = torch.empty((R, api.spin_words(n)), dtype=torch.int64, device=dev)
    ehs = torch.empty(R, dtype=torch.float64, device=dev)
    eis = torch.empty(R, dtype=torch.float64, device=dev)
    taus = np.linspace(0, steps, n_ckpt + 1).round().astype(int)
    out_hs, out_is = [], []
    for k, tau in enumerate(taus):
        if k:
            api.chym_map_integrate(Jd, hd, A, al, b=B, loss=LOSS, kl=m["kl"], beta_b2=bb2, jmag=jmag,
                                   steps=int(tau - taus[k - 1]), start_step=int(taus[k - 1]))
        api.chym_hs_energy(Jd, A, ehs)
        api.chym_readout(A, spins)
        api.chym_ising_energy(Jd, spins, None, eis)
        out_hs.append(ehs.cpu().numpy().copy())
        out_is.append(eis.cpu().numpy().copy())
    if return_state:
        return taus, np.array(out_hs), np.array(out_is), A.cpu().numpy()
    return taus, np.array(out_hs), np.array(out_is)


def report(n=100, seed=2308, n_rep=16, steps=20000, n_ckpt=40, log=None):
    """Traces of the three modes on one 20% Erdos-Renyi graph, with the XY
    ground state of the minimizer and a putative Ising ground state (the
    best energy of every run here and of a longer annealed search)."""
    from .stats import graph, search_ground
    from .xy import xy_ground

    J = graph(n, 0, seed)
    e_xy = xy_ground(J, starts=64, seed=seed)[0]
    out = {"n": n, "E_XY": e_xy, "modes": {}}
    best_ising = search_ground([J], 2000, 20000, seed)[0]
    for mode in MODES:
        taus, hs, isg = trace(J, mode, n_rep, steps, n_ckpt, seed=seed)
        best_ising = min(best_ising, int(isg[-1].min()))
        k = int(np.argmin(isg[-1]))  # the run with the lowest final Ising energy
        out["modes"][mode] = {"tau": taus.tolist(), "E_hs_best_run": hs[:, k].tolist(),
                              "E_ising_best_run": isg[:, k].tolist(), "E_hs_final_min": float(hs[-1].min()),
                              "E_ising_final_min": float(isg[-1].min())}
        if log:
            log(f"{mode}: final E_hs min {hs[-1].min():.2f}, final Ising min {isg[-1].min():.0f}")
    out["E_GS"] = best_ising
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=100)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--out", type=str, default="")
    a = ap.parse_args()
    rep = report(a.n, steps=a.steps, log=lambda m: print(m, flush=True))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rep, f)
    print(json.dumps({"n": rep["n"], "E_XY": rep["E_XY"], "E_GS": rep["E_GS"],
                      "final": {k: (v["E_hs_final_min"], v["E_ising_final_min"]) for k, v in rep["modes"].items()}}))


if __name__ == "__main__":
    main()
