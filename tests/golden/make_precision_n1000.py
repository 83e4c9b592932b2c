"""Writes ``precision_n1000_d4.npz``: the FP64 oracle's final states for a
fixed subset of the precision workload's runs (SK +-1 and Gaussian
couplings, N = 1000, D = 4, 10 000 Euler steps with the dimensional
anneal), against which the GPU test reports the error of every coupling
storage and precision form.

Calls only the oracle and the seeded input generators:

    python tests/golden/make_precision_n1000.py     (about 15 min on 8 cores)

Inputs (shared with ``tests/test_gpu_precision_n1000.py`` through
``precision_n1000_inputs``): 16 pumps in [0.5, 2] x 256 initial states
= 4096 runs, pump-major; the subset is initial states 0, 1, 128 and 255 of
every pump (64 runs).  The oracle integrates the original couplings (SK
+-1 exactly; the Gaussian matrix's float32 values), so the stored states
are the exact method's, not those of any rounded storage.  States are
stored as float32 (a relative rounding of 6e-8, far below the errors the
test reports).
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2308_02329_amd import synth  # noqa: E402

N, D, STEPS, R, N_IC = 1000, 4, 10000, 4096, 256
PUMPS = np.linspace(0.5, 2.0, 16)
IC_SUBSET = (0, 1, 128, 255)
PARAMS = dict(btil=1.0, eta=2e-4, dt=0.01)
OUT = os.path.join(HERE, "precision_n1000_d4.npz")


def precision_n1000_inputs():
    """Seeded inputs of the precision workload: couplings, float32 eps per
    coupling, pumps, initial states, annealing table, subset indices."""
    J = {"sk": synth.sk_pm1(N, 3, 0), "gauss": synth.gaussian_j(N, 3, 1)}
    eps = {k: float(np.float32(synth.default_eps(v))) for k, v in J.items()}
    pump = synth.pump_grid(N_IC, PUMPS)
    x0 = synth.initial_states(N, R, D, 3, 2)
    alpha, ss = synth.anneal_schedule(STEPS, D)
    idx = np.array([k * N_IC + i for k in range(len(PUMPS)) for i in IC_SUBSET], dtype=np.int64)
    return J, eps, pump, x0, alpha, idx


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    J, eps, pump, x0, alpha, idx = precision_n1000_inputs()
    out = {"idx": idx, "input_digest": np.array(digest(J["sk"], J["gauss"], pump, x0, alpha))}
    p = {k: float(np.float32(v)) for k, v in PARAMS.items()}
    for kind in ("sk", "gauss"):
        t0 = time.time()
        xo = oracle.ode_run(J[kind].astype(np.float64), pump[idx], x0[:, idx, :], eps=eps[kind], steps=STEPS,
                            alpha=alpha, **p)
        out[f"x_{kind}"] = xo.astype(np.float32)
        out[f"eps_{kind}"] = np.float32(eps[kind])
        print(f"{kind}: {time.time() - t0:.0f} s, max |x| {np.abs(xo).max():.3f}", flush=True)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
