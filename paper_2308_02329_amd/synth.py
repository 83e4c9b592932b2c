"""Seeded synthetic inputs for the coherent hyperspin machine (CHYM).

This module only *draws inputs*: coupling matrices J_N, initial amplitudes,
pump values and the dimensional-annealing table.  It holds none of the
method's arithmetic and is the one module that both the HIP path and the FP64
oracle take their inputs from.

Instance families:

* ``sk_pm1``      -- Sherrington-Kirkpatrick graph, J_pq = +-1 with p = 1/2 for
                     every pair p < q, symmetric, zero diagonal.
* ``er_pm1``      -- the paper's own family (main text, paragraph after Fig. 2:
                     random sparse graphs of density 20 %, J_pq = +-J with a
                     random sign).  Read as Erdos-Renyi G(N, rho) conditioned on
                     being connected, magnitude 1 (the magnitude goes into eps).
* ``regular3_pm1``-- 3-regular graph by configuration-model pairing with
                     rejection, random +-1 signs.
* ``gaussian_j``  -- J_pq ~ N(0, 1) for p < q, symmetric, zero diagonal.

Randomness is numpy's PCG64 seeded through ``SeedSequence`` so that every
(config, instance, stream) triple has an independent, reproducible stream.
"""
from __future__ import annotations

import numpy as np

MASTER_SEED = 2308023290

# stream tags keep J, x0 and other draws of the same instance independent
_TAG_J = 1
_TAG_X0 = 2
_TAG_MISC = 3


def rng(*key: int) -> np.random.Generator:
    """PCG64 generator for the integer key (config, instance, tag, ...)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([MASTER_SEED, *[int(k) for k in key]])))


def sk_pm1(n: int, *key: int) -> np.ndarray:
    """SK +-1 couplings, int8 [n, n], symmetric, zero diagonal."""
    g = rng(*key, _TAG_J)
    s = g.integers(0, 2, size=(n, n), dtype=np.int8) * 2 - 1
    j = np.triu(s, 1)
    return (j + j.T).astype(np.int8)


def gaussian_j(n: int, *key: int) -> np.ndarray:
    """Gaussian couplings N(0,1), float32 [n, n], symmetric, zero diagonal."""
    g = rng(*key, _TAG_J)
    a = g.standard_normal((n, n)).astype(np.float32)
    j = np.triu(a, 1)
    return (j + j.T).astype(np.float32)


def _connected(adj: np.ndarray) -> bool:
    n = adj.shape[0]
    if n == 0:
        return True
    seen = np.zeros(n, dtype=bool)
    stack = [0]
    seen[0] = True
    while stack:
        v = stack.pop()
        for w in np.nonzero(adj[v])[0]:
            if not seen[w]:
                seen[w] = True
                stack.append(int(w))
    return bool(seen.all())


def er_pm1(n: int, *key: int, density: float = 0.2, max_tries: int = 1000) -> np.ndarray:
    """Erdos-Renyi G(n, density) conditioned on connectivity, random +-1 signs."""
    g = rng(*key, _TAG_J)
    for _ in range(max_tries):
        mask = np.triu(g.random((n, n)) < density, 1)
        adj = mask | mask.T
        if _connected(adj):
            sign = np.triu(g.integers(0, 2, size=(n, n), dtype=np.int8) * 2 - 1, 1)
            sign = sign + sign.T
            return (sign * adj).astype(np.int8)
    raise RuntimeError(f"no connected G({n}, {density}) in {max_tries} draws")


def regular3_pm1(n: int, *key: int, max_tries: int = 10000) -> np.ndarray:
    """3-regular simple graph (configuration model, rejection), random +-1 signs."""
    if n < 4 or (3 * n) % 2:
        raise ValueError("a 3-regular simple graph needs an even n >= 4")
    g = rng(*key, _TAG_J)
    stubs = np.repeat(np.arange(n), 3)
    for _ in range(max_tries):
        perm = g.permutation(stubs)
        a, b = perm[0::2], perm[1::2]
        if np.any(a == b):
            continue
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        if len(set(zip(lo.tolist(), hi.tolist()))) != len(lo):
            continue
        j = np.zeros((n, n), dtype=np.int8)
        s = (g.integers(0, 2, size=len(lo)) * 2 - 1).astype(np.int8)
        j[lo, hi] = s
        j[hi, lo] = s
        return j
    raise RuntimeError("configuration model did not produce a simple graph")


def initial_states(n: int, r: int, d: int, *key: int, sigma: float = 1e-3) -> np.ndarray:
    """i.i.d. Gaussian amplitudes, float32 [n, r, d] (row p, replica, component)."""
    g = rng(*key, _TAG_X0)
    return (g.standard_normal((n, r, d)) * sigma).astype(np.float32)


def initial_states_torch(n: int, r: int, d: int, seed: int, device, sigma: float = 1e-3):
    """Same distribution as ``initial_states`` drawn with torch's seeded device
    generator (for workloads too large to draw on the host)."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    return torch.randn((n, r, d), generator=gen, device=device, dtype=torch.float32) * sigma


def pump_grid(n_ic: int, pumps) -> np.ndarray:
    """Per-replica pump r_i, float32 [len(pumps) * n_ic].  Replica index is
    pump-major: replica k * n_ic + i uses pumps[k] and initial condition i."""
    pumps = np.asarray(pumps, dtype=np.float64)
    return np.repeat(pumps, n_ic).astype(np.float32)


def anneal_schedule(steps: int, d: int, start: float = 0.4, end: float = 0.8) -> tuple[np.ndarray, int]:
    """Dimensional-annealing table alpha[steps, d] (float32) and the
    steady-state step.

    The protocol itself lives in the paper's supplement, which is not
    available; the reading used here: the first component keeps alpha = 1;
    every other component keeps alpha = 1 until the hyperspin steady state
    (step ``start*steps``), then ramps linearly to 0 by ``end*steps`` and
    stays 0, which morphs the D-dimensional hypergraph into the Ising model.
    """
    a = np.ones((steps, d), dtype=np.float64)
    k0 = int(round(start * steps))
    k1 = int(round(end * steps))
    if d > 1 and k1 > k0:
        k = np.arange(steps)
        ramp = np.clip(1.0 - (k - k0) / float(k1 - k0), 0.0, 1.0)
        ramp[k < k0] = 1.0
        a[:, 1:] = ramp[:, None]
    return a.astype(np.float32), k0


def constant_schedule(steps: int, d: int, values=None) -> np.ndarray:
    """alpha[steps, d] constant in time (no annealing), float32."""
    v = np.ones(d) if values is None else np.asarray(values, dtype=np.float64)
    return np.tile(v[None, :], (steps, 1)).astype(np.float32)


def lambda_max(j: np.ndarray) -> float:
    """Largest eigenvalue of the symmetric coupling matrix (host FP64)."""
    return float(np.linalg.eigvalsh(np.asarray(j, dtype=np.float64))[-1])


def default_eps(j: np.ndarray, ratio: float = 0.5) -> float:
    """Coupling strength eps = ratio / lambda_max(J): the coupled threshold
    1 - eps*lambda_max then sits at pump r = 1 - ratio."""
    return ratio / lambda_max(j)
