"""Shared helpers of the GPU tests: run the HIP path through the C ABI and
the oracle on the same seeded inputs."""
from __future__ import annotations

import numpy as np
import torch

from paper_2308_02329_amd import api, synth

DEV = "cuda:0"


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def unpack_spins(words: np.ndarray, n: int) -> np.ndarray:
    """uint64 words [r][w] -> sigma [r][n] in {-1, +1}."""
    w = words.view(np.uint64)
    r = w.shape[0]
    out = np.empty((r, n), dtype=np.int8)
    for p in range(n):
        bit = (w[:, p // 64] >> np.uint64(p % 64)) & np.uint64(1)
        out[:, p] = np.where(bit == 1, 1, -1)
    return out


def pack_spins(sigma: np.ndarray) -> np.ndarray:
    r, n = sigma.shape
    w = (n + 63) // 64
    words = np.zeros((r, w), dtype=np.uint64)
    for p in range(n):
        words[:, p // 64] |= (sigma[:, p] > 0).astype(np.uint64) << np.uint64(p % 64)
    return words.view(np.int64)


class Case:
    """A seeded problem: J, pumps, initial states and annealing table."""

    def __init__(self, n, d, r, steps, *, key=(0,), kind="sk", anneal=True, eta=2e-4, btil=1.0,
                 dt=0.01, pumps=None, eps=None, sigma=1e-3):
        self.n, self.d, self.r, self.steps = n, d, r, steps
        gen = {"sk": synth.sk_pm1, "gauss": synth.gaussian_j, "er": synth.er_pm1,
               "reg3": synth.regular3_pm1}[kind]
        self.J = gen(n, *key)
        self.x0 = synth.initial_states(n, r, d, *key, sigma=sigma)
        if pumps is None:
            pumps = np.linspace(0.5, 2.0, r).astype(np.float32)
        self.pump = np.asarray(pumps, dtype=np.float32)
        if anneal:
            self.alpha, self.ss = synth.anneal_schedule(steps, d)
        else:
            self.alpha, self.ss = synth.constant_schedule(steps, d), 0
        if eps is None:
            eps = synth.default_eps(self.J) if n > 1 else 0.1
        self.eps = float(np.float32(eps))
        self.btil, self.eta, self.dt = float(np.float32(btil)), float(np.float32(eta)), float(np.float32(dt))

    def params(self):
        # the oracle receives exactly the float32 values the device sees
        return dict(eps=self.eps, btil=self.btil, eta=self.eta, dt=self.dt)

    def gpu_inputs(self):
        return (to_dev(self.J), to_dev(self.pump), to_dev(self.x0), to_dev(self.alpha))


def gpu_integrate(case: Case, x=None, steps=None, start=0, precision="f32", J=None):
    Jd, pump, x0, alpha = case.gpu_inputs()
    if J is not None:
        Jd = J
    xd = x0 if x is None else x
    api.chym_integrate(Jd, pump, xd, alpha, steps=case.steps if steps is None else steps, start_step=start,
                       precision=precision, **case.params())
    return xd
