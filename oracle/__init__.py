"""FP64 CPU oracle of the coherent hyperspin machine -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls it, and the two share no
code: the only common dependency is the seeded input generator module,
which holds none of the method's arithmetic.

The arithmetic lives in ``chym_oracle.c`` (plain C, FP64, no fused
multiply-add); this file only marshals numpy arrays.  Every function cites
the passage of arXiv 2308.02329 it follows in the C source.

Parity status of each routine (how it is pinned, see tests/test_oracle_*):

* ode_run        -- pinned: uncoupled fixed point, linear closed form via
                    eigendecomposition / matrix products, D = 1 reduction to
                    the CIM, gauge / Z2 / O(D) covariance, Eq. (2) limit.
* map_run        -- pinned: small-signal gain, K against RK4 of the
                    coupled-mode equations, convergence to ode_run, the
                    annealing weight alpha_{mu,tau} by the linearised map's
                    closed form (eigendecomposition, alpha per component)
                    and by explicit products (non-symmetric J, alpha per
                    round trip started mid-table), split runs.
* readout, ising_energy, bruteforce_gs -- pinned by exhaustive enumeration
                    in pure Python and by the spin-flip symmetry.
* hs_energy      -- pinned: D = 1 equals the Ising energy, two-spin closed
                    form, rotation invariance, spectral lower bound.
* anneal_gs      -- heuristic (putative ground state); checked against the
                    exhaustive search where that is feasible.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chym_oracle.c")
# CHYM_SANITIZED_LIBS=1: an AddressSanitizer + UndefinedBehaviorSanitizer build
# (clang, so that it shares the ASan runtime of the library's sanitized build)
_SANITIZE = os.environ.get("CHYM_SANITIZED_LIBS") == "1"
_LIB = os.path.join(_HERE, "liboracle_san.so" if _SANITIZE else "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i8p = ctypes.POINTER(ctypes.c_int8)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, OpenMP); with
    CHYM_SANITIZED_LIBS=1, with clang and the address and undefined-behaviour
    sanitizers instead."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        if _SANITIZE:
            cmd = ["/opt/rocm/lib/llvm/bin/clang", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fopenmp",
                   "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                   "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        else:
            cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                   "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i, d = ctypes.c_int, ctypes.c_double
        lib.oracle_ode_run.argtypes = [i, i, i, _dp, _dp, _dp, d, d, d, d, i, i, _dp, i]
        lib.oracle_ode_run.restype = i
        lib.oracle_map_run.argtypes = [i, i, i, _dp, _dp, _dp, d, d, d, d, i, i, _dp, i]
        lib.oracle_map_run.restype = i
        lib.oracle_nlm_gain.argtypes = [d, d, d]
        lib.oracle_nlm_gain.restype = d
        lib.oracle_readout.argtypes = [i, i, i, _dp, _i8p]
        lib.oracle_ising_energy.argtypes = [i, i, _dp, _i8p, _dp]
        lib.oracle_hs_energy.argtypes = [i, i, i, _dp, _dp, _dp]
        lib.oracle_extra_frac.argtypes = [i, i, i, _dp, _dp]
        lib.oracle_diverged.argtypes = [i, i, i, _dp, _u8p]
        lib.oracle_bruteforce_gs.argtypes = [i, _dp, _i8p]
        lib.oracle_bruteforce_gs.restype = d
        lib.oracle_anneal_gs.argtypes = [i, _dp, i, i, ctypes.c_uint64, d, d, _i8p, i]
        lib.oracle_anneal_gs.restype = d
        lib.oracle_max_threads.restype = i
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def ode_run(J, pump, x, eps, btil, eta, dt, steps, alpha, start_step=0, nthreads=0):
    """Forward-Euler integration of the normalized CHYM equations.

    J [n,n]; pump [r]; x [n,r,d] (copied, not modified); alpha [>= start+steps, d].
    Returns the state after ``steps`` steps as float64 [n,r,d]."""
    lib = _load()
    J = _f64(J)
    pump = _f64(pump)
    xs = _f64(x).copy()
    alpha = _f64(alpha)
    n, r, d = xs.shape
    assert J.shape == (n, n) and pump.shape == (r,)
    assert alpha.ndim == 2 and alpha.shape[1] == d and alpha.shape[0] >= start_step + steps
    rc = lib.oracle_ode_run(n, d, r, _ptr(J), _ptr(pump), _ptr(xs), eps, btil, eta, dt,
                            int(steps), int(start_step), _ptr(alpha), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle_ode_run failed ({rc})")
    return xs


def map_run(J, h, A, b, dd, kl, beta, steps, alpha, start_step=0, nthreads=0):
    """Literal round-trip map of Eq. (2); J holds the coupling values."""
    lib = _load()
    J = _f64(J)
    h = _f64(h)
    As = _f64(A).copy()
    alpha = _f64(alpha)
    n, r, d = As.shape
    rc = lib.oracle_map_run(n, d, r, _ptr(J), _ptr(h), _ptr(As), b, dd, kl, beta,
                            int(steps), int(start_step), _ptr(alpha), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle_map_run failed ({rc})")
    return As


def nlm_gain(a, h, kl) -> float:
    return float(_load().oracle_nlm_gain(float(a), float(h), float(kl)))


def readout(x):
    """sigma [r, n] int8 from x [n, r, d]."""
    xs = _f64(x)
    n, r, d = xs.shape
    s = np.empty((r, n), dtype=np.int8)
    _load().oracle_readout(n, r, d, _ptr(xs), _ptr(s, _i8p))
    return s


def ising_energy(J, sigma):
    """E [r] float64 for sigma [r, n] (+-1)."""
    J = _f64(J)
    s = np.ascontiguousarray(sigma, dtype=np.int8)
    r, n = s.shape
    E = np.empty(r, dtype=np.float64)
    _load().oracle_ising_energy(n, r, _ptr(J), _ptr(s, _i8p), _ptr(E))
    return E


def hs_energy(J, x):
    J = _f64(J)
    xs = _f64(x)
    n, r, d = xs.shape
    E = np.empty(r, dtype=np.float64)
    _load().oracle_hs_energy(n, r, d, _ptr(J), _ptr(xs), _ptr(E))
    return E


def extra_frac(x):
    xs = _f64(x)
    n, r, d = xs.shape
    f = np.empty(r, dtype=np.float64)
    _load().oracle_extra_frac(n, r, d, _ptr(xs), _ptr(f))
    return f


def diverged(x):
    xs = _f64(x)
    n, r, d = xs.shape
    f = np.empty(r, dtype=np.uint8)
    _load().oracle_diverged(n, r, d, _ptr(xs), _ptr(f, _u8p))
    return f


def bruteforce_gs(J):
    """(E_GS, one minimizing sigma) by exhaustive Gray-code search."""
    J = _f64(J)
    n = J.shape[0]
    best = np.empty(max(n, 1), dtype=np.int8)
    e = _load().oracle_bruteforce_gs(n, _ptr(J), _ptr(best, _i8p))
    return float(e), best[:n].copy()


def anneal_gs(J, sweeps=2000, restarts=64, seed=1, t_hot=None, t_cold=0.05, nthreads=0):
    """Putative ground state by simulated annealing with restarts."""
    J = _f64(J)
    n = J.shape[0]
    if t_hot is None:
        t_hot = max(1.0, 2.0 * float(np.abs(J).sum(axis=1).max()))
    best = np.empty(max(n, 1), dtype=np.int8)
    e = _load().oracle_anneal_gs(n, _ptr(J), int(sweeps), int(restarts), int(seed) & (2**64 - 1),
                                 float(t_hot), float(t_cold), _ptr(best, _i8p), int(nthreads))
    return float(e), best[:n].copy()
