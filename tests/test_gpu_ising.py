"""Exact Ising energy through the C ABI against the oracle, int8 couplings.

Problems of n <= 1024 take the one-replica-per-lane kernel (row masks of the
+-1 entries by ballot, popcounts, other magnitudes one by one), larger ones
the one-replica-per-wavefront walk; both must give the oracle's integer
energy exactly, for ragged n and r, couplings of every magnitude and an
asymmetric J with a nonzero diagonal.
"""
import numpy as np
import pytest

import oracle
from paper_2308_02329_amd import api

torch = pytest.importorskip("torch")
from gpu_helpers import pack_spins, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu


def mixed_j(n, seed):
    rng = np.random.default_rng(seed)
    J = rng.choice(np.array([-2, -1, -1, 0, 0, 1, 1, 2], dtype=np.int8), size=(n, n))
    k = max(1, n // 10)  # a few extreme entries
    J[rng.integers(0, n, k), rng.integers(0, n, k)] = 127
    J[rng.integers(0, n, k), rng.integers(0, n, k)] = -128
    return J


@pytest.mark.parametrize("n,r", [(1, 3), (63, 70), (64, 64), (65, 130), (100, 257), (129, 65), (1000, 67),
                                 (1024, 64), (1025, 33), (2048, 9)])
def test_int8_energy_exact(n, r):
    rng = np.random.default_rng(n * 1000 + r)
    sig = rng.choice(np.array([-1, 1], dtype=np.int8), size=(r, n))
    spins = to_dev(pack_spins(sig))
    for J in (mixed_j(n, 7 + n), np.sign(mixed_j(n, 8 + n)).astype(np.int8)):
        want = oracle.ising_energy(J, sig)
        e32 = torch.full((r,), 123456789, dtype=torch.int32, device="cuda")
        e64 = torch.full((r,), float("nan"), dtype=torch.float64, device="cuda")
        api.chym_ising_energy(to_dev(J), spins, e32, e64)
        np.testing.assert_array_equal(e32.cpu().numpy(), want.astype(np.int32))
        np.testing.assert_array_equal(e64.cpu().numpy(), want)
