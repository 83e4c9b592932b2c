"""Sparse-row (ELL) couplings on the GPU: the gather integrator and the
scoring kernels against the FP64 oracle run on the same couplings as a dense
matrix.

Tolerance: the gather sums at most w products in float32 (fused
multiply-adds) against the oracle's float64, and the update is the same
float32 arithmetic as the dense kernels, so the float32-form bar of 1e-4
applies.  Energies of +-1 couplings are sums of small integers: exact."""
import numpy as np
import pytest

import oracle
from paper_2308_02329_amd import api, synth

torch = pytest.importorskip("torch")
from gpu_helpers import Case, pack_spins, to_dev, unpack_spins  # noqa: E402

pytestmark = pytest.mark.gpu


def ell_dev(J, width=None):
    return to_dev(api.ell_pack(J, width))


def run(case, Jd, precision="f32", x=None, steps=None):
    _, pump, x0, alpha = case.gpu_inputs()
    xd = x0 if x is None else x
    api.chym_integrate(Jd, pump, xd, alpha, steps=case.steps if steps is None else steps, precision=precision,
                       **case.params())
    return xd


@pytest.mark.parametrize("n,d,r,kind", [(16, 2, 37, "reg3"), (50, 3, 5, "reg3"), (200, 4, 40, "reg3"),
                                        (800, 3, 20, "reg3"), (100, 2, 33, "er"), (40, 1, 16, "sk"),
                                        (64, 4, 3, "er"), (300, 2, 20, "er")])
def test_sparse_parity_with_oracle(n, d, r, kind):
    # (300, 2, 20, "er"): about 60 nonzeros per row, rows past the LDS budget, read from global memory
    case = Case(n, d, r, 500, key=(80, n, d), kind=kind, sigma=0.05)
    xg = run(case, ell_dev(case.J)).cpu().numpy()
    xo = oracle.ode_run(case.J, case.pump, case.x0, steps=case.steps, alpha=case.alpha, **case.params())
    err = np.abs(xg - xo).max()
    assert err <= 1e-4, err
    assert np.abs(xo).max() > 0.1


def test_sparse_scores_and_solve():
    n, d, r = 120, 3, 48
    case = Case(n, d, r, 400, key=(81,), kind="reg3", sigma=0.05)
    Jell = ell_dev(case.J)
    xg = run(case, Jell).cpu().numpy()
    xd = to_dev(xg)
    spins = torch.empty((r, api.spin_words(n)), dtype=torch.int64, device="cuda")
    api.chym_readout(xd, spins)
    e64 = torch.empty(r, dtype=torch.float64, device="cuda")
    api.chym_ising_energy(Jell, spins, None, e64)
    sig = unpack_spins(spins.cpu().numpy(), n)
    np.testing.assert_array_equal(e64.cpu().numpy(), oracle.ising_energy(case.J, sig))
    ehs = torch.empty(r, dtype=torch.float64, device="cuda")
    api.chym_hs_energy(Jell, xd, ehs)
    np.testing.assert_allclose(ehs.cpu().numpy(), oracle.hs_energy(case.J, xg), rtol=1e-12, atol=1e-9)
    # the whole run through chym_solve
    _, pump, x0, alpha = case.gpu_inputs()
    res = api.chym_solve(Jell, pump, x0, alpha, steps=case.steps, ss_step=case.ss, **case.params(),
                         want=("spins", "e_ising_f64", "e_hs"))
    assert np.array_equal(x0.cpu().numpy(), xg)
    np.testing.assert_array_equal(res["spins"].cpu().numpy(), pack_spins(sig))
    np.testing.assert_array_equal(res["e_ising_f64"].cpu().numpy(), oracle.ising_energy(case.J, sig))


@pytest.mark.parametrize("n,d,r", [(96, 2, 32), (800, 3, 8), (400, 4, 12)])
def test_sparse_register_path_equals_lds_path(n, d, r):
    """Rows of width 3 with at most four (row, replica) units per thread take
    the register path; the same couplings padded to width 4 (a zero coupling,
    which adds an exact zero) take the LDS path.  Bit-identical, with 2, 4
    and 4 units per thread."""
    case = Case(n, d, r, 200, key=(85, n, d), kind="reg3", sigma=0.05)
    a = run(case, ell_dev(case.J)).cpu().numpy()
    b = run(case, ell_dev(case.J, width=4)).cpu().numpy()
    assert np.array_equal(a, b)


def test_sparse_register_path_short_rows():
    """Rows of width 2 (a +-1 ring) and mixed widths 0-3 on the register
    path (unused slots skipped) against the same couplings padded to width 4
    (LDS path) and against the oracle."""
    n, d, r = 150, 3, 20
    case = Case(n, d, r, 300, key=(86,), kind="reg3", sigma=0.05)
    g = np.random.default_rng(86)
    ring = np.zeros((n, n), dtype=np.int8)
    for p in range(n):
        q = (p + 1) % n
        ring[p, q] = ring[q, p] = 1 if g.random() < 0.5 else -1
    mixed = case.J.copy()
    mixed[:10, :] = 0  # rows with no couplings
    mixed[:, :10] = 0
    for J in (ring, mixed):
        case.J = J
        a = run(case, ell_dev(J)).cpu().numpy()
        b = run(case, ell_dev(J, width=4)).cpu().numpy()
        assert np.array_equal(a, b)
        xo = oracle.ode_run(J, case.pump, case.x0, steps=case.steps, alpha=case.alpha, **case.params())
        assert np.abs(a - xo).max() <= 1e-4


def test_sparse_padding_precision_forms_and_dense_agreement():
    n, d, r = 96, 2, 32
    case = Case(n, d, r, 300, key=(82,), kind="reg3", sigma=0.05)
    a = run(case, ell_dev(case.J)).cpu().numpy()
    b = run(case, ell_dev(case.J, width=7)).cpu().numpy()  # zero-coupling padding adds exact zeros
    assert np.array_equal(a, b)
    c = run(case, ell_dev(case.J), precision="bf16").cpu().numpy()  # the gather is float32 in both forms
    assert np.array_equal(a, c)
    dense = run(case, to_dev(case.J)).cpu().numpy()  # matrix-core path on the same couplings
    assert np.abs(dense - a).max() <= 1e-4


def test_sparse_header_mismatch_reads_as_uncoupled():
    n, d, r = 32, 2, 16
    case = Case(n, d, r, 200, key=(83,), kind="reg3", sigma=0.05)
    packed = api.ell_pack(case.J)
    packed[0, 0] = n + 5  # header for another size
    xg = run(case, to_dev(packed)).cpu().numpy()
    xo = oracle.ode_run(np.zeros_like(case.J), case.pump, case.x0, steps=case.steps, alpha=case.alpha,
                        **case.params())
    assert np.abs(xg - xo).max() <= 1e-5


def test_sparse_tasks_in_a_batch_equal_solo_runs():
    # sparse rows of several sizes and d (one gather group per d), ragged
    # replica counts, a task past the rows' LDS budget, and dense tasks in the
    # same batch; every task must equal its own single call bit for bit
    specs = [(120, 3, 48, "reg3", True), (400, 2, 40, "reg3", True), (64, 4, 21, "er", True),
             (800, 3, 20, "reg3", True), (40, 1, 16, "sk", True), (100, 3, 33, "sk", False),
             (48, 2, 17, "reg3", False), (300, 2, 20, "er", True)]
    tasks, want, cases = [], [], []
    for k, (n, d, r, kind, sparse) in enumerate(specs):
        case = Case(n, d, r, 300, key=(84, k), kind=kind, sigma=0.05)
        Jd = ell_dev(case.J) if sparse else to_dev(case.J)
        want.append(run(case, Jd).cpu().numpy())
        _, pump, x0, alpha = case.gpu_inputs()
        tasks.append(dict(J=Jd, pump=pump, x=x0, alpha=alpha, steps=case.steps, precision="f32", **case.params(),
                          spins=torch.empty((r, api.spin_words(n)), dtype=torch.int64, device="cuda"),
                          e_ising_f64=torch.empty(r, dtype=torch.float64, device="cuda")))
        cases.append(case)
    plan = api.chym_batch_create(tasks)
    for rep in range(3):  # graph replays: the work counters restart from zero on every launch
        for t, case in zip(tasks, cases):
            t["x"].copy_(to_dev(case.x0))
            t["spins"].fill_(-1)
            t["e_ising_f64"].fill_(float("nan"))
        plan.launch()
        torch.cuda.synchronize()
        for k, (t, w, case) in enumerate(zip(tasks, want, cases)):
            assert np.array_equal(t["x"].cpu().numpy(), w), (rep, k)
            sig = unpack_spins(t["spins"].cpu().numpy(), case.n)
            np.testing.assert_array_equal(sig, oracle.readout(w))
            np.testing.assert_array_equal(t["e_ising_f64"].cpu().numpy(), oracle.ising_energy(case.J, sig))
    plan.destroy()
