"""Precision forms of the coupling storage on the GPU: FP8 (OCP E4M3 values
with one E8M0 exponent per row) and BF16 couplings.

* chym_quantize_fp8 writes the same bytes as the oracle's quantizer
  (bit-exact: it is byte work).
* float32 form on FP8 / BF16 couplings: the stored couplings are exact in
  one bf16 term, so the trajectory follows the oracle's run on the decoded
  couplings to the float32-form tolerance (1e-4), readout and energies
  exact or to float64 rounding.
* BF16 form on BF16 couplings equals the BF16 form on the float32 couplings
  they were rounded from (the kernel rounds J to bf16 to nearest even, as
  the conversion of the input did): bit-exact.
* Error of each form against the FP64 oracle on the original Gaussian
  couplings, printed as a table and bounded loosely (not a parity gate:
  it measures the precision form, rounding of J included).
"""
import numpy as np
import pytest

import oracle
from oracle import fp8
from paper_2308_02329_amd import api, synth

torch = pytest.importorskip("torch")
from gpu_helpers import Case, to_dev, unpack_spins  # noqa: E402

pytestmark = pytest.mark.gpu
TOL_F32 = 1e-4


def fp8_bytes(Jf):
    codes, expo = fp8.quantize(Jf)
    return fp8.pack(codes, expo), fp8.decode(codes, expo)


@pytest.mark.parametrize("n", [1, 17, 64, 333, 1000])
def test_quantize_matches_oracle(n):
    J = synth.gaussian_j(n, 60, n).astype(np.float32)
    if n >= 17:
        J[3] = 0.0                      # all-zero row
        J[5, 7] = np.inf                # non-finite row
        J[9] *= 1e-30                   # tiny row (exponent near the bottom of the range)
        J[11] *= 3e4                    # large row
    ref = fp8.pack(*fp8.quantize(J))
    got = api.chym_quantize_fp8(to_dev(J)).cpu().numpy()
    np.testing.assert_array_equal(got, ref)
    assert api.chym_j_bytes(n, api.CHYM_J_FP8) == n * (n + 1)


def _run(case, Jd, precision="f32", steps=None):
    _, pump, x, alpha = case.gpu_inputs()
    api.chym_integrate(Jd, pump, x, alpha, steps=case.steps if steps is None else steps, precision=precision,
                       **case.params())
    return x


@pytest.mark.parametrize("n,d,kind", [(40, 3, "fp8"), (100, 2, "fp8"), (97, 4, "bf16"), (300, 2, "fp8"),
                                      (250, 3, "bf16")])
def test_stored_couplings_f32_form_parity(n, d, kind):
    case = Case(n, d, 24, 300, key=(61, n, d), kind="gauss", sigma=0.05)
    Jf = case.J.astype(np.float32)
    if kind == "fp8":
        raw, Jdec = fp8_bytes(Jf)
        Jd = to_dev(raw)
    else:
        Jd = to_dev(Jf).to(torch.bfloat16)
        Jdec = Jd.float().cpu().numpy().astype(np.float64)
    xg = _run(case, Jd).cpu().numpy()
    xo = oracle.ode_run(Jdec, case.pump, case.x0, steps=case.steps, alpha=case.alpha, **case.params())
    err = np.abs(xg - xo).max()
    assert err <= TOL_F32, err
    # scores of the GPU's final state against the decoded couplings
    xd = to_dev(xg)
    spins = torch.empty((case.r, api.spin_words(n)), dtype=torch.int64, device="cuda")
    api.chym_readout(xd, spins)
    e64 = torch.empty(case.r, dtype=torch.float64, device="cuda")
    api.chym_ising_energy(Jd, spins, None, e64)
    ehs = torch.empty(case.r, dtype=torch.float64, device="cuda")
    api.chym_hs_energy(Jd, xd, ehs)
    sig = unpack_spins(spins.cpu().numpy(), n)
    np.testing.assert_array_equal(sig, oracle.readout(xg))
    np.testing.assert_allclose(e64.cpu().numpy(), oracle.ising_energy(Jdec, sig), rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(ehs.cpu().numpy(), oracle.hs_energy(Jdec, xg), rtol=1e-12, atol=1e-9)
    with pytest.raises(api.ChymError):   # int32 energy needs integer couplings
        api.chym_ising_energy(Jd, spins, torch.empty(case.r, dtype=torch.int32, device="cuda"))


@pytest.mark.parametrize("n,d", [(100, 3), (400, 4)])
def test_bf16_couplings_equal_kernel_rounding(n, d):
    case = Case(n, d, 32, 200, key=(62, n, d), kind="gauss", sigma=0.05)
    a = _run(case, to_dev(case.J.astype(np.float32)), "bf16").cpu().numpy()
    b = _run(case, to_dev(case.J.astype(np.float32)).to(torch.bfloat16), "bf16").cpu().numpy()
    assert np.array_equal(a, b)


def test_sk_couplings_identical_in_every_storage():
    """+-1 couplings are exact in int8, bf16, float32 and FP8: every storage
    gives the same trajectory bit for bit in both forms."""
    case = Case(120, 3, 40, 300, key=(63,), sigma=0.05)
    J8 = case.J
    raw, dec = fp8_bytes(J8.astype(np.float32))
    assert np.array_equal(dec, J8.astype(np.float64))
    for prec in ("f32", "bf16"):
        ref = _run(case, to_dev(J8), prec).cpu().numpy()
        for Jd in (to_dev(raw), to_dev(J8.astype(np.float32)).to(torch.bfloat16)):
            assert np.array_equal(_run(case, Jd, prec).cpu().numpy(), ref)


def test_precision_report_against_fp64_oracle():
    """Per-form error of the final state and of the hyperspin energy against
    the FP64 oracle on the original Gaussian couplings (N = 200, D = 4, 400
    steps of the linear dynamics' onset, 32 replicas), and the readout
    agreement."""
    n, d, r, steps = 200, 4, 32, 400
    case = Case(n, d, r, steps, key=(64,), kind="gauss", sigma=0.05)
    Jf = case.J.astype(np.float32)
    xo = oracle.ode_run(case.J, case.pump, case.x0, steps=steps, alpha=case.alpha, **case.params())
    so = oracle.readout(xo)
    eo = oracle.hs_energy(case.J, xo)
    raw, _ = fp8_bytes(Jf)
    forms = {
        "f32 form, float32 J": (to_dev(Jf), "f32"),
        "bf16 form, float32 J": (to_dev(Jf), "bf16"),
        "bf16 form, bf16 J": (to_dev(Jf).to(torch.bfloat16), "bf16"),
        "f32 form, fp8 J": (to_dev(raw), "f32"),
        "bf16 form, fp8 J": (to_dev(raw), "bf16"),
    }
    rows = {}
    for name, (Jd, prec) in forms.items():
        xg = _run(case, Jd, prec).cpu().numpy()
        scale = np.abs(xo).max()
        rows[name] = dict(max_abs=float(np.abs(xg - xo).max()), rel=float(np.abs(xg - xo).max() / scale),
                          ehs_rel=float(np.abs(oracle.hs_energy(case.J, xg) - eo).max() / np.abs(eo).max()),
                          readout_agree=float((oracle.readout(xg) == so).mean()))
    for name, v in rows.items():
        print(f"{name:24s} max|dx| {v['max_abs']:.3e} (rel {v['rel']:.2e})  E_hs rel {v['ehs_rel']:.2e}  "
              f"readout agree {v['readout_agree']:.4f}")
    assert rows["f32 form, float32 J"]["max_abs"] <= TOL_F32
    assert rows["bf16 form, float32 J"]["max_abs"] == rows["bf16 form, bf16 J"]["max_abs"]
    for name, v in rows.items():
        assert v["rel"] < 0.2 and v["ehs_rel"] < 0.05, (name, v)
    # the coarser the coupling storage, the larger the error
    assert rows["f32 form, fp8 J"]["max_abs"] > rows["f32 form, float32 J"]["max_abs"]
