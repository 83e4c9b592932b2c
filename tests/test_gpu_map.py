"""The round-trip map of Eq. (2) on the GPU (chym_map_integrate) against the
oracle's literal map.

Parameters follow the parameter paragraph (kappa L = 0.1, beta b^2 = 25) with
b = d = 0.01 per round trip; the coupling magnitude is eps gamma / b with
eps = 0.5 / lambda_max, pumps h = r h_th with h_th the uncoupled threshold
-ln((1 - b)(1 - d)) / (kappa L).

Tolerance (float32 form): amplitudes are O(sqrt(gamma / beta b^2)) ~ 0.03.
Each round trip adds about five float32 roundings of relative size 2^-24
(the medium's gain 2 P e / ((P + h) + (P - h) e^2) needs a square root, an
exponential and a division; the contraction is exact), so over 2000 round
trips the errors, if they accumulated coherently, would reach 2000 * 5 *
2^-24 = 6e-4 of the amplitude scale; the bar is 5e-4 of the largest
amplitude (measured up to 1.3e-4).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2308_02329_amd import api, synth

torch = pytest.importorskip("torch")
from gpu_helpers import to_dev  # noqa: E402

pytestmark = pytest.mark.gpu
B = DD = 0.01
KL = 0.1
BB2 = 25.0


def setup(n, d, r, steps, key, anneal=False, kind="sk"):
    J8 = synth.sk_pm1(n, *key) if kind == "sk" else synth.er_pm1(n, *key)
    gamma = B + DD
    eps = 0.5 / synth.lambda_max(J8) if n > 1 else 0.1
    jmag = float(np.float32(eps * gamma / B))
    hth = -math.log((1 - B) * (1 - DD)) / KL
    rr = np.linspace(1.1, 2.0, r)
    h = (rr * hth).astype(np.float32)
    A0 = (synth.initial_states(n, r, d, *key, sigma=0.1) * math.sqrt(gamma / BB2)).astype(np.float32)
    alpha = synth.anneal_schedule(steps, d)[0] if anneal else synth.constant_schedule(steps, d)
    return J8, jmag, h, A0, alpha


def run_gpu(J8, jmag, h, A0, alpha, steps, precision="f32", start=0, A=None, J=None):
    Ad = to_dev(A0) if A is None else A
    api.chym_map_integrate(to_dev(J8) if J is None else J, to_dev(h), Ad, to_dev(alpha), b=B, loss=DD, kl=KL,
                           beta_b2=BB2, jmag=jmag, steps=steps, start_step=start, precision=precision)
    return Ad


def run_oracle(J8, jmag, h, A0, alpha, steps):
    # the oracle takes the coupling values themselves and beta (not beta b^2)
    return oracle.map_run(jmag * J8.astype(np.float64), h.astype(np.float64), A0.astype(np.float64), B, DD, KL,
                          BB2 / (B * B), steps, alpha)


@pytest.mark.parametrize("n,d,r,anneal", [(16, 2, 40, True), (40, 3, 33, False), (100, 1, 20, False),
                                          (100, 4, 17, True), (112, 3, 16, True), (7, 2, 5, False)])
def test_map_parity_f32(n, d, r, anneal):
    steps = 2000
    J8, jmag, h, A0, alpha = setup(n, d, r, steps, (70, n, d), anneal)
    Ag = run_gpu(J8, jmag, h, A0, alpha, steps).cpu().numpy().astype(np.float64)
    Ao = run_oracle(J8, jmag, h, A0, alpha, steps)
    scale = np.abs(Ao).max()
    assert scale > 1e-3  # above threshold: the amplitudes grew
    err = np.abs(Ag - Ao).max()
    print(f"n={n} d={d}: max |dA| = {err:.3e}, relative to the amplitude scale {err / scale:.2e}")
    assert err <= 5e-4 * scale, (err, scale)
    assert np.array_equal(oracle.readout(Ag), oracle.readout(Ao))


def test_map_split_run_equals_whole_run():
    n, d, r, steps = 48, 3, 20, 600
    J8, jmag, h, A0, alpha = setup(n, d, r, steps, (71,), anneal=True)
    whole = run_gpu(J8, jmag, h, A0, alpha, steps).cpu().numpy()
    A = to_dev(A0)
    for k0, k1 in [(0, 250), (250, 600)]:
        run_gpu(J8, jmag, h, A0, alpha, k1 - k0, start=k0, A=A)
    assert np.array_equal(A.cpu().numpy(), whole)


def test_map_bf16_form_and_storages():
    n, d, r, steps = 64, 2, 32, 1000
    J8, jmag, h, A0, alpha = setup(n, d, r, steps, (72,))
    Ao = run_oracle(J8, jmag, h, A0, alpha, steps)
    Ab = run_gpu(J8, jmag, h, A0, alpha, steps, precision="bf16").cpu().numpy()
    scale = np.abs(Ao).max()
    assert 0.0 < np.abs(Ab - Ao).max() < 5e-2 * scale
    # +-1 couplings are exact in every storage: identical trajectories
    ref = run_gpu(J8, jmag, h, A0, alpha, steps).cpu().numpy()
    Jbf = to_dev(J8.astype(np.float32)).to(torch.bfloat16)
    assert np.array_equal(run_gpu(J8, jmag, h, A0, alpha, steps, J=Jbf).cpu().numpy(), ref)
    Jf8 = api.chym_quantize_fp8(to_dev(J8.astype(np.float32)))
    assert np.array_equal(run_gpu(J8, jmag, h, A0, alpha, steps, J=Jf8).cpu().numpy(), ref)


def test_map_small_signal_gain_and_rejections():
    # uncoupled, below saturation: one round trip multiplies A by
    # (1 - d)(1 - b) K(A) (1 - beta b^2 K^2 A^2) -- compare with the oracle's K
    n, d, r = 16, 1, 16
    J8 = np.zeros((n, n), dtype=np.int8)
    h = np.full(r, 3.0, dtype=np.float32)
    A0 = np.full((n, r, d), 1e-3, dtype=np.float32)
    alpha = synth.constant_schedule(1, d)
    Ag = run_gpu(J8, 1.0, h, A0, alpha, 1).cpu().numpy()
    K = oracle.nlm_gain(1e-3, 3.0, KL)
    Bv = K * 1e-3
    want = (1 - DD) * ((1 - B) * Bv - BB2 * Bv ** 3)
    np.testing.assert_allclose(Ag, want, rtol=2e-6)
    Jd, hd, Ad, ad = to_dev(J8), to_dev(h), to_dev(A0), to_dev(alpha)
    with pytest.raises(api.ChymError, match="bf16 term"):
        api.chym_map_integrate(to_dev(J8.astype(np.float32)), hd, Ad, ad, b=B, loss=DD, kl=KL, beta_b2=BB2,
                               jmag=1.0, steps=1)
    with pytest.raises(api.ChymError, match="b must"):
        api.chym_map_integrate(Jd, hd, Ad, ad, b=1.5, loss=DD, kl=KL, beta_b2=BB2, jmag=1.0, steps=1)
    big = np.zeros((120, 120), dtype=np.int8)
    with pytest.raises(api.ChymError, match="map form runs"):
        api.chym_map_integrate(to_dev(big), hd, to_dev(np.zeros((120, r, 1), np.float32)), ad, b=B, loss=DD, kl=KL,
                               beta_b2=BB2, jmag=1.0, steps=1)


def test_map_batch_equals_single_calls():
    # several kernel variants in one call (row tiles, d, precision), ragged
    # replica counts, different step counts within a variant, a zero-step task
    specs = [(16, 2, 40, 700, True, "f32"), (40, 3, 33, 500, False, "f32"), (40, 3, 20, 900, True, "f32"),
             (100, 1, 21, 300, False, "bf16"), (7, 2, 5, 0, False, "f32"), (33, 4, 18, 400, True, "f32"),
             (112, 2, 16, 250, True, "f32")]
    singles, tasks = [], []
    for k, (n, d, r, steps, anneal, prec) in enumerate(specs):
        J8, jmag, h, A0, alpha = setup(n, d, r, max(steps, 1), (73, k), anneal, kind="er" if k % 2 else "sk")
        singles.append(run_gpu(J8, jmag, h, A0, alpha, steps, precision=prec).cpu().numpy())
        tasks.append(dict(J=to_dev(J8), h=to_dev(h), A=to_dev(A0), alpha=to_dev(alpha), b=B, loss=DD, kl=KL,
                          beta_b2=BB2, jmag=jmag, steps=steps, precision=prec))
    ws = api.chym_map_batch(tasks)
    torch.cuda.synchronize()
    del ws
    for k, (t, want) in enumerate(zip(tasks, singles)):
        assert np.array_equal(t["A"].cpu().numpy(), want), k
    # and against the oracle for one task of the batch
    n, d, r, steps, anneal, _ = specs[2]
    J8, jmag, h, A0, alpha = setup(n, d, r, steps, (73, 2), anneal, kind="sk")
    Ao = run_oracle(J8, jmag, h, A0, alpha, steps)
    assert np.abs(tasks[2]["A"].cpu().numpy() - Ao).max() <= 5e-4 * np.abs(Ao).max()


def test_map_batch_repeat_and_errors():
    n, d, r, steps = 24, 2, 48, 300
    J8, jmag, h, A0, alpha = setup(n, d, r, steps, (74,), True)
    want = run_gpu(J8, jmag, h, A0, alpha, steps).cpu().numpy()
    for _ in range(2):  # the work counters start from zero on every call
        t = dict(J=to_dev(J8), h=to_dev(h), A=to_dev(A0), alpha=to_dev(alpha), b=B, loss=DD, kl=KL, beta_b2=BB2,
                 jmag=jmag, steps=steps)
        api.chym_map_batch([t, dict(t, A=to_dev(A0))])
        torch.cuda.synchronize()
        assert np.array_equal(t["A"].cpu().numpy(), want)
    bad = dict(t, b=1.5)
    A_before = t["A"].clone()
    with pytest.raises(api.ChymError, match="task 1"):
        api.chym_map_batch([t, bad])
    assert torch.equal(t["A"], A_before)  # nothing launched
