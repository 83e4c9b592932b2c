"""GPU checks of the float32 form's exact split and of the launch plans."""
import numpy as np
import pytest

from paper_2308_02329_amd import api, synth

torch = pytest.importorskip("torch")
from gpu_helpers import Case, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu


def bf16_rne_bits(x32: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even float32 -> bf16 bit patterns (finite inputs)."""
    b = x32.view(np.uint32).astype(np.uint64)
    rounding = ((b >> 16) & 1) + 0x7FFF
    return ((b + rounding) >> 16).astype(np.uint16)


def bits_to_f64(h: np.ndarray) -> np.ndarray:
    return (h.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def test_split3_is_exact_and_rne():
    """hi + mid + lo == x exactly and hi = RNE(x) while the residual terms
    stay normal floats (|x| >= 2^-100); below that the smallest terms may be
    flushed to zero, bounded by 2^-8 |x|."""
    g = np.random.default_rng(0)
    mags = 10.0 ** g.uniform(-37, 30, 1 << 16)
    x = (g.choice([-1.0, 1.0], mags.size) * mags).astype(np.float32)
    x[:8] = [0.0, -0.0, 1.0, -1.0, 3.0e-3, 1.0 + 2 ** -23, -(1.0 + 2 ** -8), 65504.0]
    # values sitting exactly on bf16 rounding ties, at O(1) and at small magnitude
    k = np.arange(1, 1025, dtype=np.uint32)
    ties = np.concatenate([((0x3F80 + k) << 16 | 0x8000), ((0x0C00 + k) << 16 | 0x8000)]).view(np.float32)
    x = np.concatenate([x, ties, -ties]).astype(np.float32)
    x = x[: x.size // 8 * 8]
    hi, mid, lo = api.chym_split3_bf16(to_dev(x))
    hi, mid, lo = (t.cpu().numpy().view(np.uint16) for t in (hi, mid, lo))
    np.testing.assert_array_equal(hi, bf16_rne_bits(x))
    total = bits_to_f64(hi) + bits_to_f64(mid) + bits_to_f64(lo)
    x64 = x.astype(np.float64)
    big = np.abs(x64) >= 2.0 ** -100
    assert big.sum() > 60000
    assert np.array_equal(total[big], x64[big])
    assert np.all(np.abs(total[~big] - x64[~big]) <= 2.0 ** -8 * np.abs(x64[~big]) + 2.0 ** -126)


@pytest.mark.parametrize("n,d,prec", [(100, 2, "f32"), (100, 3, "bf16"), (40, 4, "f32"), (150, 1, "f32")])
@pytest.mark.parametrize("kernel,waves", [(2, 2), (2, 4), (3, 4), (3, 1)])
def test_lds_plan_matches_register_plan_bit_exact(n, d, prec, kernel, waves):
    lds_vs_register_plan(n, d, prec, kernel, waves)


@pytest.mark.parametrize("n,d,prec", [(100, 2, "f32"), (40, 4, "f32"), (150, 1, "f32"), (60, 3, "bf16"),
                                      (100, 2, "bf16")])
@pytest.mark.parametrize("waves", [4, 2])
def test_three_wave_lds_plan_matches_register_plan_bit_exact(n, d, prec, waves):
    lds_vs_register_plan(n, d, prec, api.CHYM_KERNEL_LDSJ3, waves)


def lds_vs_register_plan(n, d, prec, kernel, waves):
    specs = [(n, d, 70, 150), (n, d, 33, 120), (n, d, 16, 150)]
    cases = [Case(nn, dd, r, s, key=(30, i)) for i, (nn, dd, r, s) in enumerate(specs)]

    def run():
        tasks = []
        for c, (_, _, r, s) in zip(cases, specs):
            Jd, pump, x, alpha = c.gpu_inputs()
            tasks.append(dict(J=Jd, pump=pump, x=x, alpha=alpha, steps=s, precision=prec, **c.params()))
        b = api.chym_batch_create(tasks)
        b.launch()
        torch.cuda.synchronize()
        b.destroy()
        return [t["x"].cpu().numpy() for t in tasks]

    api.chym_plan_set(n, d, prec, torch.int8, api.CHYM_KERNEL_REGJ, 4)
    ref = run()
    api.chym_plan_set(n, d, prec, torch.int8, kernel, waves)
    assert api.chym_plan_get(n, d, prec, torch.int8)["kernel"] == kernel
    got = run()
    api.chym_plan_set(n, d, prec, torch.int8, api.CHYM_KERNEL_AUTO, 4)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("n,d,prec", [(100, 3, "f32"), (100, 2, "f32"), (100, 3, "bf16"), (80, 3, "f32"),
                                      (40, 2, "bf16"), (20, 3, "f32")])
def test_pipelined_plan_matches_register_plan_bit_exact(n, d, prec):
    """The software-pipelined kind gives the register-resident kind's results
    bit for bit: every tail of its two-step loop (1, 2, 3 and 4 steps, odd
    and even longer runs), even and odd chunk counts (n = 80: three chunks),
    ragged replica counts, and start steps inside the annealing ramp."""
    specs = [(n, d, 70, 151), (n, d, 33, 150), (n, d, 16, 1), (n, d, 17, 2), (n, d, 20, 3), (n, d, 64, 4)]
    cases = [Case(nn, dd, r, max(s, 1), key=(31, i)) for i, (nn, dd, r, s) in enumerate(specs)]

    def run(start):
        tasks = []
        for c, (_, _, r, s) in zip(cases, specs):
            Jd, pump, x, _ = c.gpu_inputs()
            al = to_dev(synth.anneal_schedule(400, d)[0])  # start steps inside the ramp (0.4 .. 0.8 of 400)
            tasks.append(dict(J=Jd, pump=pump, x=x, alpha=al, steps=s, start_step=start, precision=prec,
                              **c.params()))
        b = api.chym_batch_create(tasks)
        b.launch()
        torch.cuda.synchronize()
        b.destroy()
        return [t["x"].cpu().numpy() for t in tasks]

    for start in (0, 157):
        api.chym_plan_set(n, d, prec, torch.int8, api.CHYM_KERNEL_REGJ, 4)
        ref = run(start)
        api.chym_plan_set(n, d, prec, torch.int8, api.CHYM_KERNEL_PIPE, 4)
        assert api.chym_plan_get(n, d, prec, torch.int8)["kernel"] == api.CHYM_KERNEL_PIPE
        got = run(start)
        api.chym_plan_set(n, d, prec, torch.int8, api.CHYM_KERNEL_AUTO, 4)
        for a, b, sp in zip(ref, got, specs):
            assert np.array_equal(a, b), (sp, start)


def test_pipelined_plan_refused_where_not_built():
    with pytest.raises(api.ChymError) as ei:
        api.chym_plan_set(100, 4, "f32", torch.int8, api.CHYM_KERNEL_PIPE, 4)
    assert ei.value.code == -2
    with pytest.raises(api.ChymError):
        api.chym_plan_set(100, 3, "f32", torch.float32, api.CHYM_KERNEL_PIPE, 4)  # three coupling terms


def test_autotune_installs_a_candidate(tmp_path):
    best, cands = api.chym_plan_autotune(48, 2, "f32", torch.int8, replicas=4096, steps=50)
    assert len(cands) == 6 and all(c["ms"] > 0 for c in cands)  # the pipelined and three-wave kinds are built
    assert {api.CHYM_KERNEL_PIPE, api.CHYM_KERNEL_LDSJ3} <= {c["kernel"] for c in cands}
    assert best["ms"] == min(c["ms"] for c in cands)
    assert api.chym_plan_get(48, 2, "f32", torch.int8)["kernel"] == best["kernel"]
    path = tmp_path / "plans.txt"
    api.chym_plan_save(path)
    api.chym_plan_set(48, 2, "f32", torch.int8, api.CHYM_KERNEL_AUTO)
    api.chym_plan_load(path)
    assert api.chym_plan_get(48, 2, "f32", torch.int8)["kernel"] == best["kernel"]
    api.chym_plan_set(48, 2, "f32", torch.int8, api.CHYM_KERNEL_AUTO)


@pytest.mark.parametrize("n,d,kind", [(200, 4, "sk"), (200, 2, "gauss"), (400, 3, "sk"), (520, 2, "sk"),
                                      (800, 2, "gauss"), (500, 4, "gauss")])
def test_streamed_j_block_sizes_bit_exact(n, d, kind):
    """The streamed-J kernel's blocks of 8 and of 16 wavefronts (1, 2 or 4
    row tiles each) give the same results bit for bit, in single calls and
    in a batch with ragged replica counts; +-1 couplings take the E4M3 J
    stream, Gaussian bf16 couplings the bf16 one (sixteen-wavefront blocks
    hold 1, 2 or, at d <= 2, 4 row tiles per wavefront)."""
    g = np.random.default_rng(n + d)
    Jh = synth.sk_pm1(n, 61, n) if kind == "sk" else synth.gaussian_j(n, 61, n).astype(np.float32)
    J = to_dev(Jh) if kind == "sk" else to_dev(Jh).to(torch.bfloat16)
    eps = float(np.float32(0.5 / synth.lambda_max(Jh.astype(np.float64))))
    steps = 120
    al = to_dev(synth.anneal_schedule(steps, d)[0])
    specs = [40, 16, 3]
    x0s = [g.standard_normal((n, r, d)).astype(np.float32) * 1e-2 for r in specs]
    pumps = [to_dev(g.uniform(0.5, 2.0, r).astype(np.float32)) for r in specs]

    def run(waves):
        api.chym_plan_set(n, d, "bf16", J.dtype if kind != "sk" else torch.int8, api.CHYM_KERNEL_SLAB, waves)
        singles = []
        for x0, p in zip(x0s, pumps):
            x = to_dev(x0)
            ws = torch.empty(api.chym_integrate_workspace_size(J, x, precision="bf16") + 256, dtype=torch.uint8,
                             device="cuda")
            api.chym_integrate(J, p, x, al, eps=eps, btil=1.0, eta=2e-4, dt=0.01, steps=steps, precision="bf16",
                               workspace=ws)
            singles.append(x)
        tasks = [dict(J=J, pump=p, x=to_dev(x0), alpha=al, steps=steps, precision="bf16", eps=eps, btil=1.0, eta=2e-4,
                      dt=0.01) for x0, p in zip(x0s, pumps)]
        b = api.chym_batch_create(tasks)
        b.launch()
        torch.cuda.synchronize()
        b.destroy()
        return [x.cpu().numpy() for x in singles], [t["x"].cpu().numpy() for t in tasks]

    s8, b8 = run(8)
    s16, b16 = run(16)
    api.chym_plan_set(n, d, "bf16", J.dtype if kind != "sk" else torch.int8, api.CHYM_KERNEL_AUTO)
    for a, b_, c, e in zip(s8, s16, b8, b16):
        assert np.array_equal(a, b_) and np.array_equal(a, c) and np.array_equal(a, e)
        assert np.isfinite(a).all()


def test_autotune_streamed_j_shape():
    """The autotuner times the streamed-J block sizes of a variant beyond the
    register-resident limit and installs the faster."""
    best, cands = api.chym_plan_autotune(400, 4, "bf16", torch.int8, replicas=2048, steps=40)
    assert sorted(c["waves"] for c in cands) == [8, 16]
    assert all(c["kernel"] == api.CHYM_KERNEL_SLAB and c["ms"] > 0 for c in cands)
    assert best["kernel"] == api.CHYM_KERNEL_SLAB and best["ms"] == min(c["ms"] for c in cands)
    assert api.chym_plan_get(400, 4, "bf16", torch.int8)["waves"] == best["waves"]
    best32, cands32 = api.chym_plan_autotune(400, 2, "f32", torch.int8, replicas=1024, steps=20)
    assert [c["waves"] for c in cands32] == [8]  # sixteen-wavefront blocks are built for the bf16 form only
    for nn, dd, pp in ((400, 4, "bf16"), (400, 2, "f32")):
        api.chym_plan_set(nn, dd, pp, torch.int8, api.CHYM_KERNEL_AUTO)
