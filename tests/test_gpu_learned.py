"""GPU kernels of the learned early restart against the FP64 reference."""
import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_2308_02329_amd import api, synth

torch = pytest.importorskip("torch")
from gpu_helpers import pack_spins, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,d,kind", [(100, 3, "sk"), (70, 1, "gauss"), (200, 2, "sk")])
def test_features_match_oracle(n, d, kind):
    r = 37
    g = np.random.default_rng(n)
    J = synth.sk_pm1(n, 50, n) if kind == "sk" else synth.gaussian_j(n, 50, n)
    x_prev = g.standard_normal((n, r, d)).astype(np.float32)
    x = (x_prev + 0.7 * g.standard_normal((n, r, d))).astype(np.float32)
    x[3, 2] = 0.0
    words = api.chym_sign_words(to_dev(x_prev))
    np.testing.assert_array_equal(words.cpu().numpy(), pack_spins(oracle.readout(x_prev)))
    feat = torch.zeros((r, 32), dtype=torch.float32, device="cuda")
    api.chym_features(to_dev(J), to_dev(x), words, feat, 2)
    ref, sig = mlp.features(J, x, oracle.readout(x_prev))
    f = feat.cpu().numpy()
    assert not f[:, :8].any() and not f[:, 12:].any()
    np.testing.assert_allclose(f[:, 8:12], ref, rtol=2e-6, atol=1e-6)
    np.testing.assert_array_equal(words.cpu().numpy(), pack_spins(sig))


def test_mlp_kernels_match_reference():
    g = np.random.default_rng(7)
    b = 301
    w32 = (g.standard_normal(mlp.PARAMS) * 0.2).astype(np.float32)
    x = g.standard_normal((b, 32)).astype(np.float32)
    y = (g.random(b) < 0.4).astype(np.float32)
    wd = to_dev(w32)
    wb = api.chym_to_bf16(wd)
    wr = mlp.bf16_round(w32)
    np.testing.assert_array_equal(((wb.cpu().numpy().view(np.uint16).astype(np.uint32)) << 16).view(np.float32),
                                  wr.astype(np.float32))
    xd, yd = to_dev(x), to_dev(y)
    h1 = torch.empty((b, 128), dtype=torch.float32, device="cuda")
    h2 = torch.empty((b, 128), dtype=torch.float32, device="cuda")
    logit = api.chym_mlp_forward(xd, wb, None, h1, h2)
    z, rh1, rh2 = mlp.forward(x, wr)
    np.testing.assert_allclose(logit.cpu().numpy(), z, rtol=1e-4, atol=1e-4)
    np.testing.assert_allclose(h1.cpu().numpy(), rh1, rtol=1e-4, atol=1e-5)
    scratch = torch.empty(api.chym_mlp_scratch_floats(b), dtype=torch.float32, device="cuda")
    grad = torch.empty(mlp.PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(b, dtype=torch.float32, device="cuda")
    api.chym_mlp_backward(xd, yd, wb, logit, h1, h2, scratch, grad, loss)
    gref = mlp.grad(x, y, wr)
    gg = grad.cpu().numpy()
    np.testing.assert_allclose(gg, gref, rtol=0, atol=2e-4 * np.abs(gref).max())
    assert np.corrcoef(gg, gref)[0, 1] > 0.99999
    np.testing.assert_allclose(loss.cpu().numpy().mean(), mlp.loss(x, y, wr), rtol=1e-5)
    # deterministic
    grad2 = torch.empty_like(grad)
    api.chym_mlp_backward(xd, yd, wb, logit, h1, h2, scratch, grad2, loss)
    assert torch.equal(grad, grad2)
    m = torch.zeros_like(grad)
    v = torch.zeros_like(grad)
    w0 = wd.clone()
    api.chym_mlp_adam(wd, wb, m, v, grad, lr=1e-2, t=1)
    wn, mn, vn = mlp.adam(w32.astype(np.float64), 0.0, 0.0, gg.astype(np.float64), 1e-2, 1)
    np.testing.assert_allclose(wd.cpu().numpy(), wn, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(m.cpu().numpy(), mn, rtol=1e-6)
    assert not torch.equal(w0, wd)


def test_mlp_training_learns_a_rule():
    g = np.random.default_rng(3)
    b = 4096
    x = g.standard_normal((b, 32)).astype(np.float32)
    y = ((x[:, 0] + 0.5 * x[:, 5] - 0.3 * x[:, 17]) > 0.2).astype(np.float32)
    from paper_2308_02329_amd.learned import RestartNet

    net = RestartNet(seed=0)
    xd, yd = to_dev(x), to_dev(y)
    first = net.train_step(xd, yd, lr=3e-3)
    for _ in range(300):
        last = net.train_step(xd, yd, lr=3e-3)
    assert last < 0.25 < first
    p = torch.sigmoid(net.logits(xd)).cpu().numpy()
    assert ((p > 0.5) == (y > 0.5)).mean() > 0.95


def test_restart_policy_on_simulated_trajectories():
    """Train on trajectories the integrator generates (N=100 SK, D=3) and
    compare time-to-99%-ground-state with and without restarts."""
    import math

    from paper_2308_02329_amd import learned

    rep = learned.experiment(n_train=20, n_val=5, n_test=8, n=100, n_ic=500, n_pumps=20, steps=5000, epochs=3,
                             n_ic_eval=2000, search_steps=20000, log=None)
    print({k: v for k, v in rep.items() if k not in ("per_instance", "loss_history")})
    tts = rep["tts99_median_ms"]
    # the chosen policy is never worse than no restart on the validation instances
    base = rep["tts99_val_geomean_without_restart_ms"]
    best_val = min([v["tts99_val_geomean_ms"] for v in rep["validation"]] + [base])
    assert best_val <= base
    assert rep["chosen_epoch"] == -1 or best_val < base
    # what the network learned carries over to unseen instances
    assert rep["auc_heldout"] > 0.55
    assert rep["positives_train"] > 0
    # BF16 with learned restarts beats the plain FP32 method
    assert math.isfinite(tts["bf16_learned"]) and tts["bf16_learned"] < tts["plain_f32"]
    assert rep["updates_per_s"]["bf16"] > rep["updates_per_s"]["f32"]
