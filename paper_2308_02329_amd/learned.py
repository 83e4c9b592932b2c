"""Learned early restart for the CHYM and its time-to-solution accounting.

A run of the machine is cheap to start and expensive to finish.  At a
decision point early in the run (default: after the first 10 % of the
Euler steps) a small network scores every run from features of its first
part (see ``chym_features`` in include/chym.h); each pump's batch of runs
keeps its highest-scored fraction, integrates only those to the end, and
starts fresh runs instead of the others.  Every kept run is still
integrated to the end and judged by its exact Ising energy, so the method's
answers are unchanged; only the cost per success changes.  Keeping every
run is the plain method, always a candidate when the policy is chosen.

Runs of one problem and pump converge to the same hyperspin configuration
up to a rotation; what tells them apart early is the orientation of the
first component, the one the anneal keeps.  The features describe it
(Rayleigh quotient, Ising energy of its signs, its share of the norm, sign
flips) at 7 checkpoints over the first part, and once more for a coarse
continuation: the decision-point state integrated through the rest of the
schedule with SURROGATE_STRIDE times the step (every SURROGATE_STRIDE-th
annealing weight), about 1/SURROGATE_STRIDE of the rest's cost.  From a
given state the rest of a run is close to deterministic, so the coarse
continuation mostly ends where the run will; the features are standardized
within each pump's batch of runs, since the policy ranks runs within such a
batch.

All arithmetic runs in libchym's kernels: the integrator, the features,
their standardization, the network's forward, backward and Adam kernels,
the top-k selection of the kept runs and their gather.  This module holds
the orchestration: data generation, the training loop, the executed policy
and the time-to-99%-success (TTS99) bookkeeping

    TTS99 = t_attempt * ln(0.01) / ln(1 - p_success_per_attempt)

(t_attempt = GPU time per attempt; p >= 0.99 gives one attempt; p = 0 gives
infinity).  With restarts an attempt costs the partial run, plus the rest of
the run for the kept fraction, and succeeds when kept and successful.

The ground-state energy of an instance is the best energy found by any run
of it and by a longer search (a putative ground state; exact ones come from
exhaustive search in the tests).

    python -m paper_2308_02329_amd.learned --out report.json
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np
import torch

from . import _lib as L
from . import api, stats, synth

N_CKPT = 8            # feature slots: N_CKPT - 1 trajectory checkpoints, then the coarse continuation
N_FEAT = L.CHYM_FEATURES
SURROGATE_STRIDE = 20  # step multiple of the coarse continuation


# ---------------------------------------------------------------- network
class RestartNet:
    """32 -> 128 -> 128 -> 1 network on the GPU: float32 master weights, a
    bf16 copy used by the forward/backward kernels, and Adam moments.  Its
    inputs are features standardized within each pump's batch of runs."""

    def __init__(self, seed: int = 0, device: str = "cuda"):
        g = np.random.default_rng(seed)
        # He initialization for the ReLU layers, zero biases
        w1 = g.standard_normal((128, 32)) * math.sqrt(2.0 / 32)
        w2 = g.standard_normal((128, 128)) * math.sqrt(2.0 / 128)
        w3 = g.standard_normal(128) * math.sqrt(1.0 / 128)
        w = np.concatenate([w1.ravel(), np.zeros(128), w2.ravel(), np.zeros(128), w3, np.zeros(1)])
        self.device = torch.device(device)
        self.w = torch.from_numpy(w.astype(np.float32)).to(self.device)
        self.wb = api.chym_to_bf16(self.w)
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.t = 0
        self._bufs = {}

    def state(self):
        return [t.clone() for t in (self.w, self.wb, self.m, self.v)] + [self.t]

    def load_state(self, st):
        for dst, src in zip((self.w, self.wb, self.m, self.v), st[:4]):
            dst.copy_(src)
        self.t = st[4]

    def _buf(self, b):
        if b not in self._bufs:
            dev = self.device
            self._bufs[b] = dict(
                h1=torch.empty((b, 128), dtype=torch.float32, device=dev),
                h2=torch.empty((b, 128), dtype=torch.float32, device=dev),
                logit=torch.empty(b, dtype=torch.float32, device=dev),
                loss=torch.empty(b, dtype=torch.float32, device=dev),
                scratch=torch.empty(api.chym_mlp_scratch_floats(b), dtype=torch.float32, device=dev),
                grad=torch.empty(L.CHYM_MLP_PARAMS, dtype=torch.float32, device=dev))
        return self._bufs[b]

    def train_step(self, xs: torch.Tensor, y: torch.Tensor, lr: float) -> float:
        """One Adam step on standardized features xs [B, 32] and labels y."""
        b = xs.shape[0]
        bf = self._buf(b)
        api.chym_mlp_forward(xs, self.wb, bf["logit"], bf["h1"], bf["h2"])
        api.chym_mlp_backward(xs, y, self.wb, bf["logit"], bf["h1"], bf["h2"], bf["scratch"], bf["grad"], bf["loss"])
        self.t += 1
        api.chym_mlp_adam(self.w, self.wb, self.m, self.v, bf["grad"], lr=lr, t=self.t)
        return float(bf["loss"].mean().item())

    def logits(self, xs: torch.Tensor) -> torch.Tensor:
        """Logits (the policy ranks by them; the sigmoid is monotone)."""
        return api.chym_mlp_forward(xs.contiguous(), self.wb)

    def fit(self, xs: torch.Tensor, y: torch.Tensor, epochs: int = 4, batch: int = 8192, lr: float = 2e-3,
            seed: int = 0, pos_frac: float = 0.0, log=None) -> list:
        """Mini-batch training; returns epoch losses.  pos_frac > 0 draws that
        share of every batch from the positives (with replacement): rare
        successes are otherwise a handful per batch."""
        g = torch.Generator(device=xs.device)
        g.manual_seed(seed)
        n = xs.shape[0]
        batch = min(batch, n)
        pos = torch.nonzero(y > 0.5).flatten()
        neg = torch.nonzero(y <= 0.5).flatten()
        n_pos = int(round(pos_frac * batch)) if pos_frac > 0 and len(pos) and len(neg) else 0
        hist = []
        for ep in range(epochs):
            tot, cnt = 0.0, 0
            if n_pos:
                for _ in range(max(1, n // batch)):
                    ip = pos[torch.randint(len(pos), (n_pos,), generator=g, device=xs.device)]
                    ineg = neg[torch.randint(len(neg), (batch - n_pos,), generator=g, device=xs.device)]
                    idx = torch.cat([ip, ineg])
                    tot += self.train_step(xs[idx].contiguous(), y[idx].contiguous(), lr)
                    cnt += 1
            else:
                perm = torch.randperm(n, generator=g, device=xs.device)
                for s in range(0, n - batch + 1, batch):
                    idx = perm[s:s + batch]
                    tot += self.train_step(xs[idx].contiguous(), y[idx].contiguous(), lr)
                    cnt += 1
            hist.append(tot / max(cnt, 1))
            if log:
                log(f"epoch {ep}: loss {hist[-1]:.4f}")
        return hist


# ------------------------------------------------------------- simulation
def checkpoints(steps, frac=0.1, n_ckpt=N_CKPT - 1):
    """The n_ckpt trajectory checkpoints (step counts) spread over the first
    `frac` of the run; the last one is the decision point."""
    k_feat = max(n_ckpt, int(round(frac * steps)))
    return [int(round(k_feat * (c + 1) / n_ckpt)) for c in range(n_ckpt)]


class Problem:
    """One SK instance with its run inputs on the device."""

    def __init__(self, Jn, d=3, steps=20000, dt=0.01, eta=2e-4, device="cuda"):
        self.Jn = Jn
        self.n, self.d, self.steps = Jn.shape[0], d, steps
        self.dev = torch.device(device)
        self.J = torch.from_numpy(Jn).to(self.dev)
        self.alpha = torch.from_numpy(synth.anneal_schedule(steps, d)[0]).to(self.dev)
        self.prm = dict(eps=float(np.float32(synth.default_eps(Jn))), btil=1.0, eta=eta, dt=dt)

    def integrate(self, pump, x, k0, k1, precision, ws=None):
        if k1 > k0:
            api.chym_integrate(self.J, pump, x, self.alpha, steps=k1 - k0, start_step=k0, precision=precision,
                               workspace=ws, **self.prm)

    def workspace(self, x, precision):
        nb = api.chym_integrate_workspace_size(self.J, x, precision=precision)
        return torch.empty(nb + 256, dtype=torch.uint8, device=self.dev) if nb else None

    def energies(self, x):
        r = x.shape[1]
        spins = torch.empty((r, api.spin_words(self.n)), dtype=torch.int64, device=self.dev)
        api.chym_readout(x, spins)
        e = torch.empty(r, dtype=torch.int32, device=self.dev)
        api.chym_ising_energy(self.J, spins, e)
        return e

    def features(self, pump, x, group, precision, ws, frac=0.1, stride=SURROGATE_STRIDE):
        """Phase one of a run: integrate x to the decision point, taking the
        features at the trajectory checkpoints, then those of the coarse
        continuation of a copy of the decision-point state (last slot);
        returns them standardized within each pump batch of `group` runs,
        and the decision step."""
        r = x.shape[1]
        feats = torch.zeros((r, N_FEAT), dtype=torch.float32, device=self.dev)
        words = api.chym_sign_words(x)
        k = 0
        for c, kc in enumerate(checkpoints(self.steps, frac)):
            self.integrate(pump, x, k, kc, precision, ws)
            api.chym_features(self.J, x, words, feats, c)
            k = kc
        xs = x.clone()
        al = self.alpha[k::stride].contiguous()  # every stride-th annealing weight of the rest
        if al.shape[0]:
            api.chym_integrate(self.J, pump, xs, al, steps=al.shape[0], start_step=0, precision=precision,
                               workspace=ws, **dict(self.prm, dt=self.prm["dt"] * stride))
        api.chym_features(self.J, xs, words, feats, N_CKPT - 1)
        api.chym_feature_standardize(feats, group, out=feats)
        return feats, k


def run_with_features(prob: Problem, pump, x0, group, precision="bf16", frac=0.1):
    """Every run to the end, with the features of its first part: (features
    [R, 32], Ising energies [R], GPU ms of the first part, GPU ms of the
    rest)."""
    x = x0.clone()
    ws = prob.workspace(x, precision)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    feats, k = prob.features(pump, x, group, precision, ws, frac)
    e1.record()
    prob.integrate(pump, x, k, prob.steps, precision, ws)
    e = prob.energies(x)
    e2.record()
    torch.cuda.synchronize()
    return feats, e, e0.elapsed_time(e1), e1.elapsed_time(e2)


def run_plain(prob: Problem, pump, x0, precision):
    """The plain method: every run to the end, no features.  (energies, ms)."""
    x = x0.clone()
    ws = prob.workspace(x, precision)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    prob.integrate(pump, x, 0, prob.steps, precision, ws)
    e = prob.energies(x)
    e1.record()
    torch.cuda.synchronize()
    return e, e0.elapsed_time(e1)


def run_policy(prob: Problem, net: RestartNet, pump, x0, group, keep, precision="bf16", frac=0.1):
    """The restart policy executed: every run to the decision point with
    features, the network's scores, the ceil(keep * group) best of each pump
    batch gathered into a compact state and integrated to the end, their
    exact energies.  Returns (kept global indices [R // group, m], their
    energies [R // group * m], GPU ms of the whole)."""
    x = x0.clone()
    r = x.shape[1]
    m = max(1, int(math.ceil(keep * group)))
    ws = prob.workspace(x, precision)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    feats, k = prob.features(pump, x, group, precision, ws, frac)
    logit = net.logits(feats)
    idx = api.chym_select_top(logit, group, m)
    xk, pk = api.chym_gather_replicas(x, idx, pump=pump)
    wk = prob.workspace(xk, precision)
    prob.integrate(pk, xk, k, prob.steps, precision, wk)
    e = prob.energies(xk)
    e1.record()
    torch.cuda.synchronize()
    assert r % group == 0
    return idx, e, e0.elapsed_time(e1)


def instance(index, n=200, config=5):
    return synth.sk_pm1(n, config, index)


def initial_states(prob, r, seed):
    return synth.initial_states_torch(prob.n, r, prob.d, seed=seed, device=prob.dev)


def generate(indices, n=200, d=3, n_ic=1000, pumps=np.linspace(0.5, 2.0, 20), steps=20000, frac=0.1,
             precision="bf16", seed_base=7, log=None):
    """Runs of the instances (n_ic initial states x each pump) with features
    of their first part.  Returns per-instance dicts."""
    out = []
    for i in indices:
        prob = Problem(instance(i, n), d, steps)
        pr = torch.from_numpy(synth.pump_grid(n_ic, pumps)).to(prob.dev)
        x0 = initial_states(prob, pr.shape[0], seed_base * 1000003 + i)
        f, e, t_part, t_rest = run_with_features(prob, pr, x0, n_ic, precision, frac)
        out.append(dict(index=i, Jn=prob.Jn, feats=f, E=e, t_part_ms=t_part, t_rest_ms=t_rest, n_ic=n_ic,
                        pumps=np.asarray(pumps), steps=steps))
        if log:
            log(f"instance {i}: {precision} {t_part + t_rest:.1f} ms, best E {int(e.min().item())}")
    return out


# -------------------------------------------------------------- accounting
tts99 = stats.tts99


def auc(scores, labels):
    """Area under the ROC curve (rank statistic)."""
    scores = np.asarray(scores, dtype=np.float64)
    labels = np.asarray(labels, dtype=bool)
    npos, nneg = labels.sum(), (~labels).sum()
    if npos == 0 or nneg == 0:
        return float("nan")
    order = np.argsort(scores, kind="mergesort")
    ranks = np.empty(len(scores))
    ranks[order] = np.arange(1, len(scores) + 1)
    # average ranks of ties
    s_sorted = scores[order]
    i = 0
    while i < len(s_sorted):
        j = i
        while j + 1 < len(s_sorted) and s_sorted[j + 1] == s_sorted[i]:
            j += 1
        if j > i:
            ranks[order[i:j + 1]] = (i + j + 2) / 2.0
        i = j + 1
    return float((ranks[labels].sum() - npos * (npos + 1) / 2) / (npos * nneg))


def within_batch_auc(scores, labels, group):
    """Mean AUC over the pump batches (groups of consecutive runs) that hold
    both outcomes: how well the scores rank runs within a batch, the only
    ranking the policy uses."""
    s = np.asarray(scores).reshape(-1, group)
    y = np.asarray(labels, dtype=bool).reshape(-1, group)
    vals = [auc(a, b) for a, b in zip(s, y) if 0 < b.sum() < group]
    return float(np.mean(vals)) if vals else float("nan")


def instance_tts(inst, egs, q=None, keep=1.0):
    """Best-pump TTS99 (ms) of an instance from its runs with features (the
    cost model: the measured first part for every run, the measured rest for
    the kept ones).  With scores q, the restart policy keeps, in every
    pump's batch of runs, the ceil(keep * n_ic) runs with the highest scores
    at the decision point (ties by run index); keep = 1 is the plain
    method."""
    e = inst["E"].cpu().numpy()
    succ = e == egs
    R = len(e)
    t_part = inst["t_part_ms"] / R
    t_full = (inst["t_part_ms"] + inst["t_rest_ms"]) / R
    best = math.inf
    n_ic = inst["n_ic"]
    for k in range(R // n_ic):
        sl = slice(k * n_ic, (k + 1) * n_ic)
        s = succ[sl]
        if q is None or keep >= 1.0:
            t = tts99(t_full, s.mean())
        else:
            m = max(1, int(math.ceil(keep * n_ic)))
            kept = np.zeros(n_ic, dtype=bool)
            kept[np.argsort(-np.asarray(q[sl]), kind="stable")[:m]] = True
            cost = t_part + (m / n_ic) * (t_full - t_part)
            t = tts99(cost, (kept & s).mean())
        best = min(best, t)
    return best


def validation_score(tts, base):
    """Score of a restart policy on validation instances: the geometric mean
    of its best-pump TTS99 over the instances the plain method solves (base
    finite), or inf if it loses any of them.  A median would let a policy
    that kills every success of a minority of instances look best."""
    tts = np.asarray(tts, dtype=np.float64)
    ok = np.isfinite(np.asarray(base, dtype=np.float64))
    if not ok.any() or not np.all(np.isfinite(tts[ok])):
        return math.inf
    return float(np.exp(np.mean(np.log(tts[ok]))))


KEEP_GRID = (1.0, 0.7, 0.5, 0.3, 0.2, 0.1, 0.05, 0.02, 0.01)


def choose_keep(insts, egs, net, grid=KEEP_GRID):
    """Kept fraction with the lowest validation_score on insts (1, never
    restart, is always feasible).  Returns (keep, score in ms)."""
    qs = [net.logits(i["feats"]).cpu().numpy() for i in insts]
    base = [instance_tts(i, g) for i, g in zip(insts, egs)]
    best = (math.inf, 1.0)
    for kf in grid:
        sc = validation_score([instance_tts(i, g, q, kf) for i, g, q in zip(insts, egs, qs)], base)
        if sc < best[0]:
            best = (sc, float(kf))
    return best[1], best[0]


def search_egs(Jn, n_rep=20000, d=3, steps=20000, dt=0.01, seed=0, device="cuda"):
    """Best Ising energy of long BF16 runs (pumps r in [1.0, 2.0]): a
    stronger putative ground state than the runs under test find."""
    dev = torch.device(device)
    n = Jn.shape[0]
    pumps = np.linspace(1.0, 2.0, 10)
    pr = torch.from_numpy(synth.pump_grid(n_rep // 10, pumps)).to(dev)
    x = synth.initial_states_torch(n, pr.shape[0], d, seed=seed, device=dev)
    al = torch.from_numpy(synth.anneal_schedule(steps, d)[0]).to(dev)
    out = api.chym_solve(torch.from_numpy(Jn).to(dev), pr, x, al, eps=float(np.float32(synth.default_eps(Jn))),
                         btil=1.0, eta=2e-4, dt=dt, steps=steps, precision="bf16", want=("spins", "e_ising"))
    return int(out["e_ising"].min().item())


def bootstrap_ratio(num, den, reps=2000, seed=0):
    """Geometric mean of num / den over instances with a 95 % bootstrap
    interval (resampling instances)."""
    r = np.log(np.asarray(num, dtype=np.float64) / np.asarray(den, dtype=np.float64))
    if r.size == 0:
        return math.nan, (math.nan, math.nan)
    g = np.random.default_rng(seed)
    boots = [np.exp(np.mean(r[g.integers(0, r.size, r.size)])) for _ in range(reps)]
    return float(np.exp(r.mean())), (float(np.percentile(boots, 2.5)), float(np.percentile(boots, 97.5)))


def evaluate_instance(i, net, keep, n=200, d=3, steps=20000, pilot_ic=1000, eval_ic=20000, n_eval_pumps=3,
                      pumps=np.linspace(0.5, 2.0, 20), search_steps=20000, frac=0.1, seed_base=11):
    """One held-out instance: a plain BF16 pilot over every pump picks its
    n_eval_pumps best pumps; there, from the same eval_ic fresh initial
    states per pump, the plain FP32 form, the plain BF16 form and the BF16
    form with the restart policy are run and timed end to end.  The
    putative ground state is the best energy of all of these and of a longer
    search.  Returns the per-method best-pump TTS99 (measured costs), the
    success counts and the cost model's prediction for the policy."""
    prob = Problem(instance(i, n), d, steps)
    pr = torch.from_numpy(synth.pump_grid(pilot_ic, pumps)).to(prob.dev)
    e_pilot, _ = run_plain(prob, pr, initial_states(prob, pr.shape[0], seed_base * 1000003 + i), "bf16")
    ep = e_pilot.cpu().numpy().reshape(len(pumps), pilot_ic)
    counts = (ep == ep.min()).sum(axis=1)
    chosen = np.sort(np.argsort(-counts, kind="stable")[:n_eval_pumps])
    pe = np.asarray(pumps)[chosen]
    pr = torch.from_numpy(synth.pump_grid(eval_ic, pe)).to(prob.dev)
    x0 = initial_states(prob, pr.shape[0], (seed_base + 1) * 1000003 + i)
    e_f32, ms_f32 = run_plain(prob, pr, x0, "f32")
    e_bf, ms_bf = run_plain(prob, pr, x0, "bf16")
    idx, e_kept, ms_pol = run_policy(prob, net, pr, x0, eval_ic, keep, "bf16", frac)
    f_cm, e_cm, t_part, t_rest = run_with_features(prob, pr, x0, eval_ic, "bf16", frac)
    egs = min(int(ep.min()), int(e_f32.min().item()), int(e_bf.min().item()))
    if search_steps:
        egs = min(egs, search_egs(prob.Jn, d=d, steps=search_steps, seed=7 + i))
    R = pr.shape[0]
    m = idx.shape[1]
    s_f32 = (e_f32.cpu().numpy() == egs).reshape(len(pe), eval_ic)
    s_bf = (e_bf.cpu().numpy() == egs).reshape(len(pe), eval_ic)
    s_pol = (e_kept.cpu().numpy() == egs).reshape(len(pe), m)
    # the kept runs followed the same trajectories as in the plain BF16 run
    same = bool(np.array_equal(e_kept.cpu().numpy(), e_bf.cpu().numpy()[idx.cpu().numpy().ravel()]))
    t = {"plain_f32": min(tts99(ms_f32 / R, s.mean()) for s in s_f32),
         "bf16": min(tts99(ms_bf / R, s.mean()) for s in s_bf),
         "bf16_learned": min(tts99(ms_pol / R, s.sum() / eval_ic) for s in s_pol)}
    model_cost = (t_part + (m / eval_ic) * t_rest) / R
    lab = (e_cm.cpu().numpy() == egs)
    return dict(index=i, egs=egs, pumps=pe.tolist(), tts99_ms=t, successes={
        "plain_f32": s_f32.sum(axis=1).tolist(), "bf16": s_bf.sum(axis=1).tolist(),
        "bf16_learned": s_pol.sum(axis=1).tolist()},
        ms_per_attempt={"plain_f32": ms_f32 / R, "bf16": ms_bf / R, "bf16_learned": ms_pol / R,
                        "bf16_learned_model": model_cost},
        kept_match_plain=same, auc_within=within_batch_auc(net.logits(f_cm).cpu().numpy(), lab, eval_ic))


def experiment(n_train=50, n_val=10, n_test=20, n=200, d=3, n_ic=1000, n_pumps=20, steps=20000, epochs=6, seed=0,
               frac=0.1, pos_frac=0.1, lr=2e-3, search_steps=20000, val_ic=2500, eval_ic=20000, pilot_ic=1000,
               log=print):
    """Generate, train, choose the policy, evaluate; returns a JSON-able
    report.

    Training instances (n_train x n_pumps x n_ic runs, BF16 form) give the
    features and labels (final energy == putative ground state).  After
    every epoch the kept fraction is chosen on the validation instances
    (val_ic runs per pump) by validation_score with the cost model; the
    epoch and fraction with the lowest score win, keeping every run (the
    plain method) always a candidate.  Held-out instances are evaluated by
    evaluate_instance: the three methods run for real at each instance's
    best pumps, from the same initial states."""
    t0 = time.time()
    pumps = np.linspace(0.5, 2.0, n_pumps)
    kw = dict(n=n, d=d, pumps=pumps, steps=steps, frac=frac, log=None)
    train = generate(range(n_train), n_ic=n_ic, **kw)
    val = generate(range(5000, 5000 + n_val), n_ic=val_ic, **kw)

    def putative(insts):
        out = []
        for i in insts:
            e = int(i["E"].min().item())
            if search_steps:
                e = min(e, search_egs(i["Jn"], d=d, steps=search_steps, seed=7 + i["index"]))
            out.append(e)
        return out

    egs_train, egs_val = putative(train), putative(val)
    feats = torch.cat([i["feats"] for i in train])
    labels = torch.cat([(i["E"] == g).float() for i, g in zip(train, egs_train)])
    if log:
        log(f"data: {feats.shape[0]} training runs, {int(labels.sum().item())} successes, {time.time() - t0:.1f} s")
    net = RestartNet(seed=seed)
    t_fit = time.time()
    hist, val_curve = [], []
    base_tts = [instance_tts(i, g) for i, g in zip(val, egs_val)]
    base_val = validation_score(base_tts, base_tts)
    best = (base_val, 1.0, -1, net.state())  # never restart
    for ep in range(epochs):
        hist += net.fit(feats, labels, epochs=1, lr=lr, pos_frac=pos_frac, seed=seed * 1000 + ep)
        kf, sc_val = choose_keep(val, egs_val, net)
        val_curve.append(dict(epoch=ep, keep=kf, tts99_val_geomean_ms=sc_val))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4f} val TTS99 (geometric mean) {sc_val:.4f} ms (keep {kf:.3g}), "
                f"without restarts {base_val:.4f} ms")
        if sc_val < best[0]:
            best = (sc_val, kf, ep, net.state())
    net.load_state(best[3])
    keep = best[1]
    torch.cuda.synchronize()
    t_fit = time.time() - t_fit
    val_lab = np.concatenate([(i["E"].cpu().numpy() == g) for i, g in zip(val, egs_val)])
    val_auc = within_batch_auc(np.concatenate([net.logits(i["feats"]).cpu().numpy() for i in val]), val_lab, val_ic)
    rows = []
    for k in range(n_test):
        row = evaluate_instance(10000 + k, net, keep, n=n, d=d, steps=steps, pilot_ic=pilot_ic, eval_ic=eval_ic,
                                pumps=pumps, search_steps=search_steps, frac=frac)
        rows.append(row)
        if log:
            log(f"held-out {row['index']}: TTS99 ms " + ", ".join(f"{a} {b:.3g}" for a, b in row["tts99_ms"].items())
                + f"; successes {row['successes']}")
    fin = lambda key: [r["tts99_ms"][key] for r in rows]  # noqa: E731
    solved = {m: [math.isfinite(v) for v in fin(m)] for m in ("plain_f32", "bf16", "bf16_learned")}
    both = [a and b for a, b in zip(solved["bf16"], solved["bf16_learned"])]
    ratio, ci = bootstrap_ratio([v for v, ok in zip(fin("bf16_learned"), both) if ok],
                                [v for v, ok in zip(fin("bf16"), both) if ok])
    both32 = [a and b for a, b in zip(solved["plain_f32"], solved["bf16_learned"])]
    ratio_f32, ci_f32 = bootstrap_ratio([v for v, ok in zip(fin("bf16_learned"), both32) if ok],
                                        [v for v, ok in zip(fin("plain_f32"), both32) if ok], seed=1)
    cost = {m: float(np.mean([r["ms_per_attempt"][m] for r in rows]))
            for m in ("plain_f32", "bf16", "bf16_learned", "bf16_learned_model")}
    report = dict(
        workload=f"SK +-1 N={n}, D={d}, {n_pumps} pumps, {steps} Euler steps, decision after {frac:.0%} of the steps "
                 f"({N_CKPT - 1} feature checkpoints and a continuation at {SURROGATE_STRIDE}x the step); "
                 f"{n_train} training instances x {n_ic} runs per pump, {n_val} validation "
                 f"instances x {val_ic}; {n_test} held-out instances, each run at its 3 best pumps (pilot of "
                 f"{pilot_ic} runs per pump) from the same {eval_ic} initial states per pump by every method",
        trajectories_train=int(feats.shape[0]), positives_train=float(labels.mean().item()),
        loss_history=hist, validation=val_curve, tts99_val_geomean_without_restart_ms=base_val,
        chosen_epoch=best[2], keep_fraction=keep, train_seconds=t_fit, auc_within_batch_val=val_auc,
        auc_within_batch_heldout=float(np.nanmean([r["auc_within"] for r in rows])),
        tts99_median_ms={m: float(np.median(fin(m))) for m in ("plain_f32", "bf16", "bf16_learned")},
        instances_solved={m: int(sum(v)) for m, v in solved.items()},
        same_instances_solved=solved["bf16"] == solved["bf16_learned"],
        learned_over_bf16_geomean=ratio, learned_over_bf16_ci95=ci,
        learned_over_f32_geomean=ratio_f32, learned_over_f32_ci95=ci_f32,
        ms_per_attempt=cost, kept_runs_match_plain=all(r["kept_match_plain"] for r in rows),
        per_instance=rows, seconds=time.time() - t0)
    return report


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=50)
    ap.add_argument("--val", type=int, default=10)
    ap.add_argument("--test", type=int, default=20)
    ap.add_argument("--n", type=int, default=200)
    ap.add_argument("--d", type=int, default=3)
    ap.add_argument("--ics", type=int, default=1000)
    ap.add_argument("--pumps", type=int, default=20)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--frac", type=float, default=0.1)
    ap.add_argument("--eval-ic", type=int, default=20000)
    ap.add_argument("--search-steps", type=int, default=20000)
    ap.add_argument("--out", type=str, default="")
    a = ap.parse_args()
    rep = experiment(a.train, a.val, a.test, a.n, a.d, a.ics, a.pumps, a.steps, a.epochs, frac=a.frac,
                     search_steps=a.search_steps, eval_ic=a.eval_ic)
    s = json.dumps(rep, default=float)
    if a.out:
        with open(a.out, "w") as f:
            f.write(s)
    print(json.dumps({k: v for k, v in rep.items() if k not in ("per_instance", "loss_history")}, default=float))


if __name__ == "__main__":
    main()
