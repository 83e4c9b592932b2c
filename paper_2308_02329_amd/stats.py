"""The paper's statistical harness (statistics paragraph, Figs. 3-4) on
synthetic graphs: success probability against the pump, energy histograms,
and the three figures of merit with their finite-size scaling.

For each size N, N_g random graphs of the paper's family (Erdos-Renyi,
density 20%, connected, couplings +-1 with equal probability) are simulated
with the round-trip map of Eq. (2) (the paper's simulation model), as
  D = 1, the CIM: beta = 0, local saturation of the medium only;
  D = 2, the CHYM with dimensional annealing: beta b^2 = 25;
both with kappa L = 0.1 (the parameter paragraph), N_r repetitions at each
of N_s pumps h = h_th (1 + delta h).  All runs of one size and machine are
one chym_map_batch call (one persistent launch); the final Ising energies
come from libchym's readout and exact energy kernels.  Per graph and machine:

  P_Ising(h)  fraction of the N_r runs whose final Ising energy is E_GS;
  H_E         distribution of the final Ising energies over all runs;
  P_max       max_h P_Ising(h);
  W           the sum of P_Ising over the pumps where it is nonzero, divided
              by their number S ("W_scan": divided by N_s instead);
  dE          sum_E (E - E_GS) H_E with H_E normalized: the mean deviation
              of the final energy ("dE_per_n": divided by N).

Means over the graphs, interquartile ranges, and least-squares fits of
P_max ~ b_D exp(-a_D N) complete the report.  E_GS is exhaustive for
N <= 22; above, the best energy of every run plus a longer search (ODE
form, D = 3 with annealing).

Readings where the paper leaves values open: b = d = 0.01 per round trip;
coupling magnitude J = eps (b + d) / b with eps = 0.5 / lambda_max(J_N), so
that the coupled threshold sits at delta h = -0.5; h_th is the uncoupled
threshold -ln((1 - b)(1 - d)) / (kappa L); delta h scans [-0.5, 1.0]; the
annealing protocol is synth.anneal_schedule's; initial amplitudes are
Gaussian with standard deviation 0.1 sqrt((b + d) / 25).

    python -m paper_2308_02329_amd.stats --out stats.json
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np
import torch

from . import api, synth

B = 0.01        # coupler fraction per round trip
LOSS = 0.01     # linear loss per round trip
KL = 0.1        # kappa L of the medium
BB2 = 25.0      # beta b^2 of the CHYM (0 for the CIM)
DH_RANGE = (-0.5, 1.0)
_GRAPH_TAG = 4
_X0_TAG = 5


# ------------------------------------------------------------- figures
def figures(energies, egs, n_pumps, n_rep, n):
    """Figures of merit of one graph and machine; energies: the final Ising
    energy of every run [n_pumps * n_rep], pump-major."""
    e = np.asarray(energies, dtype=np.int64).reshape(n_pumps, n_rep)
    if (e < egs).any():
        raise ValueError("a run went below the ground-state energy")
    p = (e == egs).mean(axis=1)
    support = p > 0
    dev = (e - egs).astype(np.float64)
    return {
        "P": p.tolist(),
        "P_max": float(p.max()),
        "W": float(p[support].mean()) if support.any() else 0.0,
        "W_scan": float(p.mean()),
        "dE": float(dev.mean()),
        "dE_per_n": float(dev.mean() / n),
    }


def tts99(cost, p):
    """Time to 99 % success from the cost per attempt and the success
    probability per attempt: cost ln(0.01) / ln(1 - p); one attempt when
    p >= 0.99, infinite when p = 0."""
    if p <= 0.0:
        return math.inf
    if p >= 0.99:
        return cost
    return cost * math.log(0.01) / math.log1p(-p)


def _quantiles(v):
    """Median and quartiles (linear interpolation) of values that may be
    infinite; a quantile that involves an infinite value is None (JSON has
    no infinity)."""
    v = np.asarray(v, dtype=np.float64)
    if not v.size:
        return {"q25": None, "median": None, "q75": None}
    big = 1e300
    q = np.percentile(np.where(np.isfinite(v), v, big), [25, 50, 75])
    cvt = lambda z: None if z >= 1e299 else float(z)  # noqa: E731
    return {"q25": cvt(q[0]), "median": cvt(q[1]), "q75": cvt(q[2])}


def success_report(energies, egs, n_pumps, n_rep, n, t_run_ms=None):
    """Success statistics of a workload of many instances (statistics
    paragraph: P_Ising over the pump scan and the deviation of the final
    energy, here per instance): energies[i] holds the final Ising energies
    of instance i's runs, pump-major (n_pumps x n_rep), egs[i] its
    ground-state energy.  Returns the success probability per pump averaged
    over the instances, and over the instances the quartiles of the
    best-pump success P_max, of the mean deviation E - E_GS (raw and per
    spin), the fraction of instances with a success, and, with the GPU time
    per run t_run_ms, the quartiles of the best-pump TTS99 (infinite for an
    unsolved instance, reported as None)."""
    f = [figures(e, g, n_pumps, n_rep, n) for e, g in zip(energies, egs)]
    P = np.array([x["P"] for x in f], dtype=np.float64)
    pmax = P.max(axis=1)
    de = np.array([x["dE"] for x in f], dtype=np.float64)
    out = {"instances": len(f), "P_per_pump_mean": P.mean(axis=0).tolist(), "P_max": _quantiles(pmax),
           "solved_fraction": float((pmax > 0).mean()), "dE": _quantiles(de), "dE_per_n": _quantiles(de / n)}
    if t_run_ms is not None:
        out["t_run_ms"] = float(t_run_ms)
        out["tts99_ms"] = _quantiles([tts99(t_run_ms, p) for p in pmax])
    return out


def histogram(energies, egs):
    """H_E as {E - E_GS: fraction of the runs}."""
    d, c = np.unique(np.asarray(energies, dtype=np.int64) - egs, return_counts=True)
    return {int(k): float(v) / float(c.sum()) for k, v in zip(d, c)}


def summary(values):
    v = np.asarray(values, dtype=np.float64)
    return {"mean": float(v.mean()), "q25": float(np.percentile(v, 25)), "q75": float(np.percentile(v, 75))}


def fit_exponential(ns, values):
    """Least-squares fit of log(values) = log(b) - a N over the positive
    values: (a, b), or (nan, nan) with fewer than two of them."""
    ns = np.asarray(ns, dtype=np.float64)
    v = np.asarray(values, dtype=np.float64)
    ok = v > 0
    if ok.sum() < 2:
        return math.nan, math.nan
    slope, icpt = np.polyfit(ns[ok], np.log(v[ok]), 1)
    return float(-slope), float(math.exp(icpt))


def ground_state_exhaustive(J):
    """Exact minimum of -sum_pq J_pq s_p s_q over s in {+-1}^n (s_0 = +1 by
    the global flip symmetry), enumerated in chunks."""
    J = np.asarray(J, dtype=np.float64)
    n = J.shape[0]
    if n == 1:
        return int(round(-J[0, 0]))
    best = math.inf
    m = n - 1
    chunk = 1 << min(m, 16)
    bits = np.arange(m, dtype=np.int64)
    for start in range(0, 1 << m, chunk):
        idx = np.arange(start, min(start + chunk, 1 << m), dtype=np.int64)
        s = np.ones((idx.size, n))
        s[:, 1:] = 1.0 - 2.0 * ((idx[:, None] >> bits[None, :]) & 1)
        e = -np.einsum("ip,pq,iq->i", s, J, s, optimize=True)
        best = min(best, float(e.min()))
    return int(round(best))


# ---------------------------------------------------------------- inputs
def graph(n, g, seed):
    return synth.er_pm1(n, seed, _GRAPH_TAG, n, g)


def pumps(d):
    """delta h grid: N_s = 51 (D = 1) or 21 (D = 2) values."""
    return np.linspace(DH_RANGE[0], DH_RANGE[1], 51 if d == 1 else 21)


def h_threshold():
    return -math.log((1.0 - B) * (1.0 - LOSS)) / KL


def machine_inputs(J, d, dh, n_rep, steps, seed, g):
    """Inputs of one graph's runs (replica k * n_rep + i: pump dh[k], initial
    state i): coupling magnitude, pumps h [R], amplitudes A0 [n, R, d],
    annealing table [steps, d] and beta b^2."""
    n = J.shape[0]
    eps = 0.5 / synth.lambda_max(J)
    jmag = float(np.float32(eps * (B + LOSS) / B))
    h = synth.pump_grid(n_rep, h_threshold() * (1.0 + np.asarray(dh)))
    A0 = synth.initial_states(n, h.size, d, seed, _X0_TAG, n, g, d, sigma=0.1 * math.sqrt((B + LOSS) / BB2))
    alpha = synth.anneal_schedule(steps, d)[0] if d > 1 else synth.constant_schedule(steps, d)
    return jmag, h, A0, alpha, (BB2 if d > 1 else 0.0)


# ------------------------------------------------------------ simulation
def machine_tasks(graphs, d, n_rep, steps, seed, precision="f32", device="cuda"):
    """chym_map_batch tasks of every graph's runs on one machine; each task
    also keeps its initial amplitudes as "A0"."""
    dev = torch.device(device)
    tasks = []
    for g, J in enumerate(graphs):
        jmag, h, A0, alpha, bb2 = machine_inputs(J, d, pumps(d), n_rep, steps, seed, g)
        A0d = torch.from_numpy(A0).to(dev)
        tasks.append(dict(J=torch.from_numpy(J).to(dev), h=torch.from_numpy(h).to(dev), A=A0d.clone(), A0=A0d,
                          alpha=torch.from_numpy(alpha).to(dev), b=B, loss=LOSS, kl=KL, beta_b2=bb2, jmag=jmag,
                          steps=steps, precision=precision))
    return tasks


def final_energies(tasks):
    """Sign readout and exact Ising energy of every task's final amplitudes."""
    out = []
    for t in tasks:
        n, r, _ = t["A"].shape
        spins = torch.empty((r, api.spin_words(n)), dtype=torch.int64, device=t["A"].device)
        e = torch.empty(r, dtype=torch.int32, device=t["A"].device)
        api.chym_readout(t["A"], spins)
        api.chym_ising_energy(t["J"], spins, e)
        out.append(e)
    torch.cuda.synchronize()
    return [e.cpu().numpy() for e in out]


def run_machine(graphs, d, n_rep, steps, seed, precision="f32", device="cuda"):
    """Final Ising energies [graph][pump * rep] of all runs of one machine:
    one chym_map_batch call for every graph."""
    tasks = machine_tasks(graphs, d, n_rep, steps, seed, precision, device)
    ws = api.chym_map_batch(tasks)
    energies = final_energies(tasks)
    del ws
    return energies


def search_ground(graphs, n_rep=2000, steps=20000, seed=0, device="cuda"):
    """Best Ising energy of long annealed runs of the ODE form (D = 3, BF16,
    pumps r in [1, 2]) for every graph, one batched launch."""
    dev = torch.device(device)
    pr = torch.from_numpy(synth.pump_grid(n_rep // 10, np.linspace(1.0, 2.0, 10))).to(dev)
    al = torch.from_numpy(synth.anneal_schedule(steps, 3)[0]).to(dev)
    tasks = []
    for g, J in enumerate(graphs):
        n = J.shape[0]
        x = synth.initial_states_torch(n, pr.shape[0], 3, seed=seed * 1000003 + 7919 * g + n, device=dev)
        tasks.append(dict(J=torch.from_numpy(J).to(dev), pump=pr, x=x, alpha=al,
                          eps=float(np.float32(synth.default_eps(J))), btil=1.0, eta=2e-4, dt=0.01, steps=steps,
                          precision="bf16",
                          spins=torch.empty((pr.shape[0], api.spin_words(n)), dtype=torch.int64, device=dev),
                          e_ising=torch.empty(pr.shape[0], dtype=torch.int32, device=dev)))
    plan = api.chym_batch_create(tasks)
    plan.launch()
    torch.cuda.synchronize()
    best = [int(t["e_ising"].min().item()) for t in tasks]
    plan.destroy()
    return best


def _print(msg):
    print(msg, flush=True)


def harness(ns=(10, 20, 30, 40, 50, 60, 70, 80, 90, 100), n_graphs=100, n_rep=100, steps=150000,
            search_rep=2000, search_steps=20000, exhaustive_max=22, precision="f32", seed=2308, device="cuda",
            example_n=None, log=_print):
    t0 = time.time()
    per_n, example, timing = [], None, []
    example_n = ns[-1] if example_n is None else example_n
    for n in ns:
        graphs = [graph(n, g, seed) for g in range(n_graphs)]
        t1 = time.time()
        e1 = run_machine(graphs, 1, n_rep, steps, seed, precision, device)
        t2 = time.time()
        e2 = run_machine(graphs, 2, n_rep, steps, seed, precision, device)
        t3 = time.time()
        if n <= exhaustive_max:
            egs = [ground_state_exhaustive(J) for J in graphs]
            how = "exhaustive"
        else:
            es = search_ground(graphs, search_rep, search_steps, seed, device) if search_rep else [0] * n_graphs
            egs = [min(int(a.min()), int(b.min()), c if search_rep else int(a.min())) for a, b, c in zip(e1, e2, es)]
            how = "best run"
        f1 = [figures(e, g, pumps(1).size, n_rep, n) for e, g in zip(e1, egs)]
        f2 = [figures(e, g, pumps(2).size, n_rep, n) for e, g in zip(e2, egs)]
        row = {"n": n, "E_GS": how}
        for name, f in (("D1_cim", f1), ("D2_chym", f2)):
            row[name] = {k: summary([x[k] for x in f]) for k in ("P_max", "W", "W_scan", "dE", "dE_per_n")}
        per_n.append(row)
        updates = steps * n * n_rep * n_graphs * (pumps(1).size * 1 + pumps(2).size * 2)
        timing.append({"n": n, "map_seconds_d1": t2 - t1, "map_seconds_d2": t3 - t2,
                       "updates_per_s": updates / max(t3 - t1, 1e-9)})
        if n == example_n:
            example = {"n": n, "graph": 0, "E_GS": egs[0], "delta_h_d1": pumps(1).tolist(), "P_d1": f1[0]["P"],
                       "H_E_d1": histogram(e1[0], egs[0]), "delta_h_d2": pumps(2).tolist(), "P_d2": f2[0]["P"],
                       "H_E_d2": histogram(e2[0], egs[0])}
        if log:
            r1, r2 = row["D1_cim"], row["D2_chym"]
            log(f"N={n}: P_max {r1['P_max']['mean']:.3f} / {r2['P_max']['mean']:.3f}, W {r1['W']['mean']:.3f} / "
                f"{r2['W']['mean']:.3f}, dE {r1['dE']['mean']:.2f} / {r2['dE']['mean']:.2f} (D=1 / D=2); "
                f"map {t3 - t1:.1f} s")
    fits = {}
    for name in ("D1_cim", "D2_chym"):
        a, b = fit_exponential([r["n"] for r in per_n], [r[name]["P_max"]["mean"] for r in per_n])
        fits[name] = {"a": a, "b": b}
    a2 = fits["D2_chym"]["a"]
    ratio = fits["D1_cim"]["a"] / a2 if a2 and not math.isnan(a2) else math.nan
    return {"workload": f"Erdos-Renyi 20% +-1 graphs, N in {list(ns)}, {n_graphs} graphs per N, {n_rep} runs per "
                        f"pump, delta h in {list(DH_RANGE)} at 51 (D=1 CIM) / 21 (D=2 CHYM, annealed) values, "
                        f"{steps} round trips of the map, {precision} form",
            "per_n": per_n, "fits": fits, "a1_over_a2": ratio, "example": example, "timing": timing,
            "seconds": time.time() - t0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--ns", type=str, default="10,20,30,40,50,60,70,80,90,100")
    ap.add_argument("--graphs", type=int, default=100)
    ap.add_argument("--rep", type=int, default=100)
    ap.add_argument("--steps", type=int, default=150000)
    ap.add_argument("--search-rep", type=int, default=2000)
    ap.add_argument("--out", type=str, default="")
    a = ap.parse_args()
    rep = harness(tuple(int(v) for v in a.ns.split(",")), a.graphs, a.rep, a.steps, search_rep=a.search_rep)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rep, f)
    print(json.dumps({k: v for k, v in rep.items() if k != "example"}))


if __name__ == "__main__":
    main()
