#!/usr/bin/env python3
"""Throughput benchmark of the CHYM hot path on one MI355X.

Workload (default): 1000 Sherrington-Kirkpatrick +-1 instances with N = 100
hyperspins, each run at D = 2 and at D = 3, 100 initial states x 20 pump
values (r in [0.5, 2.0]) = 2000 replicas per (instance, D), 5000 Euler steps
of dt = 0.01 with the linear dimensional anneal, float32 form; then sign
readout, exact Ising energy and float64 hyperspin energy of every run.

One bench step = the whole workload: reset the state to the initial
condition (one device copy), integrate all 2000 (instance, D) tasks with the
persistent batched kernels, score every run.  All inputs are resident in
HBM before the timed region.

Prints one JSON line (see the "metric" field); the roofline figures are for
the dominant kernel, the persistent integrator of the D = 3 tasks, timed
with HIP events on the stream it runs on.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin-comp updates/s; TTS99 to Ising GS: plain FP32 vs BF16+learned stop"
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense bf16 matrix peak (TFLOP/s)
PEAK_FP32_MATRIX_TFLOPS = 157.3
# float32 vector peak without packed float32 instructions (the library is
# built without them): 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz.
PEAK_FP32_VECTOR_UNPACKED_TFLOPS = 78.6


# HBM bytes per launch of the dominant kernel on the default workload, from
# rocprofv3 FETCH_SIZE / WRITE_SIZE passes scaled by the same counters on the
# bench's own 4 GB state copy (profiles/integrate_persistent_sk100_d23_f32.md);
# keyed by kernel and workload, valid for the kernels as they are now.
TRAFFIC_SOURCE = ("profiles/integrate_persistent_sk100_d23_f32.md: rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE "
                  "of this kernel on this workload, scaled by the same counters on a copy of known size; "
                  "not measured in this run")
TRAFFIC = {("k_integrate_persistent_lds<7, 3, 3, 1, 2>", 100, 1000, 2000): 9.70e9}
# The same for the precision workload's +-1 launch (bf16 form, N = 1000, D = 4,
# 4096 replicas, 10 000 steps), scaled by its own 65.5 MB state copies.
PRECISION_TRAFFIC = 1.512e8
PRECISION_TRAFFIC_SOURCE = ("profiles/hbm_traffic_slab_n1000_d4.md: rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE of "
                            "this kernel on this workload, scaled by the same counters on a copy of known size; "
                            "not measured in this run")


def kernel_name(tiles, d, precision, plan):
    xs = 3 if precision == "f32" else 1
    kind = plan.get("kernel")
    if kind == 2:
        return f"k_integrate_persistent_lds<{tiles}, {d}, {xs}, 1, 2>"
    if kind == 3:
        return f"k_integrate_persistent_lds<{tiles}, {d}, {xs}, 1, 1>"
    return f"k_integrate_persistent<{tiles}, {d}, {xs}, 1, false>"  # false: the continuous-limit form


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--instances", type=int, default=1000)
    ap.add_argument("--n", type=int, default=100)
    ap.add_argument("--dims", type=str, default="2,3")
    ap.add_argument("--ics", type=int, default=100)
    ap.add_argument("--pumps", type=int, default=20)
    ap.add_argument("--euler-steps", type=int, default=5000)
    ap.add_argument("--dt", type=float, default=0.01)
    ap.add_argument("--precision", type=str, default="f32", choices=["f32", "bf16"])
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--autotune", type=int, default=1, help="time the launch plans of each variant first")
    ap.add_argument("--plan-cache", type=str, default="", help="load plans from this file instead of tuning")
    ap.add_argument("--save-plans", type=str, default="", help="write the plans used to this file")
    ap.add_argument("--cpu-baseline", type=int, default=1, help="0 disables the oracle timing leg")
    ap.add_argument("--cpu-replicas", type=int, default=2000)
    ap.add_argument("--tts", type=int, default=1, help="0 skips the time-to-99%%-ground-state comparison")
    ap.add_argument("--success", type=int, default=1,
                    help="0 skips the success statistics of the default workload (untimed: a batched search for "
                         "each instance's putative ground state, then P_Ising per pump, E - E_GS and TTS99)")
    ap.add_argument("--success-out", type=str, default="",
                    help="write the per-instance success tables of the default workload to this .npz file")
    ap.add_argument("--workload", type=str, default="sk100",
                    choices=["sk100", "precision", "batched", "map", "sparse", "stats", "xy"],
                    help="sk100: the default throughput workload; precision: N=1000, D=4, 4096 replicas, "
                         "10000 steps with +-1, bf16 Gaussian and FP8 Gaussian couplings; batched: 10000 "
                         "solves of mixed N, D and graph family in one graph launch; map: the round-trip "
                         "map of Eq. (2) at the paper's parameters, N=100, D=3, 65536 replicas; sparse: "
                         "3-regular and 20%% Erdos-Renyi couplings in sparse rows against the dense path; "
                         "stats: the statistical harness's launches at N=100 (100 graphs, CIM and annealed "
                         "CHYM, batched map); xy: the XY-machine mode (D=2, no annealing, kappa L=1e-3) on 100 "
                         "graphs at N=100 with hyperspin energies")
    ap.add_argument("--round-trips", type=int, default=15000, help="stats workload: round trips per run")
    ap.add_argument("--dense-3reg", action="store_true",
                    help="batched workload: store the 3-regular couplings dense (matrix-core path)")
    return ap.parse_args()


def build_workload(args, torch, synth, api, dev):
    dims = [int(v) for v in args.dims.split(",")]
    n, steps = args.n, args.euler_steps
    R = args.ics * args.pumps
    pumps = synth.pump_grid(args.ics, np.linspace(0.5, 2.0, args.pumps))
    pump_d = torch.from_numpy(pumps).to(dev)
    Js = np.stack([synth.sk_pm1(n, 1, i) for i in range(args.instances)])
    lam = np.linalg.eigvalsh(Js.astype(np.float64))[:, -1]
    eps = (0.5 / lam).astype(np.float32)
    J_d = torch.from_numpy(Js).to(dev)
    alphas = {d: torch.from_numpy(synth.anneal_schedule(steps, d)[0]).to(dev) for d in dims}
    # one contiguous buffer for all states, and a pristine copy of the initial states
    sizes = [n * R * d for d in dims]
    per_inst = sum(sizes)
    x0 = synth.initial_states_torch(args.instances * per_inst, 1, 1, seed=2308023290 + 1, device=dev).view(-1)
    x = torch.empty_like(x0)
    w = api.spin_words(n)
    plans = {}
    outs = []
    score_tasks = []
    for di, d in enumerate(dims):
        tasks = []
        for i in range(args.instances):
            off = i * per_inst + sum(sizes[:di])
            xv = x[off:off + sizes[di]].view(n, R, d)
            t = dict(J=J_d[i], pump=pump_d, x=xv, alpha=alphas[d], eps=float(eps[i]), btil=1.0, eta=2e-4,
                     dt=args.dt, steps=steps, precision=args.precision)
            tasks.append(t)
            o = dict(spins=torch.empty((R, w), dtype=torch.int64, device=dev),
                     e_ising=torch.empty(R, dtype=torch.int32, device=dev),
                     e_hs=torch.empty(R, dtype=torch.float64, device=dev),
                     diverged=torch.empty(R, dtype=torch.uint8, device=dev))
            outs.append((i, d, o))
            st = dict(t)
            st["steps"] = 0
            st.update(o)
            score_tasks.append(st)
        plans[d] = api.chym_batch_create(tasks)
    score_plan = api.chym_batch_create(score_tasks)
    updates = sum(args.instances * n * R * d * steps for d in dims)
    return dict(dims=dims, plans=plans, score_plan=score_plan, x=x, x0=x0, outs=outs, updates=updates, R=R,
                Js=Js, eps=eps, pumps=pumps)


def cpu_baseline(args, synth, wl):
    """The FP64 oracle on a bounded sample of the same workload."""
    import oracle

    n, steps = args.n, args.euler_steps
    rs = min(args.cpu_replicas, wl["R"])
    J = wl["Js"][0]
    x0 = synth.initial_states(n, rs, 3, 1, 0)
    t0 = time.perf_counter()
    ups = 0
    for d in wl["dims"]:
        al, _ = synth.anneal_schedule(steps, d)
        oracle.ode_run(J, wl["pumps"][:rs], x0[:, :, :d], float(wl["eps"][0]), 1.0, 2e-4, args.dt, steps, al)
        ups += n * rs * d * steps
    sec = time.perf_counter() - t0
    return {"value": ups / sec, "unit": "spin-component updates/s", "cores": oracle.max_threads(),
            "cpu_model": host_cpu_model(), "kind": "oracle",
            "sample": f"instance 0, D in {wl['dims']}, replicas 0..{rs - 1} of {wl['R']}, {steps} steps, "
                      f"{ups:.3e} updates in {sec:.2f} s"}


def success_leg(args, wl, kern_ms):
    """Success statistics of the default workload's last step (untimed):
    the putative ground state of every instance is the best energy of its
    4000 benchmarked runs and of 2000 longer annealed runs (BF16 form,
    20 000 steps, pumps 1..2, one batched launch); then, per D, P_Ising per
    pump, E - E_GS per instance and the best-pump TTS99 at the measured GPU
    time per run (stats.success_report)."""
    import torch

    from paper_2308_02329_amd import stats

    t0 = time.perf_counter()
    n, R, inst = args.n, wl["R"], args.instances
    energies = {d: [None] * inst for d in wl["dims"]}
    for i, d, o in wl["outs"]:
        energies[d][i] = o["e_ising"].cpu().numpy()
    search = stats.search_ground([wl["Js"][i] for i in range(inst)], n_rep=2000, steps=20000, seed=2308023292)
    egs = [min([search[i]] + [int(energies[d][i].min()) for d in wl["dims"]]) for i in range(inst)]
    torch.cuda.synchronize()
    out = {"egs_source": "best of the benchmarked runs and 2000 BF16 runs x 20000 steps per instance",
           "egs_from_search": int(sum(search[i] == egs[i] for i in range(inst))),
           "pumps": np.linspace(0.5, 2.0, args.pumps).tolist()}
    for d in wl["dims"]:
        t_run = kern_ms[d] / args.steps / (inst * R)
        out[str(d)] = stats.success_report(energies[d], egs, args.pumps, args.ics, n, t_run_ms=t_run)
    if args.success_out:
        tab = {f"P_d{d}": np.array([stats.figures(e, g, args.pumps, args.ics, n)["P"]
                                    for e, g in zip(energies[d], egs)]) for d in wl["dims"]}
        tab.update({f"dE_d{d}": np.array([(e.astype(np.int64) - g).mean() for e, g in zip(energies[d], egs)])
                    for d in wl["dims"]})
        np.savez_compressed(args.success_out, egs=np.array(egs), **tab)
    out["seconds"] = time.perf_counter() - t0
    return out


def host_cpu_model() -> str:
    """Model name of the host CPU (first entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def tts_leg():
    """Time to 99 % ground-state success of the learned-restart workload
    (SK N = 200, D = 3): plain FP32, BF16 and BF16 with the learned restart,
    each executed and timed end to end on held-out instances (untimed by the
    bench clock)."""
    from paper_2308_02329_amd import learned

    rep = learned.experiment(log=None)
    keep = ("workload", "tts99_median_ms", "instances_solved", "same_instances_solved", "learned_over_bf16_geomean",
            "learned_over_bf16_ci95", "learned_over_f32_geomean", "learned_over_f32_ci95", "keep_fraction",
            "chosen_epoch", "auc_within_batch_val", "auc_within_batch_heldout", "trajectories_train",
            "positives_train", "ms_per_attempt", "kept_runs_match_plain", "seconds")
    def finite(v):
        if isinstance(v, dict):
            return {k: finite(x) for k, x in v.items()}
        return None if isinstance(v, float) and not np.isfinite(v) else v

    out = {k: finite(rep[k]) for k in keep}
    out["unit"] = "ms (median over instances of the best-pump TTS99)"
    return out


def lambda_max_power(J, iters=200):
    """Largest eigenvalue of a symmetric matrix by power iteration on the
    shifted matrix J + s I (host, float64); sets the run input eps only."""
    J = J.astype(np.float64)
    s = np.abs(J).sum(axis=1).max()  # Gershgorin: J + s I is positive semidefinite
    v = np.random.default_rng(0).standard_normal(J.shape[0])
    lam = 0.0
    for _ in range(iters):
        w = J @ v + s * v
        lam = float(np.linalg.norm(w))
        v = w / lam
    return lam - s


def timed_events(torch, stream, fn, reps):
    """Runs fn reps times between HIP events on stream; returns ms per call."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def run_precision(args, torch, api, synth):
    """N = 1000, D = 4, 16 pumps x 256 initial states = 4096 replicas, 10000
    steps, BF16 form, three couplings: SK +-1 (int8, exact), Gaussian rounded
    to bf16, Gaussian in FP8 (E4M3 + E8M0 row exponents).  The float32 form of
    the SK problem (component passes at this size) is timed beside it and
    reported apart from the line's value."""
    dev = torch.device("cuda:0")
    n, d, steps = 1000, 4, args.euler_steps if args.euler_steps != 5000 else 10000
    R = 4096
    pumps = torch.from_numpy(synth.pump_grid(256, np.linspace(0.5, 2.0, 16))).to(dev)
    alpha = torch.from_numpy(synth.anneal_schedule(steps, d)[0]).to(dev)
    sk = synth.sk_pm1(n, 3, 0)
    ga = synth.gaussian_j(n, 3, 1).astype(np.float32)
    Js = {"sk_pm1_int8": torch.from_numpy(sk).to(dev),
          "gauss_bf16": torch.from_numpy(ga).to(dev).to(torch.bfloat16),
          "gauss_fp8": api.chym_quantize_fp8(torch.from_numpy(ga).to(dev))}
    eps = {"sk_pm1_int8": 0.5 / lambda_max_power(sk), "gauss_bf16": 0.5 / lambda_max_power(ga)}
    eps["gauss_fp8"] = eps["gauss_bf16"]
    x0 = synth.initial_states_torch(n, R, d, seed=2308023293, device=dev)
    x = torch.empty_like(x0)
    nb = max(api.chym_integrate_workspace_size(Js["sk_pm1_int8"], x, precision=p) for p in ("bf16", "f32"))
    ws = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    res_kind = {}

    def run(kind):
        api.chym_integrate(Js[kind], pumps, x, alpha, eps=float(eps[kind]), btil=1.0, eta=2e-4, dt=args.dt,
                           steps=steps, precision="bf16", workspace=ws)

    for kind in Js:
        x.copy_(x0)
        run(kind)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for kind in Js:
            x.copy_(x0)
            res_kind[kind] = res_kind.get(kind, 0.0) + timed_events(torch, stream, lambda: run(kind), 1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    res_kind = {k: v / args.steps for k, v in res_kind.items()}
    upd = n * R * d * steps * len(Js)
    ms_sk = res_kind["sk_pm1_int8"]
    flops = n * R * d * steps * 2.0 * (n - 1)
    achieved = flops / (ms_sk / 1e3) / 1e12

    def run_f32():
        api.chym_integrate(Js["sk_pm1_int8"], pumps, x, alpha, eps=float(eps["sk_pm1_int8"]), btil=1.0, eta=2e-4,
                           dt=args.dt, steps=steps, precision="f32", workspace=ws)

    x.copy_(x0)
    run_f32()
    x.copy_(x0)
    ms_f32 = timed_events(torch, stream, run_f32, 1)
    return {"metric": METRIC, "value": upd / (wall / args.steps), "unit": "spin-component updates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 1, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
            "config": {"workload": f"N={n} D={d}, 16 pumps x 256 initial states = {R} replicas, {steps} Euler steps, "
                                   f"bf16 form; couplings SK +-1 int8, Gaussian bf16, Gaussian FP8 E4M3+E8M0",
                       "n": n, "d": d, "replicas": R, "euler_steps": steps, "precision": "bf16"},
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / PEAK_BF16_TFLOPS, "traffic": PRECISION_TRAFFIC,
                         "traffic_source": PRECISION_TRAFFIC_SOURCE,
                         "kernel": "k_integrate_slab<4, 1, 1, 8, 8> (SK +-1 J, bf16 fragments)", "kernel_ms": ms_sk},
            "integrate_ms": res_kind,
            "float32_form": {"couplings": "SK +-1 int8", "kernel": "k_integrate_slab<4, 3, 1, 8, 8, true> "
                                                                   "(component passes)",
                             "integrate_ms": ms_f32,
                             "frac_bf16_peak": flops / (ms_f32 / 1e3) / 1e12 / PEAK_BF16_TFLOPS}}


def run_batched(args, torch, api, synth):
    """10000 solves in one graph launch: N uniform in {50, 100, 200, 400,
    800}, D uniform in {2, 3, 4}, SK +-1 or 3-regular +-1 (half each), one
    pump r ~ U[0.5, 2] per solve, 32 initial states, 5000 steps, BF16 form,
    plans autotuned per resident (N, D) bucket.  The 3-regular couplings are
    stored as sparse rows (the gather integrator) unless --dense-3reg."""
    dev = torch.device("cuda:0")
    g = np.random.default_rng(2308023294)
    n_solves, reps, steps = args.instances if args.instances != 1000 else 10000, 32, args.euler_steps
    Ns = g.choice([50, 100, 200, 400, 800], n_solves)
    Ds = g.choice([2, 3, 4], n_solves)
    fam = g.random(n_solves) < 0.5
    hs = g.uniform(0.5, 2.0, n_solves).astype(np.float32)
    tuned = {}
    for nn in (50, 100, 200, 400, 800):
        for dd in (2, 3, 4):
            try:
                tuned[f"{nn}/{dd}"] = api.chym_plan_autotune(int(nn), int(dd), "bf16", torch.int8, steps=200)[0]
            except api.ChymError:
                tuned[f"{nn}/{dd}"] = "streamed-J (no plan)"
    jsz = [int(nn) * int(nn) for nn in Ns]
    xsz = [int(nn) * reps * int(dd) for nn, dd in zip(Ns, Ds)]
    Jh = np.empty(sum(jsz), dtype=np.int8)
    eps = np.empty(n_solves)
    off = 0
    flops = 0.0
    dense_flops = 0.0  # every coupling matrix counted dense: 2 (N - 1) per update
    for i in range(n_solves):
        nn = int(Ns[i])
        J = synth.regular3_pm1(nn, 4, i) if fam[i] else synth.sk_pm1(nn, 4, i)
        Jh[off:off + nn * nn] = J.ravel()
        eps[i] = 0.5 / lambda_max_power(J, 100)
        off += nn * nn
        flops += nn * reps * int(Ds[i]) * steps * (6.0 if fam[i] else 2.0 * (nn - 1))
        dense_flops += nn * reps * int(Ds[i]) * steps * 2.0 * (nn - 1)
    Jd = torch.from_numpy(Jh).to(dev)
    sparse = fam & (not args.dense_3reg)
    x0 = synth.initial_states_torch(sum(xsz), 1, 1, seed=2308023294, device=dev).view(-1)
    x = torch.empty_like(x0)
    alphas = {dd: torch.from_numpy(synth.anneal_schedule(steps, dd)[0]).to(dev) for dd in (2, 3, 4)}
    pump_all = torch.from_numpy(np.repeat(hs, reps)).to(dev)
    tasks = []
    joff = xoff = 0
    for i in range(n_solves):
        nn, dd = int(Ns[i]), int(Ds[i])
        Ji = Jd[joff:joff + nn * nn].view(nn, nn)
        t = dict(J=Ji, pump=pump_all[i * reps:(i + 1) * reps], x=x[xoff:xoff + nn * reps * dd].view(nn, reps, dd),
                 alpha=alphas[dd], eps=float(eps[i]), btil=1.0, eta=2e-4, dt=args.dt, steps=steps, precision="bf16",
                 spins=torch.empty((reps, api.spin_words(nn)), dtype=torch.int64, device=dev))
        if sparse[i]:
            t["J"] = torch.from_numpy(api.ell_pack(Jh[joff:joff + nn * nn].reshape(nn, nn))).to(dev)
            t["e_ising_f64"] = torch.empty(reps, dtype=torch.float64, device=dev)
        else:
            t["e_ising"] = torch.empty(reps, dtype=torch.int32, device=dev)
        tasks.append(t)
        joff += nn * nn
        xoff += nn * reps * dd
    t_setup = time.perf_counter()
    plan = api.chym_batch_create(tasks)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    stream = torch.cuda.current_stream()

    def one():
        x.copy_(x0)
        plan.launch()

    one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = 0.0
    for _ in range(args.steps):
        ms += timed_events(torch, stream, one, 1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    upd = float(sum(int(nn) * reps * int(dd) * steps for nn, dd in zip(Ns, Ds)))
    achieved = flops / (ms / args.steps / 1e3) / 1e12
    plan.destroy()
    return {"metric": METRIC, "value": upd / (wall / args.steps), "unit": "spin-component updates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 1, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
            "config": {"workload": f"{n_solves} solves in one graph launch: N in {{50,100,200,400,800}}, D in {{2,3,4}}, "
                                   f"SK or 3-regular +-1 (3-regular in "
                                   f"{'dense' if args.dense_3reg else 'sparse'} rows), one pump per solve, {reps} "
                                   f"initial states, {steps} steps, bf16 form", "solves": n_solves,
                       "replicas_per_solve": reps,
                       "euler_steps": steps, "precision": "bf16"},
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / PEAK_BF16_TFLOPS, "traffic": None,
                         "kernel": "whole batch launch (algorithmic flops: 2(N-1) per SK update, 6 per 3-regular)",
                         "kernel_ms": ms / args.steps},
            "dense_equivalent": {"achieved": dense_flops / (ms / args.steps / 1e3) / 1e12, "unit": "TFLOP/s",
                                 "frac": dense_flops / (ms / args.steps / 1e3) / 1e12 / PEAK_BF16_TFLOPS},
            "setup_s": t_setup, "plans": tuned}


def run_map(args, torch, api, synth):
    """The literal round-trip map: N = 100 SK, D = 3, 65536 replicas (pumps
    1.1 .. 2 h_th), kappa L = 0.1, beta b^2 = 25, b = d = 0.01, 2000 round
    trips with the anneal, float32 form."""
    import math

    dev = torch.device("cuda:0")
    n, d, R, steps = 100, 3, 65536, 2000
    b = dd = 0.01
    kl, bb2 = 0.1, 25.0
    J = synth.sk_pm1(n, 6, 0)
    jmag = 0.5 / lambda_max_power(J) * (b + dd) / b
    hth = -math.log((1 - b) * (1 - dd)) / kl
    h = torch.from_numpy((np.linspace(1.1, 2.0, R) * hth).astype(np.float32)).to(dev)
    A0 = synth.initial_states_torch(n, R, d, seed=2308023295, device=dev) * (100.0 * math.sqrt((b + dd) / bb2))
    A = torch.empty_like(A0)
    alpha = torch.from_numpy(synth.anneal_schedule(steps, d)[0]).to(dev)
    Jd = torch.from_numpy(J).to(dev)
    stream = torch.cuda.current_stream()

    def run():
        api.chym_map_integrate(Jd, h, A, alpha, b=b, loss=dd, kl=kl, beta_b2=bb2, jmag=jmag, steps=steps)

    A.copy_(A0)
    run()
    torch.cuda.synchronize()
    ms = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        A.copy_(A0)
        ms += timed_events(torch, stream, run, 1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    upd = n * R * d * steps
    kms = ms / args.steps
    achieved = upd * 2.0 * (n - 1) / (kms / 1e3) / 1e12
    return {"metric": METRIC, "value": upd / (wall / args.steps), "unit": "spin-component updates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 1, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"round-trip map of Eq. (2): SK +-1 N={n}, D={d}, {R} replicas, {steps} round "
                                   f"trips, kappa L={kl}, beta b^2={bb2}, b=d={b}, linear anneal, f32 form",
                       "n": n, "d": d, "replicas": R, "round_trips": steps, "precision": "f32"},
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / PEAK_BF16_TFLOPS, "traffic": None,
                         "kernel": "k_integrate_resident<7, 3, 3, 1, true>", "kernel_ms": kms}}


def run_sparse(args, torch, api, synth):
    """Sparse-row couplings against the dense matrix-core path on the same
    problems: 3-regular +-1 graphs (N = 200, 400, 800) and a 20% Erdos-Renyi
    +-1 graph (N = 100, the paper's family), D = 3, 4096 replicas, 2000 steps
    with the anneal; the sparse path in float32, the dense one in bf16."""
    dev = torch.device("cuda:0")
    d, R, steps = 3, 4096, 2000
    stream = torch.cuda.current_stream()
    pumps = torch.from_numpy(synth.pump_grid(256, np.linspace(0.5, 2.0, 16))).to(dev)
    alpha = torch.from_numpy(synth.anneal_schedule(steps, d)[0]).to(dev)
    rows = []
    tot_upd, tot_ms = 0.0, 0.0
    for kind, n in (("reg3", 200), ("reg3", 400), ("reg3", 800), ("er20", 100)):
        J = synth.regular3_pm1(n, 7, n) if kind == "reg3" else synth.er_pm1(n, 7, n)
        eps = 0.5 / lambda_max_power(J)
        x0 = synth.initial_states_torch(n, R, d, seed=2308023296 + n, device=dev)
        x = torch.empty_like(x0)
        kw = dict(eps=float(eps), btil=1.0, eta=2e-4, dt=args.dt, steps=steps)
        Je = torch.from_numpy(api.ell_pack(J)).to(dev)
        Jd = torch.from_numpy(J).to(dev)
        ws = None
        nb = api.chym_integrate_workspace_size(Jd, x, precision="bf16")
        if nb:
            ws = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        res = {}
        for name, Jx, prec in (("sparse_f32", Je, "f32"), ("dense_bf16", Jd, "bf16")):
            def run():
                api.chym_integrate(Jx, pumps, x, alpha, precision=prec, workspace=ws, **kw)
            x.copy_(x0)
            run()
            ms = 0.0
            for _ in range(args.steps):
                x.copy_(x0)
                ms += timed_events(torch, stream, run, 1)
            res[name] = ms / args.steps
        upd = n * R * d * steps
        nnz = int((J != 0).sum())
        rows.append({"graph": kind, "n": n, "row_width": int(Je.shape[1] // 2), "nonzeros_per_row": nnz / n,
                     "ms": res, "updates_per_s": {k: upd / (v / 1e3) for k, v in res.items()},
                     "speedup_sparse_over_dense": res["dense_bf16"] / res["sparse_f32"]})
        tot_upd += upd
        tot_ms += res["sparse_f32"]
    # roofline of the sparse gather: algorithmic flops 2 nnz/n per update
    r0 = rows[2]
    achieved = r0["updates_per_s"]["sparse_f32"] * 2.0 * r0["nonzeros_per_row"] / 1e12
    return {"metric": METRIC, "value": tot_upd / (tot_ms / 1e3), "unit": "spin-component updates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 1, "ms_per_step": tot_ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"sparse rows: 3-regular +-1 N in (200, 400, 800) and 20% Erdos-Renyi +-1 N=100, "
                                   f"D={d}, {R} replicas, {steps} Euler steps with the anneal, float32 gather",
                       "d": d, "replicas": R, "euler_steps": steps},
            "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_UNPACKED_TFLOPS,
                         "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR_UNPACKED_TFLOPS, "traffic": None,
                         "peak_note": "float32 vector ALU without packed float32 (not used by the library)",
                         "kernel": "k_integrate_ell<3> (3-regular N=800)", "kernel_ms": r0["ms"]["sparse_f32"]},
            "graphs": rows}


def run_stats(args, torch, api, synth):
    """The statistical harness at its largest size: 100 Erdos-Renyi 20% +-1
    graphs at N = 100, each run as the CIM (D = 1, 51 pumps x 100 runs) and
    as the annealed CHYM (D = 2, 21 pumps x 100 runs) with the round-trip
    map, float32 form.  One step = both chym_map_batch calls plus the
    readout and exact Ising energy of every run."""
    from paper_2308_02329_amd import stats

    n, n_graphs, n_rep, steps = 100, 100, 100, args.round_trips
    graphs = [stats.graph(n, g, 2308) for g in range(n_graphs)]
    machines = {d: stats.machine_tasks(graphs, d, n_rep, steps, 2308) for d in (1, 2)}
    stream = torch.cuda.current_stream()
    kms = {1: 0.0, 2: 0.0}
    keep = []

    def step(timed):
        for d, tasks in machines.items():
            for t in tasks:
                t["A"].copy_(t["A0"])
            if timed:
                kms[d] += timed_events(torch, stream, lambda: keep.append(api.chym_map_batch(tasks)), 1)
            else:
                keep.append(api.chym_map_batch(tasks))
            for t in tasks:
                r = t["A"].shape[1]
                if "spins" not in t:
                    t["spins"] = torch.empty((r, api.spin_words(n)), dtype=torch.int64, device="cuda")
                    t["e"] = torch.empty(r, dtype=torch.int32, device="cuda")
                api.chym_readout(t["A"], t["spins"])
                api.chym_ising_energy(t["J"], t["spins"], t["e"])

    step(False)
    torch.cuda.synchronize()
    keep.clear()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    upd = {d: n * d * sum(t["A"].shape[1] for t in machines[d]) * steps for d in (1, 2)}
    total = upd[1] + upd[2]
    ms1 = kms[1] / args.steps
    achieved = upd[1] * 2.0 * (n - 1) / (ms1 / 1e3) / 1e12
    return {"metric": METRIC, "value": total / wall, "unit": "spin-component updates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 1, "ms_per_step": wall * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"statistical harness at N={n}: {n_graphs} Erdos-Renyi 20% +-1 graphs, CIM "
                                   f"(D=1, 51 pumps x {n_rep} runs) and annealed CHYM (D=2, 21 x {n_rep}), {steps} "
                                   f"round trips of the map each, kappa L=0.1, beta b^2=25 (CHYM) / 0 (CIM), "
                                   f"b=d=0.01, f32 form, readout and exact energies",
                       "n": n, "graphs": n_graphs, "runs": {"d1": 51 * n_rep, "d2": 21 * n_rep},
                       "round_trips": steps, "precision": "f32"},
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / PEAK_BF16_TFLOPS, "traffic": None,
                         "kernel": "k_integrate_persistent<7, 1, 3, 1, true>", "kernel_ms": ms1},
            "map_batch_ms": {"d1": ms1, "d2": kms[2] / args.steps}}


def run_xy(args, torch, api, synth):
    """The XY-machine mode: 100 Erdos-Renyi 20% +-1 graphs at N = 100, D = 2,
    no annealing, kappa L = 1e-3, beta b^2 = 25, 4 pumps x 100 runs each,
    20000 round trips of the map, float32 form.  One step = one
    chym_map_batch call plus the hyperspin energy of every run."""
    from paper_2308_02329_amd import stats, xy

    n, n_graphs, n_rep, steps = 100, 100, 100, 20000
    dh = (0.1, 0.25, 0.5, 1.0)
    dev = torch.device("cuda:0")
    tasks = []
    for g in range(n_graphs):
        J = stats.graph(n, g, 2308)
        jmag, h, A0, alpha = xy.machine_inputs(J, n_rep, steps, dh, 2308, g)
        A0d = torch.from_numpy(A0).to(dev)
        tasks.append(dict(J=torch.from_numpy(J).to(dev), h=torch.from_numpy(h).to(dev), A=A0d.clone(), A0=A0d,
                          alpha=torch.from_numpy(alpha).to(dev), b=xy.B, loss=xy.LOSS, kl=xy.KL, beta_b2=xy.BB2,
                          jmag=jmag, steps=steps,
                          e=torch.empty(A0.shape[1], dtype=torch.float64, device=dev)))
    stream = torch.cuda.current_stream()
    keep = []
    kms = 0.0

    def step(timed):
        nonlocal kms
        for t in tasks:
            t["A"].copy_(t["A0"])
        if timed:
            kms += timed_events(torch, stream, lambda: keep.append(api.chym_map_batch(tasks)), 1)
        else:
            keep.append(api.chym_map_batch(tasks))
        for t in tasks:
            api.chym_hs_energy(t["J"], t["A"], t["e"])

    step(False)
    torch.cuda.synchronize()
    keep.clear()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    runs = n_graphs * len(dh) * n_rep
    upd = n * 2 * runs * steps
    ms = kms / args.steps
    achieved = upd * 2.0 * (n - 1) / (ms / 1e3) / 1e12
    return {"metric": METRIC, "value": upd / wall, "unit": "spin-component updates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 1, "ms_per_step": wall * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"XY machine: {n_graphs} Erdos-Renyi 20% +-1 graphs at N={n}, D=2, no annealing, "
                                   f"kappa L={xy.KL}, beta b^2={xy.BB2}, b=d={xy.B}, {len(dh)} pumps x {n_rep} runs, "
                                   f"{steps} round trips of the map, f32 form, hyperspin energies",
                       "n": n, "graphs": n_graphs, "runs": runs, "round_trips": steps, "precision": "f32"},
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / PEAK_BF16_TFLOPS, "traffic": None,
                         "kernel": "k_integrate_persistent<7, 2, 3, 1, true>", "kernel_ms": ms}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)
    import torch

    if args.workload != "sk100":
        from paper_2308_02329_amd import api, synth

        torch.cuda.set_device(0)
        fn = {"precision": run_precision, "batched": run_batched, "map": run_map,
              "sparse": run_sparse, "stats": run_stats, "xy": run_xy}[args.workload]
        print(json.dumps(fn(args, torch, api, synth), default=str), flush=True)
        return

    from paper_2308_02329_amd import api, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    plans = {}
    if args.plan_cache:
        api.chym_plan_load(args.plan_cache)
    elif args.autotune:
        for d in [int(v) for v in args.dims.split(",")]:
            best, cands = api.chym_plan_autotune(args.n, d, args.precision, torch.int8, steps=400)
            plans[str(d)] = {"chosen": best, "candidates": cands}
    if args.save_plans:
        api.chym_plan_save(args.save_plans)
    wl = build_workload(args, torch, synth, api, dev)
    stream = torch.cuda.current_stream()
    dims = wl["dims"]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(dims) + 2)]

    def one_step(record):
        wl["x"].copy_(wl["x0"])
        if record:
            ev[0].record(stream)
        for k, d in enumerate(dims):
            p = wl["plans"][d]
            p.launch_nograph() if args.no_graph else p.launch()
            if record:
                ev[k + 1].record(stream)
        wl["score_plan"].launch_nograph() if args.no_graph else wl["score_plan"].launch()
        if record:
            ev[-1].record(stream)

    for _ in range(args.warmup):
        one_step(False)
    torch.cuda.synchronize()
    kern_ms = {d: 0.0 for d in dims}
    score_ms = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step(True)
        torch.cuda.synchronize()
        for k, d in enumerate(dims):
            kern_ms[d] += ev[k].elapsed_time(ev[k + 1])
        score_ms += ev[len(dims)].elapsed_time(ev[-1])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    value = wl["updates"] / (wall / args.steps)

    # dominant kernel: persistent integrator of the largest D
    dk = max(dims)
    n, R = args.n, wl["R"]
    upd_k = args.instances * n * R * dk * args.euler_steps
    flops_k = upd_k * 2.0 * (n - 1)  # algorithmic: 2 (N-1) flops per update (dense J, zero diagonal)
    avg_s = kern_ms[dk] / args.steps / 1e3
    achieved = flops_k / avg_s / 1e12
    plan = api.chym_plan_get(args.n, dk, args.precision, torch.int8)
    kname = kernel_name((n + 15) // 16, dk, args.precision, plan)
    roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_BF16_TFLOPS, "traffic": TRAFFIC.get((kname, args.n, args.instances, R)),
            "traffic_source": TRAFFIC_SOURCE if (kname, args.n, args.instances, R) in TRAFFIC else None,
            "kernel": kname, "kernel_ms": kern_ms[dk] / args.steps}

    # run statistics of the last step (not timed)
    diverged = sum(int(o["diverged"].sum().item()) for _, _, o in wl["outs"])
    res = {"metric": METRIC, "value": value, "unit": "spin-component updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32" if args.precision == "f32" else "bf16",
           "data": "synthetic",
           "config": {"workload": f"{args.instances} SK +-1 instances N={n}, D in {dims}, "
                                  f"{args.ics} initial states x {args.pumps} pumps, {args.euler_steps} Euler steps "
                                  f"dt={args.dt}, linear dimensional anneal, {args.precision} form",
                      "instances": args.instances, "n": n, "dims": dims, "replicas": R,
                      "euler_steps": args.euler_steps, "precision": args.precision,
                      "graph": not args.no_graph},
           "roofline": roof,
           "integrate_ms_per_step": {str(d): kern_ms[d] / args.steps for d in dims},
           "score_ms_per_step": score_ms / args.steps,
           "diverged_runs": diverged,
           "plans": {str(d): api.chym_plan_get(args.n, d, args.precision, torch.int8) for d in dims},
           "autotune": plans}
    if args.success:
        res["success"] = success_leg(args, wl, kern_ms)
    if args.cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(args, synth, wl)
    if args.tts:
        res["tts99"] = tts_leg()
    for p in list(wl["plans"].values()) + [wl["score_plan"]]:
        p.destroy()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
