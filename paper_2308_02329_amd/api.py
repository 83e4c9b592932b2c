"""Python binding of libchym with the C ABI's names (include/chym.h).

Argument marshalling only: torch tensors supply device memory and the
current HIP stream; every step of the computation runs in the library's
kernels.  There is no CPU fallback: if libchym.so is missing or the device is
not gfx950 the calls raise.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from ._lib import (CHYM_J_BF16, CHYM_J_ELL, CHYM_J_F32, CHYM_J_FP8, CHYM_J_I8, CHYM_KERNEL_AUTO, CHYM_KERNEL_LDSJ, CHYM_KERNEL_LDSJ1, CHYM_KERNEL_PIPE, CHYM_KERNEL_REGJ, CHYM_KERNEL_SLAB, CHYM_KERNEL_LDSJ3,
                   CHYM_PREC_BF16, CHYM_PREC_F32, ChymError, ChymOut, ChymPlanEntry, ChymProblem, ChymRun)

__all__ = ["chym_sign_words", "chym_features", "chym_mlp_forward", "chym_mlp_backward", "chym_mlp_adam",
           "chym_mlp_scratch_floats", "chym_to_bf16", "chym_integrate_workspace_size", "chym_version", "chym_last_error", "chym_integrate", "chym_readout", "chym_ising_energy",
           "chym_hs_energy", "chym_solve", "make_problem", "make_run", "spin_words", "ChymError",
           "CHYM_J_I8", "CHYM_J_F32", "CHYM_J_BF16", "CHYM_J_FP8", "CHYM_J_ELL", "ell_pack", "chym_map_integrate", "j_size", "chym_j_bytes", "chym_quantize_fp8", "CHYM_PREC_F32", "CHYM_PREC_BF16", "precision_code",
           "chym_batch_workspace_size", "chym_batch_create", "chym_batch_launch", "chym_batch_launch_nograph",
           "chym_batch_destroy", "ChymBatch", "chym_plan_set", "chym_plan_get", "chym_plan_autotune",
           "chym_plan_save", "chym_plan_load", "chym_split3_bf16", "CHYM_KERNEL_REGJ", "CHYM_KERNEL_LDSJ",
           "CHYM_KERNEL_AUTO", "CHYM_KERNEL_LDSJ1", "CHYM_KERNEL_PIPE", "CHYM_KERNEL_SLAB",
           "CHYM_KERNEL_LDSJ3"]


def precision_code(p) -> int:
    if isinstance(p, str):
        return {"f32": CHYM_PREC_F32, "fp32": CHYM_PREC_F32, "bf16": CHYM_PREC_BF16}[p.lower()]
    return int(p)


def spin_words(n: int) -> int:
    return (n + 63) // 64


def _vp(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _need(t, name, dtype, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def _jdtype(J) -> int:
    """Storage type of J: int8 [n, n], float32 [n, n], bfloat16 [n, n], uint8
    [n + 1, n] for FP8 (E4M3 rows, then the row of E8M0 exponents), or int32
    [n + 1, 2 w] for sparse rows (ELL, see ell_pack)."""
    t = {torch.int8: CHYM_J_I8, torch.float32: CHYM_J_F32, torch.bfloat16: CHYM_J_BF16,
         torch.uint8: CHYM_J_FP8, torch.int32: CHYM_J_ELL}.get(J.dtype)
    if t is None:
        raise TypeError("J must be int8, float32, bfloat16, uint8 (FP8 with row exponents) or int32 (ELL)")
    return t


def j_size(J) -> int:
    """Hyperspin count n of a coupling tensor in any storage type."""
    return int(J.shape[0] - 1) if J.dtype == torch.int32 else int(J.shape[1])


def _need_j(J, n):
    if J.dtype == torch.int32:
        if J.ndim != 2 or J.shape[0] != n + 1 or J.shape[1] < 2 or J.shape[1] % 2:
            raise ValueError(f"sparse J must be int32 [{n + 1}, 2 w], got {tuple(J.shape)}")
        return _need(J, "J", J.dtype)
    shape = (n + 1, n) if J.dtype == torch.uint8 else (n, n)
    return _need(J, "J", J.dtype, shape)


def ell_pack(J, width=None):
    """Host packing of a dense coupling matrix into the sparse-row (ELL)
    storage: int32 [n + 1, 2 w], row 0 = (n, w, 0, ...), row p + 1 = the
    nonzero columns of row p in ascending order, then their couplings as
    float32 bit patterns; rows with fewer than w nonzeros are padded with
    column p and coupling 0.  Returns a numpy array."""
    import numpy as np

    J = np.asarray(J)
    n = J.shape[0]
    nz = [np.flatnonzero(J[p]) for p in range(n)]
    w = max(1, max((len(c) for c in nz), default=1)) if width is None else int(width)
    if any(len(c) > w for c in nz):
        raise ValueError("a row has more nonzeros than the width")
    out = np.zeros((n + 1, 2 * w), dtype=np.int32)
    out[0, 0], out[0, 1] = n, w
    for p, c in enumerate(nz):
        cols = np.full(w, p, dtype=np.int32)
        vals = np.zeros(w, dtype=np.float32)
        cols[:len(c)] = c
        vals[:len(c)] = J[p, c].astype(np.float32)
        out[p + 1, :w] = cols
        out[p + 1, w:] = vals.view(np.int32)
    return out


def make_problem(J, d: int, eps: float, btil: float, eta: float) -> ChymProblem:
    n = j_size(J)
    _need_j(J, n)
    return ChymProblem(n=n, d=int(d), j_dtype=_jdtype(J), reserved=0, j=_vp(J), eps=float(eps),
                       btil=float(btil), eta=float(eta), reserved_f=0.0)


def make_run(n, d, pump, x, alpha, dt, steps, start_step=0, precision=CHYM_PREC_F32) -> ChymRun:
    r = pump.shape[0]
    _need(pump, "pump", torch.float32, (r,))
    _need(x, "x", torch.float32, (n, r, d))
    _need(alpha, "alpha", torch.float32)
    if alpha.ndim != 2 or alpha.shape[1] != d or alpha.shape[0] < start_step + steps:
        raise ValueError(f"alpha must be [>= {start_step + steps}, {d}], got {tuple(alpha.shape)}")
    return ChymRun(r=r, steps=int(steps), start_step=int(start_step), precision=precision_code(precision),
                   dt=float(dt), reserved_f=0.0, pump=_vp(pump), x=_vp(x), alpha=_vp(alpha))


def chym_version() -> int:
    return int(L.load().chym_version())


def chym_last_error() -> str:
    m = L.load().chym_last_error()
    return m.decode() if m else ""


def _workspace(prob, run, device, workspace):
    """Device workspace for the streamed-J integrator (None if not needed)."""
    nbytes = ctypes.c_size_t(0)
    L.check(L.load().chym_integrate_workspace_size(ctypes.byref(prob), ctypes.byref(run), ctypes.byref(nbytes)),
            "chym_integrate_workspace_size")
    if nbytes.value == 0:
        return None, 0
    if workspace is None or workspace.numel() < nbytes.value + 256:
        workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=device)
    off = (-workspace.data_ptr()) % 256
    return workspace[off:], int(nbytes.value)


def chym_integrate_workspace_size(J, x, *, steps=1, precision=CHYM_PREC_F32) -> int:
    n, r, d = x.shape
    prob = make_problem(J, d, 0.0, 0.0, 0.0)
    run = ChymRun(r=r, steps=int(steps), start_step=0, precision=precision_code(precision), dt=1.0, reserved_f=0.0,
                  pump=ctypes.c_void_p(1), x=_vp(x), alpha=ctypes.c_void_p(1))
    nbytes = ctypes.c_size_t(0)
    L.check(L.load().chym_integrate_workspace_size(ctypes.byref(prob), ctypes.byref(run), ctypes.byref(nbytes)),
            "chym_integrate_workspace_size")
    return int(nbytes.value)


def chym_integrate(J, pump, x, alpha, *, eps, btil, eta, dt, steps, start_step=0,
                   precision=CHYM_PREC_F32, stream=None, workspace=None):
    """Advance x [n, r, d] (float32, in place) by ``steps`` Euler steps.
    Problems on the streamed-J integrator get a device workspace (the one
    passed, if large enough, else a new tensor)."""
    lib = L.load()
    n, r, d = x.shape
    prob = make_problem(J, d, eps, btil, eta)
    run = make_run(n, d, pump, x, alpha, dt, steps, start_step, precision)
    ws, nb = _workspace(prob, run, x.device, workspace)
    if ws is None:
        L.check(lib.chym_integrate(ctypes.byref(prob), ctypes.byref(run), _stream(stream)), "chym_integrate")
    else:
        L.check(lib.chym_integrate_ws(ctypes.byref(prob), ctypes.byref(run), _vp(ws), nb, _stream(stream)),
                "chym_integrate_ws")
    return x


def chym_integrate_noalloc(J, pump, x, alpha, *, eps, btil, eta, dt, steps, start_step=0,
                           precision=CHYM_PREC_F32, stream=None):
    """chym_integrate for every size, with the streamed-J staging in the
    library's static device scratch (no workspace, no allocation)."""
    n, r, d = x.shape
    prob = make_problem(J, d, eps, btil, eta)
    run = make_run(n, d, pump, x, alpha, dt, steps, start_step, precision)
    L.check(L.load().chym_integrate_noalloc(ctypes.byref(prob), ctypes.byref(run), _stream(stream)),
            "chym_integrate_noalloc")
    return x


def chym_map_integrate(J, h, A, alpha, *, b, loss, kl, beta_b2, jmag, steps, start_step=0,
                       precision=CHYM_PREC_F32, stream=None):
    """Advance the amplitudes A [n, r, d] (float32, in place) by ``steps``
    round trips of the map of Eq. (2); h [r] is the pump of each replica."""
    n, r, d = A.shape
    _need_j(J, n)
    run = make_run(n, d, h, A, alpha, 1.0, steps, start_step, precision)
    prob = L.ChymMapProblem(n=n, d=d, j_dtype=_jdtype(J), reserved=0, j=_vp(J), b=float(b), loss=float(loss),
                            kl=float(kl), beta_b2=float(beta_b2), jmag=float(jmag), reserved_f=0.0)
    L.check(L.load().chym_map_integrate(ctypes.byref(prob), ctypes.byref(run), _stream(stream)),
            "chym_map_integrate")
    return A


def _map_task(t: dict):
    A = t["A"]
    n, r, d = A.shape
    _need_j(t["J"], n)
    run = make_run(n, d, t["h"], A, t["alpha"], 1.0, t["steps"], t.get("start_step", 0),
                   t.get("precision", CHYM_PREC_F32))
    prob = L.ChymMapProblem(n=n, d=d, j_dtype=_jdtype(t["J"]), reserved=0, j=_vp(t["J"]), b=float(t["b"]),
                            loss=float(t["loss"]), kl=float(t["kl"]), beta_b2=float(t["beta_b2"]),
                            jmag=float(t["jmag"]), reserved_f=0.0)
    return prob, run


def chym_map_batch(tasks, stream=None):
    """Many chym_map_integrate calls in one launch per kernel variant.  tasks:
    dicts with the keyword arguments of chym_map_integrate (J, h, A, alpha, b,
    loss, kl, beta_b2, jmag, steps, [start_step, precision]); every A is
    advanced in place."""
    lib = L.load()
    pairs = [_map_task(t) for t in tasks]
    probs = (L.ChymMapProblem * len(pairs))(*[p for p, _ in pairs])
    runs = (L.ChymRun * len(pairs))(*[r for _, r in pairs])
    nbytes = ctypes.c_size_t(0)
    L.check(lib.chym_map_batch_workspace_size(probs, runs, len(pairs), ctypes.byref(nbytes)),
            "chym_map_batch_workspace_size")
    dev = tasks[0]["A"].device
    ws = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    L.check(lib.chym_map_batch(probs, runs, len(pairs), ctypes.c_void_p(ws.data_ptr() + off), int(nbytes.value),
                               _stream(stream)), "chym_map_batch")
    if stream is not None:
        ws.record_stream(stream)
    return ws  # keep alive until the launches have run (torch's allocator orders reuse on its stream)


def chym_readout(x, spins=None, extra_frac=None, diverged=None, stream=None):
    lib = L.load()
    n, r, d = x.shape
    _need(x, "x", torch.float32)
    if spins is not None:
        _need(spins, "spins", torch.int64, (r, spin_words(n)))
    if extra_frac is not None:
        _need(extra_frac, "extra_frac", torch.float64, (r,))
    if diverged is not None:
        _need(diverged, "diverged", torch.uint8, (r,))
    L.check(lib.chym_readout(n, d, r, _vp(x), _vp(spins), _vp(extra_frac), _vp(diverged), _stream(stream)),
            "chym_readout")


def chym_ising_energy(J, spins, e_i32=None, e_f64=None, stream=None):
    lib = L.load()
    n = j_size(J)
    r = spins.shape[0]
    _need_j(J, n)
    _need(spins, "spins", torch.int64, (r, spin_words(n)))
    if e_i32 is not None:
        _need(e_i32, "e_i32", torch.int32, (r,))
    if e_f64 is not None:
        _need(e_f64, "e_f64", torch.float64, (r,))
    L.check(lib.chym_ising_energy(n, r, _vp(J), _jdtype(J), _vp(spins), _vp(e_i32), _vp(e_f64),
                                  _stream(stream)), "chym_ising_energy")


def chym_hs_energy(J, x, e_hs, stream=None):
    lib = L.load()
    n, r, d = x.shape
    _need_j(J, n)
    _need(x, "x", torch.float32)
    _need(e_hs, "e_hs", torch.float64, (r,))
    L.check(lib.chym_hs_energy(n, d, r, _vp(J), _jdtype(J), _vp(x), _vp(e_hs), _stream(stream)),
            "chym_hs_energy")


def chym_solve(J, pump, x, alpha, *, eps, btil, eta, dt, steps, ss_step=0, start_step=0,
               precision=CHYM_PREC_F32, stream=None, want=("spins", "e_ising", "e_hs", "e_hs_ss",
                                                           "extra_frac", "diverged")):
    """Whole run on x (in place).  Returns a dict of device result tensors."""
    lib = L.load()
    n, r, d = x.shape
    dev = x.device
    prob = make_problem(J, d, eps, btil, eta)
    run = make_run(n, d, pump, x, alpha, dt, steps, start_step, precision)
    res = {}
    want = set(want)
    if want & {"spins", "e_ising", "e_ising_f64"}:
        res["spins"] = torch.empty((r, spin_words(n)), dtype=torch.int64, device=dev)
    if "e_ising" in want and J.dtype == torch.int8:
        res["e_ising"] = torch.empty(r, dtype=torch.int32, device=dev)
    if "e_ising_f64" in want or ("e_ising" in want and J.dtype != torch.int8):
        res["e_ising_f64"] = torch.empty(r, dtype=torch.float64, device=dev)
    for k in ("e_hs", "e_hs_ss", "extra_frac"):
        if k in want:
            res[k] = torch.empty(r, dtype=torch.float64, device=dev)
    if "diverged" in want:
        res["diverged"] = torch.empty(r, dtype=torch.uint8, device=dev)
    out = ChymOut(spins=_vp(res.get("spins")), e_ising=_vp(res.get("e_ising")),
                  e_ising_f64=_vp(res.get("e_ising_f64")), e_hs=_vp(res.get("e_hs")),
                  extra_frac=_vp(res.get("extra_frac")), diverged=_vp(res.get("diverged")))
    ws, nb = _workspace(prob, run, dev, None)
    L.check(lib.chym_solve_ws(ctypes.byref(prob), ctypes.byref(run), int(ss_step), _vp(res.get("e_hs_ss")),
                              ctypes.byref(out), _vp(ws), nb, _stream(stream)), "chym_solve_ws")
    return res


# ------------------------------------------------------------------ batches
def _task_struct(t: dict) -> L.ChymTask:
    J, x = t["J"], t["x"]
    n, r, d = x.shape
    prob = make_problem(J, d, t["eps"], t["btil"], t["eta"])
    run = make_run(n, d, t["pump"], x, t["alpha"], t["dt"], t["steps"], t.get("start_step", 0),
                   t.get("precision", CHYM_PREC_F32))
    w = spin_words(n)
    checks = {"spins": (torch.int64, (r, w)), "e_ising": (torch.int32, (r,)), "e_ising_f64": (torch.float64, (r,)),
              "e_hs": (torch.float64, (r,)), "extra_frac": (torch.float64, (r,)), "diverged": (torch.uint8, (r,))}
    for k, (dt, shp) in checks.items():
        if t.get(k) is not None:
            _need(t[k], k, dt, shp)
    out = ChymOut(spins=_vp(t.get("spins")), e_ising=_vp(t.get("e_ising")), e_ising_f64=_vp(t.get("e_ising_f64")),
                  e_hs=_vp(t.get("e_hs")), extra_frac=_vp(t.get("extra_frac")), diverged=_vp(t.get("diverged")))
    return L.ChymTask(prob=prob, run=run, out=out)


class ChymBatch:
    """A batch plan: keeps the task tensors and the workspace alive."""

    def __init__(self, tasks, handle, workspace, structs):
        self.tasks = tasks
        self.handle = handle
        self.workspace = workspace
        self._structs = structs

    def launch(self, stream=None):
        chym_batch_launch(self, stream)

    def launch_nograph(self, stream=None):
        chym_batch_launch_nograph(self, stream)

    def destroy(self):
        chym_batch_destroy(self)

    def __del__(self):
        try:
            if self.handle is not None:
                self.destroy()
        except Exception:
            pass


def chym_batch_workspace_size(tasks) -> int:
    lib = L.load()
    arr = (L.ChymTask * len(tasks))(*[_task_struct(t) for t in tasks])
    nbytes = ctypes.c_size_t(0)
    L.check(lib.chym_batch_workspace_size(arr, len(tasks), ctypes.byref(nbytes)), "chym_batch_workspace_size")
    return int(nbytes.value)


def chym_batch_create(tasks, device=None) -> ChymBatch:
    """tasks: list of dicts with keys J, pump, x, alpha, eps, btil, eta, dt,
    steps, [start_step, precision] and optional result tensors spins,
    e_ising, e_ising_f64, e_hs, extra_frac, diverged."""
    lib = L.load()
    structs = [_task_struct(t) for t in tasks]
    arr = (L.ChymTask * len(tasks))(*structs)
    nbytes = ctypes.c_size_t(0)
    L.check(lib.chym_batch_workspace_size(arr, len(tasks), ctypes.byref(nbytes)), "chym_batch_workspace_size")
    dev = device if device is not None else tasks[0]["x"].device
    ws = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    wsv = ws[off:off + int(nbytes.value)]
    handle = ctypes.c_void_p()
    L.check(lib.chym_batch_create(arr, len(tasks), ctypes.c_void_p(wsv.data_ptr()), int(nbytes.value),
                                  ctypes.byref(handle)), "chym_batch_create")
    return ChymBatch(list(tasks), handle, ws, arr)


def chym_solve_batched(tasks, stream=None):
    """One-shot batched solve (no graph, no plan kept): the tasks as for
    chym_batch_create, integrated and scored in one call on the stream.
    Returns the workspace tensor, which must stay alive until the launches
    have run (torch's allocator orders its reuse on the stream)."""
    lib = L.load()
    arr = (L.ChymTask * len(tasks))(*[_task_struct(t) for t in tasks])
    nbytes = ctypes.c_size_t(0)
    L.check(lib.chym_batch_workspace_size(arr, len(tasks), ctypes.byref(nbytes)), "chym_batch_workspace_size")
    ws = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=tasks[0]["x"].device)
    off = (-ws.data_ptr()) % 256
    L.check(lib.chym_solve_batched(arr, len(tasks), ctypes.c_void_p(ws.data_ptr() + off), int(nbytes.value),
                                   _stream(stream)), "chym_solve_batched")
    if stream is not None:
        ws.record_stream(stream)
    return ws


def chym_batch_launch(batch: ChymBatch, stream=None):
    L.check(L.load().chym_batch_launch(batch.handle, _stream(stream)), "chym_batch_launch")


def chym_batch_launch_nograph(batch: ChymBatch, stream=None):
    L.check(L.load().chym_batch_launch_nograph(batch.handle, _stream(stream)), "chym_batch_launch_nograph")


def chym_batch_destroy(batch: ChymBatch):
    if batch.handle is not None and batch.handle.value:
        h, batch.handle = batch.handle, None
        L.check(L.load().chym_batch_destroy(h), "chym_batch_destroy")
    batch.handle = None


# ------------------------------------------------------------------ plans
def _entry_dict(e: ChymPlanEntry) -> dict:
    return dict(n=e.n, d=e.d, precision=e.precision, j_dtype=e.j_dtype, kernel=e.kernel, waves=e.waves, ms=e.ms)


def _jcode(j_dtype) -> int:
    if isinstance(j_dtype, torch.dtype):
        return {torch.int8: CHYM_J_I8, torch.float32: CHYM_J_F32, torch.bfloat16: CHYM_J_BF16,
                torch.uint8: CHYM_J_FP8}[j_dtype]
    return int(j_dtype)


def chym_plan_set(n, d, precision, j_dtype, kernel, waves=4):
    e = ChymPlanEntry(n=n, d=d, precision=precision_code(precision), j_dtype=_jcode(j_dtype), kernel=int(kernel),
                      waves=int(waves), ms=0.0, reserved=0.0)
    L.check(L.load().chym_plan_set(ctypes.byref(e)), "chym_plan_set")


def chym_plan_get(n, d, precision, j_dtype) -> dict:
    e = ChymPlanEntry()
    L.check(L.load().chym_plan_get(n, d, precision_code(precision), _jcode(j_dtype), ctypes.byref(e)),
            "chym_plan_get")
    return _entry_dict(e)


def chym_plan_autotune(n, d, precision, j_dtype, replicas=None, steps=200, device=None, stream=None):
    """Time the candidate plans on a synthetic problem and install the best.
    Returns (best, candidates) as dicts."""
    lib = L.load()
    dev = torch.device("cuda") if device is None else torch.device(device)
    if replicas is None:
        cus = torch.cuda.get_device_properties(dev).multi_processor_count
        replicas = cus * 4 * 2 * 16 * 2  # two rounds of two wavefronts per SIMD
    nbytes = ctypes.c_size_t(0)
    L.check(lib.chym_plan_autotune_workspace_size(n, d, replicas, steps, ctypes.byref(nbytes)),
            "chym_plan_autotune_workspace_size")
    ws = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    best = ChymPlanEntry()
    cands = (ChymPlanEntry * 8)()
    nc = ctypes.c_int32(0)
    L.check(lib.chym_plan_autotune(n, d, precision_code(precision), _jcode(j_dtype), replicas, steps,
                                   ctypes.c_void_p(ws.data_ptr() + off), int(nbytes.value), ctypes.byref(best), cands,
                                   8, ctypes.byref(nc), _stream(stream)), "chym_plan_autotune")
    return _entry_dict(best), [_entry_dict(cands[i]) for i in range(nc.value)]


def chym_plan_save(path):
    L.check(L.load().chym_plan_save(str(path).encode()), "chym_plan_save")


def chym_plan_load(path):
    L.check(L.load().chym_plan_load(str(path).encode()), "chym_plan_load")


def chym_split3_bf16(x):
    """(hi, mid, lo) bf16 bit patterns (int16 tensors) of the float32 form's split."""
    n = x.numel()
    _need(x, "x", torch.float32)
    hi, mid, lo = (torch.empty(n, dtype=torch.int16, device=x.device) for _ in range(3))
    L.check(L.load().chym_split3_bf16(_vp(x), n, _vp(hi), _vp(mid), _vp(lo), _stream(None)), "chym_split3_bf16")
    return hi, mid, lo


# --------------------------------------------------------- learned restart
def chym_sign_words(x, words=None, stream=None):
    n, r, d = x.shape
    _need(x, "x", torch.float32)
    if words is None:
        words = torch.empty((r, spin_words(n)), dtype=torch.int64, device=x.device)
    _need(words, "words", torch.int64, (r, spin_words(n)))
    L.check(L.load().chym_sign_words(n, d, r, _vp(x), _vp(words), _stream(stream)), "chym_sign_words")
    return words


def chym_features(J, x, prev_words, features, checkpoint, stream=None):
    n, r, d = x.shape
    _need_j(J, n)
    _need(x, "x", torch.float32)
    _need(prev_words, "prev_words", torch.int64, (r, spin_words(n)))
    _need(features, "features", torch.float32, (r, L.CHYM_FEATURES))
    L.check(L.load().chym_features(n, d, r, _vp(J), _jdtype(J), _vp(x), _vp(prev_words), _vp(features),
                                   int(checkpoint), _stream(stream)), "chym_features")


def chym_feature_standardize(features, group, out=None, stream=None):
    """Standardize features [groups * group, 32] within each group of `group`
    consecutive rows (one pump's batch of runs); out may be features."""
    r = features.shape[0]
    _need(features, "features", torch.float32, (r, L.CHYM_FEATURES))
    if group < 1 or r % group:
        raise ValueError(f"{r} feature rows are not a whole number of groups of {group}")
    if out is None:
        out = torch.empty_like(features)
    _need(out, "out", torch.float32, (r, L.CHYM_FEATURES))
    L.check(L.load().chym_feature_standardize(r // group, int(group), _vp(features), _vp(out), _stream(stream)),
            "chym_feature_standardize")
    return out


def chym_select_top(score, group, keep, idx=None, stream=None):
    """Global indices int32 [groups, keep] of the `keep` highest scores of each
    group of `group` consecutive scores, ascending."""
    r = score.shape[0]
    _need(score, "score", torch.float32, (r,))
    if group < 1 or r % group:
        raise ValueError(f"{r} scores are not a whole number of groups of {group}")
    if idx is None:
        idx = torch.empty((r // group, int(keep)), dtype=torch.int32, device=score.device)
    _need(idx, "idx", torch.int32, (r // group, int(keep)))
    L.check(L.load().chym_select_top(r // group, int(group), int(keep), _vp(score), _vp(idx), _stream(stream)),
            "chym_select_top")
    return idx


def chym_gather_replicas(x, idx, pump=None, x_out=None, pump_out=None, stream=None):
    """Runs idx (int32 [m], entries in [0, r)) of x [n, r, d] into x_out
    [n, m, d], and their pumps into pump_out [m] when pump is given."""
    n, r, d = x.shape
    _need(x, "x", torch.float32)
    idx = idx.reshape(-1)
    _need(idx, "idx", torch.int32)
    m = idx.shape[0]
    if x_out is None:
        x_out = torch.empty((n, m, d), dtype=torch.float32, device=x.device)
    _need(x_out, "x_out", torch.float32, (n, m, d))
    if pump is not None:
        _need(pump, "pump", torch.float32, (r,))
        if pump_out is None:
            pump_out = torch.empty(m, dtype=torch.float32, device=x.device)
        _need(pump_out, "pump_out", torch.float32, (m,))
    L.check(L.load().chym_gather_replicas(n, d, r, _vp(x), _vp(pump), m, _vp(idx), _vp(x_out), _vp(pump_out),
                                          _stream(stream)), "chym_gather_replicas")
    return x_out, pump_out


def chym_mlp_forward(features, w_bf16, logit=None, h1=None, h2=None, stream=None):
    b = features.shape[0]
    _need(features, "features", torch.float32, (b, L.CHYM_FEATURES))
    _need(w_bf16, "w_bf16", torch.int16, (L.CHYM_MLP_PARAMS,))
    if logit is None:
        logit = torch.empty(b, dtype=torch.float32, device=features.device)
    L.check(L.load().chym_mlp_forward(b, _vp(features), _vp(w_bf16), _vp(logit), _vp(h1), _vp(h2), _stream(stream)),
            "chym_mlp_forward")
    return logit


def chym_mlp_scratch_floats(batch) -> int:
    f = ctypes.c_size_t(0)
    L.check(L.load().chym_mlp_scratch_floats(int(batch), ctypes.byref(f)), "chym_mlp_scratch_floats")
    return int(f.value)


def chym_mlp_backward(features, labels, w_bf16, logit, h1, h2, scratch, grad, loss, stream=None):
    b = features.shape[0]
    _need(labels, "labels", torch.float32, (b,))
    _need(grad, "grad", torch.float32, (L.CHYM_MLP_PARAMS,))
    _need(loss, "loss", torch.float32, (b,))
    if scratch.numel() < chym_mlp_scratch_floats(b):
        raise ValueError("scratch too small")
    L.check(L.load().chym_mlp_backward(b, _vp(features), _vp(labels), _vp(w_bf16), _vp(logit), _vp(h1), _vp(h2),
                                       _vp(scratch), _vp(grad), _vp(loss), _stream(stream)), "chym_mlp_backward")


def chym_mlp_adam(w_master, w_bf16, m, v, grad, lr, t, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    for name, tsr in (("w_master", w_master), ("m", m), ("v", v), ("grad", grad)):
        _need(tsr, name, torch.float32, (L.CHYM_MLP_PARAMS,))
    _need(w_bf16, "w_bf16", torch.int16, (L.CHYM_MLP_PARAMS,))
    L.check(L.load().chym_mlp_adam(_vp(w_master), _vp(w_bf16), _vp(m), _vp(v), _vp(grad), float(lr), float(beta1),
                                   float(beta2), float(eps), int(t), _stream(stream)), "chym_mlp_adam")


def chym_to_bf16(src, dst=None, stream=None):
    _need(src, "src", torch.float32)
    if dst is None:
        dst = torch.empty(src.numel(), dtype=torch.int16, device=src.device)
    L.check(L.load().chym_to_bf16(_vp(src), _vp(dst), src.numel(), _stream(stream)), "chym_to_bf16")
    return dst


# ------------------------------------------------------------ FP8 couplings
def chym_j_bytes(n, j_dtype) -> int:
    b = ctypes.c_size_t(0)
    L.check(L.load().chym_j_bytes(int(n), int(j_dtype), ctypes.byref(b)), "chym_j_bytes")
    return int(b.value)


def chym_quantize_fp8(J, out=None, stream=None):
    """float32 J [n, n] (device) -> uint8 [n + 1, n]: E4M3 rows, then the
    E8M0 row exponents."""
    n = J.shape[0]
    _need(J, "J", torch.float32, (n, n))
    if out is None:
        out = torch.empty((n + 1, n), dtype=torch.uint8, device=J.device)
    _need(out, "out", torch.uint8, (n + 1, n))
    L.check(L.load().chym_quantize_fp8(n, _vp(J), _vp(out), _stream(stream)), "chym_quantize_fp8")
    return out
