"""The C-ABI library loads, exports every declared symbol, and validates its
arguments before touching a device (CPU only: no compute calls)."""
import ctypes
import os
import re

import pytest

from paper_2308_02329_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chym.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(chym_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.EXPORTS)


def test_version_and_error_string():
    lib = L.load()
    assert lib.chym_version() == 1
    assert isinstance(lib.chym_last_error(), bytes)


def _prob(**kw):
    base = dict(n=16, d=2, j_dtype=L.CHYM_J_I8, reserved=0, j=0x1000, eps=0.1, btil=1.0, eta=0.0, reserved_f=0.0)
    base.update(kw)
    return L.ChymProblem(**base)


def _run(**kw):
    base = dict(r=4, steps=10, start_step=0, precision=L.CHYM_PREC_F32, dt=0.01, reserved_f=0.0, pump=0x2000,
                x=0x3000, alpha=0x4000)
    base.update(kw)
    return L.ChymRun(**base)


@pytest.mark.parametrize("pk,rk,msg", [
    ({"n": 0}, {}, "n = 0"), ({"d": 0}, {}, "d = 0"), ({"d": 5}, {}, "d = 5"), ({"j_dtype": 7}, {}, "j_dtype"),
    ({"j": None}, {}, "J is NULL"), ({"reserved": 1}, {}, "reserved"), ({"eps": float("inf")}, {}, "finite"),
    ({}, {"r": 0}, "r = 0"), ({}, {"steps": -1}, "steps"), ({}, {"start_step": -2}, "start_step"),
    ({}, {"precision": 9}, "precision"), ({}, {"dt": 0.0}, "dt"), ({}, {"dt": float("nan")}, "dt"),
    ({}, {"x": None}, "NULL"), ({}, {"alpha": None}, "NULL"), ({}, {"pump": None}, "NULL"),
])
def test_integrate_rejects_invalid_arguments(pk, rk, msg):
    lib = L.load()
    p, r = _prob(**pk), _run(**rk)
    rc = lib.chym_integrate(ctypes.byref(p), ctypes.byref(r), None)
    assert rc == L.CHYM_EINVAL
    assert msg in lib.chym_last_error().decode()


def test_null_structs_rejected():
    lib = L.load()
    assert lib.chym_integrate(None, ctypes.byref(_run()), None) == L.CHYM_EINVAL
    assert lib.chym_integrate(ctypes.byref(_prob()), None, None) == L.CHYM_EINVAL


def test_unsupported_size_reported_before_device():
    lib = L.load()
    # beyond every integrator
    rc = lib.chym_integrate(ctypes.byref(_prob(n=1100, d=4)), ctypes.byref(_run()), None)
    assert rc == L.CHYM_EUNSUPPORTED
    # float32 form operand of 16 replicas too large for LDS
    rc = lib.chym_integrate(ctypes.byref(_prob(n=1000, d=4)), ctypes.byref(_run()), None)
    assert rc == L.CHYM_EUNSUPPORTED
    # streamed-J sizes need a workspace
    prob, run = _prob(n=1000, d=4), _run(precision=L.CHYM_PREC_BF16)
    assert lib.chym_integrate(ctypes.byref(prob), ctypes.byref(run), None) == L.CHYM_EUNSUPPORTED
    assert "workspace" in lib.chym_last_error().decode()
    nbytes = ctypes.c_size_t(0)
    assert lib.chym_integrate_workspace_size(ctypes.byref(prob), ctypes.byref(run), ctypes.byref(nbytes)) == 0
    # header, row scales of 63 x 16 rows, 63 row tiles x 32 chunks x 1 KiB fragments, and four chunks of
    # padding that the kernel's prefetch ring may load (and discard) past the last tile
    assert nbytes.value == 256 + 4096 + (63 * 32 + 4) * 1024
    assert lib.chym_integrate_ws(ctypes.byref(prob), ctypes.byref(run), ctypes.c_void_p(0x10000), 100,
                                 None) == L.CHYM_ENOMEM
    small = _prob(n=100, d=2)
    assert lib.chym_integrate_workspace_size(ctypes.byref(small), ctypes.byref(_run()), ctypes.byref(nbytes)) == 0
    assert nbytes.value == 0


def test_other_entry_points_validate():
    lib = L.load()
    assert lib.chym_readout(0, 2, 4, 0x1000, 0x2000, None, None, None) == L.CHYM_EINVAL
    assert lib.chym_readout(16, 2, 4, None, 0x2000, None, None, None) == L.CHYM_EINVAL
    assert lib.chym_readout(16, 2, 4, 0x1000, None, None, None, None) == L.CHYM_OK  # nothing requested
    # int32 energy needs integer couplings
    assert lib.chym_ising_energy(16, 4, 0x1000, L.CHYM_J_F32, 0x2000, 0x3000, None, None) == L.CHYM_EINVAL
    assert lib.chym_ising_energy(4096, 4, 0x1000, L.CHYM_J_I8, 0x2000, 0x3000, None, None) == L.CHYM_EUNSUPPORTED
    assert lib.chym_hs_energy(3000, 4, 2, 0x1000, L.CHYM_J_I8, 0x2000, 0x3000, None) == L.CHYM_EUNSUPPORTED
    out = L.ChymOut(e_ising=0x5000)  # energy without spins
    assert lib.chym_solve(ctypes.byref(_prob()), ctypes.byref(_run()), 0, None, ctypes.byref(out),
                          None) == L.CHYM_EINVAL
    assert lib.chym_solve(ctypes.byref(_prob()), ctypes.byref(_run()), -1, None, None, None) == L.CHYM_EINVAL


def test_batch_validation():
    lib = L.load()
    tasks = (L.ChymTask * 2)(L.ChymTask(prob=_prob(), run=_run()), L.ChymTask(prob=_prob(n=0), run=_run()))
    nbytes = ctypes.c_size_t(0)
    assert lib.chym_batch_workspace_size(tasks, 2, ctypes.byref(nbytes)) == L.CHYM_EINVAL
    assert "task 1" in lib.chym_last_error().decode()
    assert lib.chym_batch_workspace_size(tasks, 1, ctypes.byref(nbytes)) == L.CHYM_OK
    assert nbytes.value > 0
    assert lib.chym_batch_workspace_size(tasks, 0, ctypes.byref(nbytes)) == L.CHYM_EINVAL
    plan = ctypes.c_void_p()
    # too small a workspace is reported before any device work
    assert lib.chym_batch_create(tasks, 1, ctypes.c_void_p(0x10000), 16, ctypes.byref(plan)) == L.CHYM_ENOMEM
    assert lib.chym_batch_create(tasks, 1, ctypes.c_void_p(0x10001), nbytes.value,
                                 ctypes.byref(plan)) == L.CHYM_EINVAL
    assert lib.chym_batch_launch(None, None) == L.CHYM_EINVAL
    assert lib.chym_batch_destroy(None) == L.CHYM_OK


def test_valid_call_without_device_reports_enodev():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = L.load()
    assert lib.chym_integrate(ctypes.byref(_prob()), ctypes.byref(_run()), None) == L.CHYM_ENODEV


def test_python_binding_has_no_fallback(tmp_path, monkeypatch):
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(ImportError):
        L.load()


def test_plan_table_validation_and_file_roundtrip(tmp_path):
    lib = L.load()
    e = L.ChymPlanEntry(n=100, d=3, precision=L.CHYM_PREC_F32, j_dtype=L.CHYM_J_I8, kernel=L.CHYM_KERNEL_LDSJ,
                        waves=2, ms=0.0, reserved=0.0)
    assert lib.chym_plan_set(ctypes.byref(e)) == L.CHYM_OK
    got = L.ChymPlanEntry()
    assert lib.chym_plan_get(112, 3, L.CHYM_PREC_F32, L.CHYM_J_I8, ctypes.byref(got)) == L.CHYM_OK  # same tiles
    assert (got.kernel, got.waves) == (L.CHYM_KERNEL_LDSJ, 2)
    path = str(tmp_path / "plan.txt").encode()
    assert lib.chym_plan_save(path) == L.CHYM_OK
    e.kernel = L.CHYM_KERNEL_AUTO
    assert lib.chym_plan_set(ctypes.byref(e)) == L.CHYM_OK
    assert lib.chym_plan_get(100, 3, L.CHYM_PREC_F32, L.CHYM_J_I8, ctypes.byref(got)) == L.CHYM_OK
    assert got.kernel == L.CHYM_KERNEL_REGJ  # default
    assert lib.chym_plan_load(path) == L.CHYM_OK
    assert lib.chym_plan_get(100, 3, L.CHYM_PREC_F32, L.CHYM_J_I8, ctypes.byref(got)) == L.CHYM_OK
    assert got.kernel == L.CHYM_KERNEL_LDSJ
    e.kernel = L.CHYM_KERNEL_AUTO
    lib.chym_plan_set(ctypes.byref(e))
    bad = tmp_path / "bad.txt"
    bad.write_text("7 3 3 1 9 2 0.0\n")
    assert lib.chym_plan_load(str(bad).encode()) == L.CHYM_EINVAL
    for kw in ({"kernel": 7}, {"waves": 0}, {"waves": 5}, {"d": 0}, {"n": 0}, {"n": 4000}):
        e2 = L.ChymPlanEntry(n=100, d=3, precision=0, j_dtype=0, kernel=L.CHYM_KERNEL_REGJ, waves=2)
        for k, v in kw.items():
            setattr(e2, k, v)
        assert lib.chym_plan_set(ctypes.byref(e2)) in (L.CHYM_EINVAL, L.CHYM_EUNSUPPORTED)
    assert lib.chym_split3_bf16(None, 8, None, None, None, None) == L.CHYM_EINVAL
    assert lib.chym_split3_bf16(0x1000, 7, 0x2000, 0x3000, 0x4000, None) == L.CHYM_EINVAL


def test_three_wave_lds_plans():
    """CHYM_KERNEL_LDSJ3 (three wavefronts per SIMD) is accepted where its
    step loop is built (up to 10 / 7 / 4 / 3 row tiles at d = 1..4, 8 / 5 /
    3 / 3 with float couplings in the float32 form) and refused elsewhere."""
    lib = L.load()
    bf, f32, i8, fl = L.CHYM_PREC_BF16, L.CHYM_PREC_F32, L.CHYM_J_I8, L.CHYM_J_F32
    got = L.ChymPlanEntry()
    for n, d, prec, jd, ok in ((100, 2, f32, i8, True), (160, 1, f32, i8, True), (40, 4, f32, i8, True),
                               (64, 3, bf, i8, True), (80, 2, f32, fl, True), (128, 1, f32, fl, True),
                               (100, 3, f32, i8, False), (112, 2, bf, i8, True), (128, 2, bf, i8, False),
                               (96, 2, f32, fl, False), (64, 4, bf, i8, False), (176, 1, f32, i8, False)):
        e = L.ChymPlanEntry(n=n, d=d, precision=prec, j_dtype=jd, kernel=L.CHYM_KERNEL_LDSJ3, waves=4, ms=0.0,
                            reserved=0.0)
        rc = lib.chym_plan_set(ctypes.byref(e))
        assert rc == (L.CHYM_OK if ok else L.CHYM_EUNSUPPORTED), (n, d, prec, jd)
        if ok:
            assert lib.chym_plan_get(n, d, prec, jd, ctypes.byref(got)) == L.CHYM_OK
            assert (got.kernel, got.waves) == (L.CHYM_KERNEL_LDSJ3, 4)
            e.kernel = L.CHYM_KERNEL_AUTO
            assert lib.chym_plan_set(ctypes.byref(e)) == L.CHYM_OK


def test_plan_file_refuses_kinds_not_built(tmp_path):
    """A plan file naming a kind that is not built for its variant is
    refused as a whole (tiles d xs js kernel waves ms)."""
    lib = L.load()
    good = tmp_path / "good.txt"
    good.write_text("7 2 3 1 6 4 1.0\n7 3 3 1 2 4 1.0\n")
    assert lib.chym_plan_load(str(good).encode()) == L.CHYM_OK
    got = L.ChymPlanEntry()
    assert lib.chym_plan_get(100, 2, L.CHYM_PREC_F32, L.CHYM_J_I8, ctypes.byref(got)) == L.CHYM_OK
    assert got.kernel == L.CHYM_KERNEL_LDSJ3
    for line in ("7 3 3 1 6 4 1.0\n",    # three wavefronts per SIMD: not built at 7 tiles, d = 3
                 "7 4 3 1 4 4 1.0\n",    # pipelined: d = 2, 3 only
                 "6 3 3 3 4 4 1.0\n"):   # pipelined: one coupling term only
        bad = tmp_path / "bad.txt"
        bad.write_text(line)
        assert lib.chym_plan_load(str(bad).encode()) == L.CHYM_EINVAL, line
    for n, d in ((100, 2), (100, 3)):
        e = L.ChymPlanEntry(n=n, d=d, precision=L.CHYM_PREC_F32, j_dtype=L.CHYM_J_I8, kernel=L.CHYM_KERNEL_AUTO,
                            waves=4, ms=0.0, reserved=0.0)
        assert lib.chym_plan_set(ctypes.byref(e)) == L.CHYM_OK


def test_streamed_j_plans(tmp_path):
    """Streamed-J variants (beyond the register-resident tile limits) take
    CHYM_KERNEL_SLAB plans whose `waves` is the block size: 16 by default up
    to 32 row tiles in the bf16 form, 8 beyond and in the float32 form; the
    other kinds are refused there, and CHYM_KERNEL_SLAB is refused on
    register-resident variants."""
    lib = L.load()
    got = L.ChymPlanEntry()
    bf, f32, i8 = L.CHYM_PREC_BF16, L.CHYM_PREC_F32, L.CHYM_J_I8
    for n, d, prec, want in ((400, 4, bf, 16), (512, 2, bf, 16), (800, 4, bf, 8), (1000, 3, bf, 8), (400, 2, f32, 8)):
        assert lib.chym_plan_get(n, d, prec, i8, ctypes.byref(got)) == L.CHYM_OK
        assert (got.kernel, got.waves) == (L.CHYM_KERNEL_SLAB, want), (n, d, prec)
    assert lib.chym_plan_get(100, 3, bf, i8, ctypes.byref(got)) == L.CHYM_OK
    assert got.kernel == L.CHYM_KERNEL_REGJ
    assert lib.chym_plan_get(1100, 2, bf, i8, ctypes.byref(got)) == L.CHYM_EUNSUPPORTED  # beyond every integrator

    def entry(n, d, prec, kernel, waves):
        return L.ChymPlanEntry(n=n, d=d, precision=prec, j_dtype=i8, kernel=kernel, waves=waves, ms=0.0, reserved=0.0)

    e = entry(800, 2, bf, L.CHYM_KERNEL_SLAB, 16)
    assert lib.chym_plan_set(ctypes.byref(e)) == L.CHYM_OK
    assert lib.chym_plan_get(800, 2, bf, i8, ctypes.byref(got)) == L.CHYM_OK
    assert (got.kernel, got.waves) == (L.CHYM_KERNEL_SLAB, 16)
    path = str(tmp_path / "plan.txt").encode()
    assert lib.chym_plan_save(path) == L.CHYM_OK
    e.kernel = L.CHYM_KERNEL_AUTO
    assert lib.chym_plan_set(ctypes.byref(e)) == L.CHYM_OK
    assert lib.chym_plan_get(800, 2, bf, i8, ctypes.byref(got)) == L.CHYM_OK and got.waves == 8
    assert lib.chym_plan_load(path) == L.CHYM_OK
    assert lib.chym_plan_get(800, 2, bf, i8, ctypes.byref(got)) == L.CHYM_OK and got.waves == 16
    assert lib.chym_plan_set(ctypes.byref(e)) == L.CHYM_OK  # back to the default
    for bad, rc in ((entry(800, 4, bf, L.CHYM_KERNEL_LDSJ, 2), L.CHYM_EUNSUPPORTED),   # resident kind on streamed-J
                    (entry(100, 3, bf, L.CHYM_KERNEL_SLAB, 8), L.CHYM_EUNSUPPORTED),  # streamed-J kind on resident
                    (entry(800, 4, bf, L.CHYM_KERNEL_SLAB, 4), L.CHYM_EINVAL),        # block size
                    (entry(800, 4, bf, L.CHYM_KERNEL_SLAB, 16), L.CHYM_EUNSUPPORTED),  # 4 tiles of d = 4 per wave
                    (entry(400, 2, f32, L.CHYM_KERNEL_SLAB, 16), L.CHYM_EUNSUPPORTED)):  # not built in float32
        assert lib.chym_plan_set(ctypes.byref(bad)) == rc
    for line in ("50 4 1 1 5 4 0.0\n", "7 3 1 1 5 8 0.0\n", "25 2 3 1 5 16 0.0\n"):
        f = tmp_path / "bad.txt"
        f.write_text(line)
        assert lib.chym_plan_load(str(f).encode()) == L.CHYM_EINVAL, line


def test_coupling_storage_sizes_and_quantizer_validation():
    lib = L.load()
    b = ctypes.c_size_t(0)
    for jt, want in ((L.CHYM_J_I8, 25), (L.CHYM_J_F32, 100), (L.CHYM_J_BF16, 50), (L.CHYM_J_FP8, 30)):
        assert lib.chym_j_bytes(5, jt, ctypes.byref(b)) == L.CHYM_OK
        assert b.value == want
    assert lib.chym_j_bytes(5, 9, ctypes.byref(b)) == L.CHYM_EINVAL
    assert lib.chym_j_bytes(0, L.CHYM_J_FP8, ctypes.byref(b)) == L.CHYM_EINVAL
    assert lib.chym_j_bytes(5, L.CHYM_J_FP8, None) == L.CHYM_EINVAL
    assert lib.chym_quantize_fp8(0, 0x1000, 0x2000, None) == L.CHYM_EINVAL
    assert lib.chym_quantize_fp8(8, None, 0x2000, None) == L.CHYM_EINVAL
    assert lib.chym_quantize_fp8(8, 0x1000, None, None) == L.CHYM_EINVAL
    for jt in (L.CHYM_J_BF16, L.CHYM_J_FP8):
        # int32 energies need integer couplings (rejected before any device work)
        assert lib.chym_ising_energy(16, 4, 0x1000, jt, 0x2000, 0x3000, None, None) == L.CHYM_EINVAL
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        return  # the calls below pass fake pointers: only where no device can run them
    for jt in (L.CHYM_J_BF16, L.CHYM_J_FP8):
        # the new storages pass validation and stop at the missing device
        rc = lib.chym_integrate(ctypes.byref(_prob(j_dtype=jt)), ctypes.byref(_run()), None)
        assert rc == L.CHYM_ENODEV


def test_map_entry_point_validates_before_device():
    lib = L.load()

    def mp(**kw):
        base = dict(n=16, d=2, j_dtype=L.CHYM_J_I8, reserved=0, j=0x1000, b=0.01, loss=0.01, kl=0.1, beta_b2=25.0,
                    jmag=1.0, reserved_f=0.0)
        base.update(kw)
        return L.ChymMapProblem(**base)

    run1 = _run(dt=1.0)
    for kw, code in (({"b": 0.0}, L.CHYM_EINVAL), ({"b": 1.0}, L.CHYM_EINVAL), ({"loss": 1.0}, L.CHYM_EINVAL),
                     ({"kl": 0.0}, L.CHYM_EINVAL), ({"beta_b2": -1.0}, L.CHYM_EINVAL), ({"n": 0}, L.CHYM_EINVAL),
                     ({"d": 5}, L.CHYM_EINVAL), ({"j": None}, L.CHYM_EINVAL), ({"reserved_f": 1.0}, L.CHYM_EINVAL),
                     ({"j_dtype": L.CHYM_J_F32}, L.CHYM_EUNSUPPORTED), ({"n": 113}, L.CHYM_EUNSUPPORTED)):
        assert lib.chym_map_integrate(ctypes.byref(mp(**kw)), ctypes.byref(run1), None) == code, kw
    # one round trip per step
    assert lib.chym_map_integrate(ctypes.byref(mp()), ctypes.byref(_run(dt=0.5)), None) == L.CHYM_EINVAL
    assert "dt must be 1" in lib.chym_last_error().decode()
    assert lib.chym_map_integrate(None, ctypes.byref(run1), None) == L.CHYM_EINVAL


def test_map_batch_layout_and_validation():
    lib = L.load()

    def mp(**kw):
        base = dict(n=40, d=2, j_dtype=L.CHYM_J_I8, reserved=0, j=0x1000, b=0.01, loss=0.01, kl=0.1, beta_b2=25.0,
                    jmag=1.0, reserved_f=0.0)
        base.update(kw)
        return L.ChymMapProblem(**base)

    probs = (L.ChymMapProblem * 3)(mp(), mp(n=16, d=1), mp(b=1.5))
    runs = (L.ChymRun * 3)(_run(dt=1.0, r=40), _run(dt=1.0, r=17), _run(dt=1.0))
    nbytes = ctypes.c_size_t(0)
    assert lib.chym_map_batch_workspace_size(probs, runs, 3, ctypes.byref(nbytes)) == L.CHYM_EINVAL
    assert "task 2" in lib.chym_last_error().decode() and "b must" in lib.chym_last_error().decode()
    assert lib.chym_map_batch_workspace_size(probs, runs, 2, ctypes.byref(nbytes)) == L.CHYM_OK
    # task table, work items (3 + 2 groups of 16 replicas), one counter per variant: 256-byte aligned areas
    assert nbytes.value % 256 == 0 and nbytes.value >= 3 * 256
    assert lib.chym_map_batch_workspace_size(probs, runs, 0, ctypes.byref(nbytes)) == L.CHYM_EINVAL
    assert lib.chym_map_batch_workspace_size(None, runs, 1, ctypes.byref(nbytes)) == L.CHYM_EINVAL
    # an invalid task fails before any device work or workspace check
    assert lib.chym_map_batch(probs, runs, 3, None, 0, None) == L.CHYM_EINVAL
    assert "task 2" in lib.chym_last_error().decode()
    ell = (L.ChymMapProblem * 1)(mp(j_dtype=L.CHYM_J_ELL))
    assert lib.chym_map_batch_workspace_size(ell, runs, 1, ctypes.byref(nbytes)) == L.CHYM_EUNSUPPORTED
    import torch

    if not torch.cuda.is_available():
        # a valid batch without a workspace is refused before the device is touched
        assert lib.chym_map_batch(probs, runs, 2, None, 0, None) == L.CHYM_EINVAL
        assert "workspace" in lib.chym_last_error().decode()


def test_sparse_couplings_validation():
    lib = L.load()
    b = ctypes.c_size_t(0)
    assert lib.chym_j_bytes(10, L.CHYM_J_ELL, ctypes.byref(b)) == L.CHYM_EINVAL  # depends on the row width
    assert lib.chym_integrate(ctypes.byref(_prob(n=5000, j_dtype=L.CHYM_J_ELL)), ctypes.byref(_run()),
                              None) == L.CHYM_EUNSUPPORTED
    assert lib.chym_features(16, 2, 4, 0x1000, L.CHYM_J_ELL, 0x2000, 0x3000, 0x4000, 0, None) == L.CHYM_EUNSUPPORTED
    assert lib.chym_ising_energy(16, 4, 0x1000, L.CHYM_J_ELL, 0x2000, 0x3000, None, None) == L.CHYM_EINVAL
    # batches take sparse rows (no staging area: the tables only), up to the gather kernel's n
    tasks = (L.ChymTask * 1)(L.ChymTask(prob=_prob(j_dtype=L.CHYM_J_ELL), run=_run()))
    nbytes = ctypes.c_size_t(0)
    assert lib.chym_batch_workspace_size(tasks, 1, ctypes.byref(nbytes)) == L.CHYM_OK
    dense = (L.ChymTask * 1)(L.ChymTask(prob=_prob(), run=_run()))
    nb2 = ctypes.c_size_t(0)
    assert lib.chym_batch_workspace_size(dense, 1, ctypes.byref(nb2)) == L.CHYM_OK
    assert 0 < nbytes.value <= nb2.value
    big = (L.ChymTask * 1)(L.ChymTask(prob=_prob(n=5000, j_dtype=L.CHYM_J_ELL), run=_run()))
    assert lib.chym_batch_workspace_size(big, 1, ctypes.byref(nbytes)) == L.CHYM_EUNSUPPORTED
    assert "task 0" in lib.chym_last_error().decode()
    # the exact int32 energy is for int8 couplings only
    out = L.ChymOut(spins=0x5000, e_ising=0x6000)
    ell_i32 = (L.ChymTask * 1)(L.ChymTask(prob=_prob(j_dtype=L.CHYM_J_ELL), run=_run(), out=out))
    assert lib.chym_batch_workspace_size(ell_i32, 1, ctypes.byref(nbytes)) != L.CHYM_OK


def test_ell_pack_layout():
    import numpy as np

    from paper_2308_02329_amd import api

    J = np.array([[0, 1, 0, -2], [1, 0, 0, 0], [0, 0, 0, 0], [-2, 0, 0, 0]], dtype=np.float32)
    e = api.ell_pack(J)
    assert e.shape == (5, 4) and e.dtype == np.int32
    assert (e[0, 0], e[0, 1]) == (4, 2)
    assert list(e[1, :2]) == [1, 3] and list(e[1, 2:].view(np.float32)) == [1.0, -2.0]
    assert list(e[2, :2]) == [0, 1] and list(e[2, 2:].view(np.float32)) == [1.0, 0.0]  # padded with (p, 0)
    assert list(e[3, 2:].view(np.float32)) == [0.0, 0.0]
    with pytest.raises(ValueError):
        api.ell_pack(J, width=1)


def test_streamed_j_size_limits():
    """Largest n per d and form that validates: 1024 (the block's eight
    wavefronts take at most 8 row tiles each) in both forms; the float32 form
    beyond n = 832, 544, 416 (d = 2, 3, 4) takes component passes."""
    lib = L.load()

    def ok(n, d, prec):
        prob = _prob(n=n, d=d)
        run = _run(r=16, precision=prec)
        nb = ctypes.c_size_t(0)
        return lib.chym_integrate_workspace_size(ctypes.byref(prob), ctypes.byref(run), ctypes.byref(nb)) == L.CHYM_OK

    for d in (1, 2, 3, 4):
        for prec in (L.CHYM_PREC_F32, L.CHYM_PREC_BF16):
            assert ok(1024, d, prec) and not ok(1025, d, prec), (d, prec)
        for n in (416, 417, 544, 545, 832, 833):
            assert ok(n, d, L.CHYM_PREC_F32), (n, d)
