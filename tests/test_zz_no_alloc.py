"""chym_integrate_noalloc (streamed-J staging in the library's static
device scratch, no workspace, no allocation) against chym_integrate_ws on
the same inputs: bit-identical states, on two calls in a row whose second
input is smaller (the scratch keeps the first call's staging), and on a
size the register-resident integrator takes (no staging)."""
import ctypes

import numpy as np
import pytest

from paper_2308_02329_amd import _lib as L
from paper_2308_02329_amd import api

torch = pytest.importorskip("torch")
from gpu_helpers import Case, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu


def _ws_reference(case, Jd, prec):
    _, pump, x, alpha = case.gpu_inputs()
    ws = torch.empty(api.chym_integrate_workspace_size(Jd, x, precision=prec) + 256, dtype=torch.uint8,
                     device="cuda")
    api.chym_integrate(Jd, pump, x, alpha, steps=case.steps, precision=prec, workspace=ws, **case.params())
    return x


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_equals_workspace_entry_point(order):
    # (n, d, r, steps, couplings, form): the first needs the largest staging of the three
    # (float32 couplings in three bf16 terms), the second a smaller one, the third none
    specs = [(700, 2, 37, 120, "gauss", "f32"), (300, 3, 20, 150, "sk", "bf16"), (100, 3, 24, 200, "sk", "f32")]
    for i, (n, d, r, steps, kind, prec) in enumerate(specs):
        print(f"[noalloc] call {i}: n={n} d={d} r={r} steps={steps} {kind} {prec}", flush=True)
        case = Case(n, d, r, steps, key=(48, i), kind=kind, sigma=0.03)
        Jd = to_dev(case.J)
        need = api.chym_integrate_workspace_size(Jd, to_dev(case.x0), precision=prec)
        assert (need > 0) == (i < 2)
        ref = _ws_reference(case, Jd, prec)
        _, pump, x, alpha = case.gpu_inputs()
        api.chym_integrate_noalloc(Jd, pump, x, alpha, steps=steps, precision=prec, **case.params())
        torch.cuda.synchronize()
        assert torch.equal(x, ref), (n, d, prec)
        assert torch.isfinite(x).all()


def test_noalloc_validates_before_any_device_work():
    lib = L.load()
    prob = L.ChymProblem(n=1100, d=1, j_dtype=L.CHYM_J_I8, reserved=0, j=0x1000, eps=0.1, btil=1.0, eta=0.0,
                         reserved_f=0.0)
    run = L.ChymRun(r=16, steps=10, start_step=0, precision=L.CHYM_PREC_BF16, dt=0.01, reserved_f=0.0,
                    pump=ctypes.c_void_p(0x2000), x=ctypes.c_void_p(0x3000), alpha=ctypes.c_void_p(0x4000))
    assert lib.chym_integrate_noalloc(ctypes.byref(prob), ctypes.byref(run), None) == L.CHYM_EUNSUPPORTED
    prob.n, prob.eps = 300, float("nan")
    assert lib.chym_integrate_noalloc(ctypes.byref(prob), ctypes.byref(run), None) == L.CHYM_EINVAL
