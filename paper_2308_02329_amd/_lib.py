"""ctypes view of libchym's C ABI (include/chym.h).  Marshalling only."""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
# CHYM_SANITIZED_LIBS=1: the host-sanitized build (python -m paper_2308_02329_amd.build --sanitize)
LIB_PATH = os.path.join(PKG, "libchym_san.so" if os.environ.get("CHYM_SANITIZED_LIBS") == "1" else "libchym.so")

CHYM_OK = 0
CHYM_EINVAL = -1
CHYM_EUNSUPPORTED = -2
CHYM_ENODEV = -3
CHYM_EHIP = -4
CHYM_ENOMEM = -5
ERROR_NAMES = {0: "CHYM_OK", -1: "CHYM_EINVAL", -2: "CHYM_EUNSUPPORTED", -3: "CHYM_ENODEV",
               -4: "CHYM_EHIP", -5: "CHYM_ENOMEM"}

CHYM_J_I8 = 0
CHYM_J_F32 = 1
CHYM_J_BF16 = 2
CHYM_J_FP8 = 3
CHYM_J_ELL = 4
CHYM_PREC_F32 = 0
CHYM_PREC_BF16 = 1

# every symbol include/chym.h declares
EXPORTS = (
    "chym_version", "chym_last_error", "chym_integrate", "chym_readout", "chym_ising_energy",
    "chym_hs_energy", "chym_solve", "chym_batch_workspace_size", "chym_batch_create",
    "chym_batch_launch", "chym_batch_launch_nograph", "chym_batch_destroy", "chym_solve_batched", "chym_plan_set",
    "chym_plan_get", "chym_plan_autotune_workspace_size", "chym_plan_autotune", "chym_split3_bf16", "chym_j_bytes",
    "chym_quantize_fp8", "chym_plan_save",
    "chym_plan_load", "chym_integrate_workspace_size", "chym_integrate_ws", "chym_solve_ws",
    "chym_sign_words", "chym_features", "chym_mlp_scratch_floats", "chym_mlp_forward", "chym_mlp_backward",
    "chym_mlp_adam", "chym_to_bf16", "chym_map_integrate", "chym_map_batch_workspace_size", "chym_map_batch",
    "chym_integrate_noalloc", "chym_feature_standardize", "chym_select_top", "chym_gather_replicas",
)

CHYM_FEATURES = 32
CHYM_MLP_PARAMS = 20865

CHYM_KERNEL_AUTO = 0
CHYM_KERNEL_REGJ = 1
CHYM_KERNEL_LDSJ = 2
CHYM_KERNEL_LDSJ1 = 3
CHYM_KERNEL_PIPE = 4
CHYM_KERNEL_SLAB = 5
CHYM_KERNEL_LDSJ3 = 6

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32


class ChymProblem(ctypes.Structure):
    _fields_ = [("n", _i32), ("d", _i32), ("j_dtype", _i32), ("reserved", _i32), ("j", _vp),
                ("eps", ctypes.c_float), ("btil", ctypes.c_float), ("eta", ctypes.c_float),
                ("reserved_f", ctypes.c_float)]


class ChymMapProblem(ctypes.Structure):
    _fields_ = [("n", _i32), ("d", _i32), ("j_dtype", _i32), ("reserved", _i32), ("j", _vp),
                ("b", ctypes.c_float), ("loss", ctypes.c_float), ("kl", ctypes.c_float),
                ("beta_b2", ctypes.c_float), ("jmag", ctypes.c_float), ("reserved_f", ctypes.c_float)]


class ChymRun(ctypes.Structure):
    _fields_ = [("r", _i32), ("steps", _i32), ("start_step", _i32), ("precision", _i32),
                ("dt", ctypes.c_float), ("reserved_f", ctypes.c_float), ("pump", _vp), ("x", _vp),
                ("alpha", _vp)]


class ChymOut(ctypes.Structure):
    _fields_ = [("spins", _vp), ("e_ising", _vp), ("e_ising_f64", _vp), ("e_hs", _vp),
                ("extra_frac", _vp), ("diverged", _vp)]


class ChymError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Load the in-tree libchym.so; fail loudly if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2308_02329_amd.build` "
                          "(there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.chym_version.restype = ctypes.c_int
    lib.chym_last_error.restype = ctypes.c_char_p
    lib.chym_integrate.argtypes = [P(ChymProblem), P(ChymRun), _vp]
    lib.chym_integrate.restype = ctypes.c_int
    lib.chym_map_integrate.argtypes = [P(ChymMapProblem), P(ChymRun), _vp]
    lib.chym_map_integrate.restype = ctypes.c_int
    lib.chym_map_batch_workspace_size.argtypes = [P(ChymMapProblem), P(ChymRun), ctypes.c_int32,
                                                  P(ctypes.c_size_t)]
    lib.chym_map_batch_workspace_size.restype = ctypes.c_int
    lib.chym_map_batch.argtypes = [P(ChymMapProblem), P(ChymRun), ctypes.c_int32, _vp, ctypes.c_size_t, _vp]
    lib.chym_map_batch.restype = ctypes.c_int
    lib.chym_readout.argtypes = [_i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp]
    lib.chym_readout.restype = ctypes.c_int
    lib.chym_ising_energy.argtypes = [_i32, _i32, _vp, _i32, _vp, _vp, _vp, _vp]
    lib.chym_ising_energy.restype = ctypes.c_int
    lib.chym_hs_energy.argtypes = [_i32, _i32, _i32, _vp, _i32, _vp, _vp, _vp]
    lib.chym_hs_energy.restype = ctypes.c_int
    lib.chym_solve.argtypes = [P(ChymProblem), P(ChymRun), _i32, _vp, P(ChymOut), _vp]
    lib.chym_solve.restype = ctypes.c_int
    lib.chym_solve_ws.argtypes = [P(ChymProblem), P(ChymRun), _i32, _vp, P(ChymOut), _vp, ctypes.c_size_t, _vp]
    lib.chym_solve_ws.restype = ctypes.c_int
    lib.chym_integrate_workspace_size.argtypes = [P(ChymProblem), P(ChymRun), P(ctypes.c_size_t)]
    lib.chym_integrate_workspace_size.restype = ctypes.c_int
    lib.chym_integrate_ws.argtypes = [P(ChymProblem), P(ChymRun), _vp, ctypes.c_size_t, _vp]
    lib.chym_integrate_ws.restype = ctypes.c_int
    lib.chym_integrate_noalloc.argtypes = [P(ChymProblem), P(ChymRun), _vp]
    lib.chym_integrate_noalloc.restype = ctypes.c_int
    _load_batch(lib)
    _load_plan(lib)
    _load_learned(lib)
    _lib = lib
    return lib


def check(rc: int, where: str):
    if rc != CHYM_OK:
        msg = load().chym_last_error()
        raise ChymError(rc, where, msg.decode() if msg else "")


class ChymTask(ctypes.Structure):
    _fields_ = [("prob", ChymProblem), ("run", ChymRun), ("out", ChymOut)]


def _load_batch(lib):
    P = ctypes.POINTER
    lib.chym_batch_workspace_size.argtypes = [P(ChymTask), _i32, P(ctypes.c_size_t)]
    lib.chym_batch_workspace_size.restype = ctypes.c_int
    lib.chym_batch_create.argtypes = [P(ChymTask), _i32, _vp, ctypes.c_size_t, P(_vp)]
    lib.chym_batch_create.restype = ctypes.c_int
    lib.chym_solve_batched.argtypes = [P(ChymTask), _i32, _vp, ctypes.c_size_t, _vp]
    lib.chym_solve_batched.restype = ctypes.c_int
    lib.chym_batch_launch.argtypes = [_vp, _vp]
    lib.chym_batch_launch.restype = ctypes.c_int
    lib.chym_batch_launch_nograph.argtypes = [_vp, _vp]
    lib.chym_batch_launch_nograph.restype = ctypes.c_int
    lib.chym_batch_destroy.argtypes = [_vp]
    lib.chym_batch_destroy.restype = ctypes.c_int


class ChymPlanEntry(ctypes.Structure):
    _fields_ = [("n", _i32), ("d", _i32), ("precision", _i32), ("j_dtype", _i32), ("kernel", _i32),
                ("waves", _i32), ("ms", ctypes.c_float), ("reserved", ctypes.c_float)]


def _load_plan(lib):
    P = ctypes.POINTER
    lib.chym_plan_set.argtypes = [P(ChymPlanEntry)]
    lib.chym_plan_get.argtypes = [_i32, _i32, _i32, _i32, P(ChymPlanEntry)]
    lib.chym_plan_autotune_workspace_size.argtypes = [_i32, _i32, _i32, _i32, P(ctypes.c_size_t)]
    lib.chym_plan_autotune.argtypes = [_i32, _i32, _i32, _i32, _i32, _i32, _vp, ctypes.c_size_t, P(ChymPlanEntry),
                                       P(ChymPlanEntry), _i32, P(_i32), _vp]
    lib.chym_split3_bf16.argtypes = [_vp, ctypes.c_int64, _vp, _vp, _vp, _vp]
    lib.chym_j_bytes.argtypes = [_i32, _i32, P(ctypes.c_size_t)]
    lib.chym_quantize_fp8.argtypes = [_i32, _vp, _vp, _vp]
    lib.chym_plan_save.argtypes = [ctypes.c_char_p]
    lib.chym_plan_load.argtypes = [ctypes.c_char_p]
    for f in ("chym_plan_set", "chym_plan_get", "chym_plan_autotune_workspace_size", "chym_plan_autotune",
              "chym_split3_bf16", "chym_plan_save", "chym_plan_load", "chym_j_bytes", "chym_quantize_fp8"):
        getattr(lib, f).restype = ctypes.c_int


def _load_learned(lib):
    P = ctypes.POINTER
    lib.chym_sign_words.argtypes = [_i32, _i32, _i32, _vp, _vp, _vp]
    lib.chym_features.argtypes = [_i32, _i32, _i32, _vp, _i32, _vp, _vp, _vp, _i32, _vp]
    lib.chym_mlp_scratch_floats.argtypes = [_i32, P(ctypes.c_size_t)]
    lib.chym_mlp_forward.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.chym_mlp_backward.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    f = ctypes.c_float
    lib.chym_mlp_adam.argtypes = [_vp, _vp, _vp, _vp, _vp, f, f, f, f, _i32, _vp]
    lib.chym_to_bf16.argtypes = [_vp, _vp, _i32, _vp]
    lib.chym_feature_standardize.argtypes = [_i32, _i32, _vp, _vp, _vp]
    lib.chym_select_top.argtypes = [_i32, _i32, _i32, _vp, _vp, _vp]
    lib.chym_gather_replicas.argtypes = [_i32, _i32, _i32, _vp, _vp, _i32, _vp, _vp, _vp, _vp]
    for name in ("chym_sign_words", "chym_features", "chym_mlp_scratch_floats", "chym_mlp_forward",
                 "chym_mlp_backward", "chym_mlp_adam", "chym_to_bf16", "chym_feature_standardize",
                 "chym_select_top", "chym_gather_replicas"):
        getattr(lib, name).restype = ctypes.c_int
