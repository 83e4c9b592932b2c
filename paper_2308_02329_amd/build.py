"""Build libchym.so in-tree for gfx950 with hipcc.

    python -m paper_2308_02329_amd.build [-j JOBS]

Each .hip source under csrc/ is compiled to an object in _build/ (in
parallel), then linked into paper_2308_02329_amd/libchym.so.  Every call
recompiles: this is the build check, not a cache.  --sanitize builds
libchym_san.so instead, its host code instrumented with AddressSanitizer and
UndefinedBehaviorSanitizer; _lib loads it when CHYM_SANITIZED_LIBS=1 (run
the CPU tests with the clang ASan runtime preloaded).
"""
from __future__ import annotations

import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libchym.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

# -packed-fp32-ops: no packed FP32 VALU instructions are generated.
# -ffp-contract=off: only the multiply-adds written as fmaf() are fused.
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


# host-side AddressSanitizer and UndefinedBehaviorSanitizer for a CPU check of
# the argument validation and bookkeeping (device code is built as usual):
# every -fsanitize= goes to the host pass only
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
SAN_BUILD = os.path.join(PKG, "_build_san")
SAN_LIB = os.path.join(PKG, "libchym_san.so")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str, sanitize: bool = False) -> tuple[str, str]:
    obj = os.path.join(SAN_BUILD if sanitize else BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC, *CFLAGS, *(SAN_FLAGS if sanitize else []), "-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{p.stderr}")
    return obj, p.stderr


def build(jobs: int | None = None, verbose: bool = False, sanitize: bool = False) -> str:
    """Compile every source and link the library (libchym_san.so with the
    host-side sanitizers when sanitize is set)."""
    os.makedirs(SAN_BUILD if sanitize else BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda src: _compile(src, sanitize), srcs))
    objs = [o for o, _ in results]
    if verbose:
        for _, err in results:
            err = "\n".join(l for l in err.splitlines() if "packed-fp32-ops" not in l and l.strip())
            if err:
                print(err, file=sys.stderr)
    lib = SAN_LIB if sanitize else LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *(SAN_FLAGS if sanitize else []), "-o", tmp, *objs]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"link failed:\n{p.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", "--jobs", type=int, default=None)
    ap.add_argument("-v", "--verbose", action="store_true")
    ap.add_argument("--sanitize", action="store_true",
                    help="build libchym_san.so with host-side AddressSanitizer and UndefinedBehaviorSanitizer")
    args = ap.parse_args()
    print(build(args.jobs, args.verbose, args.sanitize))
