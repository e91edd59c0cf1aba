"""Build the gfx950 HIP library ``libpcdn.so`` in-tree with hipcc.

    python -m paper_1306_4080_amd.build
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = [os.path.join(CSRC, f)
           for f in ("pcdn_api.hip", "pcdn_batch.hip", "pcdn_kernels.hip", "pcdn_static.hip")]
HEADERS = [os.path.join(CSRC, "pcdn_device.h"), os.path.join(CSRC, "pcdn_host.h"),
           os.path.join(ROOT, "include", "pcdn.h")]
LIB = os.path.join(HERE, "libpcdn.so")
ARCH = os.environ.get("PCDN_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"),
                 shutil.which("hipcc") or ""):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the PCDN library needs ROCm's hipcc to build")


def command(out: str = LIB) -> list:
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            # keep FP64 rounding close to a plain evaluation of each formula
            "-ffp-contract=off",
            # hardware FP64 atomics for the d^T x scatter
            "-munsafe-fp-atomics",
            # no packed FP32 instructions
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"),
            "-o", out] + SOURCES


STAMP = LIB + ".stamp"


def fingerprint() -> str:
    """SHA-256 of the sources, the headers and the compile command: what the
    library is built from (contents, not modification times, which a copy of
    the tree does not keep)."""
    h = hashlib.sha256()
    h.update(" ".join(command("libpcdn.so")[1:]).replace(ROOT, "").encode())
    for f in SOURCES + HEADERS:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    fp = fingerprint()
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    with open(STAMP, "w") as f:
        f.write(fp + "\n")
    return LIB


def is_stale() -> bool:
    """Whether libpcdn.so is missing or was built from other sources."""
    if not (os.path.exists(LIB) and os.path.exists(STAMP)):
        return True
    with open(STAMP) as f:
        return f.read().strip() != fingerprint()


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
