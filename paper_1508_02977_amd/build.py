"""Build the HIP library ``libsfdd.so`` in-tree for gfx950.

All sources under ``csrc/`` are compiled by one ``hipcc`` invocation into a
shared library next to this file; the Python binding loads it from there.
The library carries a digest of the sources it was built from
(``sf_build_digest``), and the binding refuses a library whose digest differs
from that of the sources in the tree.
"""
from __future__ import annotations

import glob
import hashlib
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsfdd.so")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # keep hipcc from forming packed FP32 ops (v_pk_add/mul/fma_f32): some of
    # their forms have returned wrong results on this hardware
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in ordinary VGPRs: the factor keeps 13 accumulator
    # chains live and interleaves them; with the accumulator-register form the
    # compiler copied every block in and out around its MFMAs (and, with the
    # interleaved order, runs out of aligned registers)
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def sources() -> list[str]:
    """Every file the library is built from (sorted, repository-relative)."""
    pats = (os.path.join(HERE, "csrc", "*.hip"), os.path.join(HERE, "csrc", "*.h"),
            os.path.join(ROOT, "include", "*.h"))
    return sorted(os.path.relpath(f, ROOT) for pat in pats for f in glob.glob(pat))


def source_digest() -> str:
    """SHA-256 over the names and bytes of :func:`sources`."""
    h = hashlib.sha256()
    for rel in sources():
        h.update(rel.encode() + b"\0")
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
        h.update(b"\0")
    return h.hexdigest()


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm toolchain required to build libsfdd.so)")


def build(verbose: bool = False) -> str:
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *FLAGS, f'-DSFDD_SOURCE_DIGEST="{source_digest()}"', "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(HERE, "csrc"), "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
