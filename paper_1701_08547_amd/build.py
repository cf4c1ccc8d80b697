"""Build the gfx950 library ``libsa.so`` in-tree with hipcc (cross-compiles
without a GPU)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libsa.so")
SOURCES = ["sa_api.hip", "sa_eval.hip", "sa_plan.hip", "sa_mlp.hip", "sa_mlp_api.hip", "sa_corrected.hip",
           "sa_runtime.hip", "sa_gen.hip", "sa_cpi.hip", "sa_product.hip", "sa_probe.hip", "sa_noalloc.hip"]
# gfx950 assembly of the measured kernel families, read by the static
# feature extractor (same device flags as the library)
RUNTIME_ASM = os.path.join(PKG, "sa_runtime_gfx950.s")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # one rounding per binary32 step: no contraction into fused multiply-add
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


# sources the planned scoring kernel is built from: counter figures taken on
# other sources are not reported
PLAIN_KERNEL_SOURCES = ("sa_internal.h", "sa_dev.h", "sa_eval.hip", "sa_plan.hip")


def plain_kernel_digest() -> str:
    import hashlib

    h = hashlib.sha256()
    for name in PLAIN_KERNEL_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    build_runtime_asm(verbose)
    return LIB


def build_runtime_asm(verbose: bool = False) -> str:
    flags = [f for f in HIPCC_FLAGS if f not in ("-fPIC", "-shared")]
    tmp = RUNTIME_ASM + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *flags, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "--cuda-device-only", "-S",
           os.path.join(CSRC, "sa_runtime.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, RUNTIME_ASM)
    return RUNTIME_ASM


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
