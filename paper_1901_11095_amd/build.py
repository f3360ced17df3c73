"""Build libsal.so (gfx950 HIP kernels + C ABI) in-tree with hipcc.

Usage: python -m paper_1901_11095_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libsal.so")
SOURCES = ["sal_api.hip", "sal_kernels.hip", "sal_energy16.hip", "sal_energy_gen.hip", "sal_energy_win.hip", "sal_energy_slide.hip",
           "sal_merge.hip", "sal_net.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 VALU forms stay off (compiler-generated v_pk_*_f32 disabled)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in ordinary VGPRs: the magnitudes are computed from them directly
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wall", "-Wno-unused-result",
    # every symbol resolved at link time (a kernel whose host stub failed to instantiate
    # would otherwise leave an undefined reference in the library)
    "-Wl,-z,defs",
    "-I", INCLUDE, "-I", CSRC,
]


def build(verbose: bool = False, out: str = LIB, extra=()) -> str:
    """Compile every source; always rebuilds.  Returns the library path."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + list(extra) + ["-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    log = "\n".join(l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        if os.path.exists(tmp):
            os.remove(tmp)
        raise RuntimeError("hipcc failed:\n" + log)
    if verbose and log.strip():
        print(log)
    os.replace(tmp, out)
    return out


def is_built() -> bool:
    return os.path.exists(LIB)


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
    print(LIB)
