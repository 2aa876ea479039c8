"""Build libks.so (the gfx950 HIP kernels and the C ABI) in-tree with hipcc.

Each source is compiled to an object in parallel, then linked."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libks.so")
# (source, extra flags): the H.psi files are compiled once per precision
SOURCES = [("ks_hpsi.hip", ["-DKS_HPSI_PART=0"]),
           ("ks_hpsi.hip", ["-DKS_HPSI_PART=1"]),
           ("ks_batch.hip", ["-DKS_HPSI_PART=0"]),
           ("ks_batch.hip", ["-DKS_HPSI_PART=1"]),
           ("ks_kernels.hip", []), ("ks_poisson.hip", []),
           ("ks_observe.hip", []), ("ks_noalloc.hip", []),
           ("ks_api.cpp", [])]
# sources whose text determines the device code of the H.psi path
KERNEL_SOURCES = ["ks_device.h", "ks_internal.h", "ks_hpsi.hip",
                  "ks_batch.hip", "ks_kernels.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd))


def build(verbose: bool = False) -> str:
    """Compile every HIP source for gfx950 into paper_1912_07921_amd/libks.so."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, f"{s}.{i}.o")
            for i, (s, _) in enumerate(SOURCES)]
    cmds = [[HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, s), "-o", o]
            for (s, extra), o in zip(SOURCES, objs)]
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o",
          tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
