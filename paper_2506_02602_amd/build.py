"""Build the HIP library for gfx950: generate the unrolled mechanism kernels
from every ``mech/*.mech`` file, then compile ``libchemgpu.so`` in-tree."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
GEN = os.path.join(CSRC, "generated")
LIB = os.path.join(PKG, "libchemgpu.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
BUILD_DIR = os.path.join(ROOT, "_build")

HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=on",
             "-Wshadow",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-mllvm", "-disable-machine-licm",
             "-Rpass-analysis=kernel-resource-usage"]


def mech_files():
    return sorted(glob.glob(os.path.join(PKG, "mech", "*.mech")))


def build(verbose: bool = False) -> str:
    from . import codegen
    infos = codegen.generate(mech_files(), GEN)
    os.makedirs(BUILD_DIR, exist_ok=True)
    src = [os.path.join(CSRC, "chemgpu.hip")]
    cmd = [HIPCC] + HIP_FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC] + src + \
        ["-o", LIB + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    with open(os.path.join(BUILD_DIR, "resource_usage.txt"), "w") as f:
        f.write(" ".join(cmd) + "\n" + res.stderr)
    if res.returncode != 0:
        sys.stderr.write(res.stderr[-20000:])
        raise RuntimeError("hipcc failed building libchemgpu.so")
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        print("built", LIB, "mechanisms:", [i["tag"] for i in infos])
    return LIB


if __name__ == "__main__":
    build(verbose=True)
