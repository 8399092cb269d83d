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

HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=on",
             "-Wshadow",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Rpass-analysis=kernel-resource-usage"]
# Per compilation unit: the per-lane kernels keep loop-invariant values out
# of registers (hoisting them costs registers and spills there); the
# cooperative kernel's step loop keeps its constants in registers.
UNITS = [("chemgpu.hip", ["-mllvm", "-disable-machine-licm"]),
         ("coop.hip", [])]


def mech_files():
    return sorted(glob.glob(os.path.join(PKG, "mech", "*.mech")))


def build(verbose: bool = False) -> str:
    from . import codegen
    infos = codegen.generate(mech_files(), GEN)
    os.makedirs(BUILD_DIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    procs, objs, log = [], [], []
    for name, extra in UNITS:
        obj = os.path.join(BUILD_DIR, name.replace(".hip", ".o"))
        cmd = [HIPCC] + HIP_FLAGS + extra + inc + ["-c", os.path.join(CSRC, name), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                            text=True)))
        objs.append(obj)
    failed = False
    for cmd, pr in procs:
        _, err = pr.communicate()
        log.append(" ".join(cmd) + "\n" + err)
        if pr.returncode != 0:
            sys.stderr.write(err[-20000:])
            failed = True
    with open(os.path.join(BUILD_DIR, "resource_usage.txt"), "w") as f:
        f.write("\n".join(log))
    if failed:
        raise RuntimeError("hipcc failed building libchemgpu.so")
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", LIB + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stderr[-20000:])
        raise RuntimeError("linking libchemgpu.so failed")
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        print("built", LIB, "mechanisms:", [i["tag"] for i in infos])
    return LIB


if __name__ == "__main__":
    build(verbose=True)
