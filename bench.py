"""Throughput of the per-cell FP64 chemistry integrator on one MI355X.

One step = one flow step of the whole hot path over the 1024 x 1024
reacting-front field (1,048,576 cells of the 9-species / 21-reaction
mechanism, dt = 1e-7 s, rtol 1e-8, atol 1e-10): every cell is advanced by dt
with the LSRK4(3)5 two-register scheme and WRMS control, in the persistent
compacting kernel.  Inputs are resident in HBM; each timed step first
restores the pristine field with a device-to-device copy (inside the timed
region) so every step integrates the same input.

Prints one JSON line.  --gpus N with N > 1 is refused: this build runs on a
single GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "chem-integrated cells/s per flow step: plain FP64 vs surrogate+fallback"
PEAK_FP64_VECTOR_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    return ap.parse_args()


def cpu_baseline(state, path, dt, threads):
    """The oracle, as it stands, on a bounded sample of the same field."""
    import oracle
    om = oracle.Mech(path)
    n = state.shape[1]
    rng = np.random.Generator(np.random.PCG64(123))
    ns = min(n, 262144)
    idx = np.sort(rng.choice(n, ns, replace=False))
    sub = np.ascontiguousarray(state[:, idx])
    t0 = time.perf_counter()
    om.integrate(sub, dt, nthreads=threads)
    el = time.perf_counter() - t0
    return {"value": ns / el, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"{ns} cells drawn uniformly (seed 123) from the same field, one flow step, "
                      f"{el:.2f} s wall on {threads} host threads"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the chemistry step needs no cross-GPU exchange, see the design notes",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2506_02602_amd import chemgpu, codegen, workloads as wl

    path = wl.mech_file("mech9")
    s0, hot = wl.front_2d(path)
    n = s0.shape[1]
    dt = wl.DT_FLOW
    dev = torch.device("cuda:0")
    pristine = torch.from_numpy(s0).to(dev)
    work = torch.empty_like(pristine)
    counts = torch.zeros(2 * n, dtype=torch.int32, device=dev)
    status = torch.zeros(n, dtype=torch.int32, device=dev)
    mech = chemgpu.chem_mech_load(path)
    chemgpu.chem_workspace_reserve(mech, n)
    opts = chemgpu.make_opts(rtol=wl.RTOL, atol=wl.ATOL, chunk_steps=args.chunk,
                             block_size=args.block)
    stream = torch.cuda.current_stream()

    for _ in range(max(args.warmup, 1)):
        work.copy_(pristine)
        chemgpu.chem_integrate(mech, work, dt, opts, status=status, counts=counts)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    cn = counts.cpu().numpy().reshape(2, n)
    total_steps = int(cn.sum())
    m = codegen.parse(path)
    flops_per_launch = total_steps * codegen.step_flops(m)

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        work.copy_(pristine)
        ev[k][0].record(stream)
        chemgpu.chem_integrate(mech, work, dt, opts)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    ms_per_step = elapsed * 1e3 / args.steps
    value = n * args.steps / elapsed
    achieved = flops_per_launch / (kern_ms * 1e-3) / 1e12

    out = {
        "metric": METRIC, "value": value, "unit": "cells/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "reacting front 1024x1024 (1,048,576 cells), 2% hot band "
                               "1500-3000 K / 5-30 atm, rest 300 K / 1 atm; seeded 9-species "
                               "21-reaction H/O/N mechanism; dt 1e-7 s, rtol 1e-8, atol 1e-10; "
                               "plain FP64 LSRK with active-cell compaction",
                   "cells": n, "hot_cells": int(hot.sum()),
                   "chunk_steps": args.chunk, "block_size": args.block},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR_TFLOPS,
                     "traffic": None},
        "kernel_ms": kern_ms,
        "steps_per_flow_step": {"total_rk_steps": total_steps,
                                "rejected": int(cn[1].sum()),
                                "max_per_cell": int(cn.sum(axis=0).max()),
                                "status_nonzero": int((st != 0).sum())},
        "flops_per_rk_step": codegen.step_flops(m),
    }
    if not args.no_cpu:
        threads = args.cpu_threads or min(os.cpu_count() or 1, 16)
        out["cpu_baseline"] = cpu_baseline(s0, path, dt, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
