"""Throughput of one flow step of the per-cell chemistry path on one MI355X:
plain FP64 vs surrogate+fallback.

Default workload: the 256^3 evaluation field (16,777,216 cells of the seeded
9-species / 21-reaction H/O/N mechanism; 90 % states of held-out
stoichiometric H2/O2/N2 ignition trajectories in smooth 3-D blobs, 10 %
reacting-front states, cold and hot, outside the surrogate's training hull),
dt = 1e-7 s, rtol 1e-8, atol 1e-10.  Set-up, untimed: training pairs from the
FP64 integrator (4096 cells integrated through ignition), the surrogate
trained on the GPU by its own kernels, trust thresholds chosen on held-out
trajectories, the field built on the GPU.  Timed, each step from the same
pristine field (a device-to-device restore before every step, outside the
HIP-event interval):

* plain FP64: every cell advanced by dt with the LSRK4(3)5 two-register
  scheme and WRMS control (persistent compacting kernel, cooperative tail),
  the batched call captured in one HIP graph;
* surrogate+fallback: features, BF16-MFMA network and FP64 trust test for
  every cell; trusted cells take the network's increment, the others are
  integrated by the FP64 path in the same call.

`value` is the surrogate+fallback rate in cells/s (cells over the mean
HIP-event time of the step on the launch stream); the plain FP64 rate, the
speedup, the fallback fraction and the trusted cells' error against FP64 sit
beside it.  `roofline` is the surrogate+fallback step's dominant kernel,
`plain_fp64.roofline` the plain step's.  The 1024 x 1024 reacting-front field
is measured as well (`front`).  `--workload` selects another field as the
headline instead (front, AMR hierarchy, stress fields, divergence fields).

Prints one JSON line.  --gpus N with N > 1 is refused: the path runs on one
GPU per process (cells are independent; sharding them over GPUs is described
in the design notes, not built).
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "chem-integrated cells/s per flow step: plain FP64 vs surrogate+fallback"
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_BF16_MFMA_TFLOPS = 2500.0
# algorithmic flops of one surrogate evaluation: 2 (12*128 + 128*128 + 128*128 + 128*10)
SURROGATE_FLOPS_PER_CELL = 2 * (12 * 128 + 2 * 128 * 128 + 128 * 10)


def log(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--scheme", default="lsrk", choices=["lsrk", "rkf45", "ros4"],
                    help="lsrk: the paper's two-register LSRK4(3)5; rkf45: the full-storage "
                         "Runge-Kutta-Fehlberg 4(5) comparison scheme; ros4: the implicit "
                         "(Rosenbrock) comparator (fields other than the surrogate field)")
    ap.add_argument("--tail", type=int, default=0,
                    help="steps after which a cell moves to the cooperative kernel "
                         "(0 = default, < 0 = never)")
    ap.add_argument("--tail-cap", type=int, default=0,
                    help="most handed-over cells per CU the cooperative kernel takes "
                         "(0 = default, < 0 = no limit)")
    ap.add_argument("--pool-order", type=int, default=0,
                    help="deal cells expected to be slow over the first claims (1), group "
                         "by NASA-7 range (2), group by range and step the cells below the "
                         "switch after the resumed ones (3), keep the pool order (-1), or the "
                         "tuned choice (0)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--workload", default="surrogate256",
                    choices=["surrogate256", "front", "front_hot_tiled", "amr", "stress9",
                             "stress32", "cells", "diverge_a1", "diverge_a01"])
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2506_02602_amd",
                                                         "tuning_gfx950.json"),
                    help="autotuner cache (JSON, keyed by mechanism hash, size bucket, GPU "
                         "architecture); a hit skips the sweep; 'none' = always sweep")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner (block/chunk/hand-off from the library defaults)")
    ap.add_argument("--no-front", action="store_true",
                    help="with the surrogate field as headline, skip the front-field leg")
    ap.add_argument("--surrogate-epochs", type=int, default=12)
    ap.add_argument("--surrogate-file", default="",
                    help="if the file exists, load the trained surrogate and its trust "
                         "thresholds from it (and FILE.trust.json) instead of training; "
                         "otherwise train and save there (for profiling runs)")
    return ap.parse_args()


# HBM bytes per launch of the dominant kernels, from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE) of this bench, each scaled by what the counter
# reads for the restore copy of known size in the same run (12 rows x 8 B per
# cell of the field: FETCH_SIZE reports 0.500 of it, WRITE_SIZE 1.000).  For
# the per-lane kernel a launch is the flow step's two launches (the persistent
# kernel and the resumption of the tail list), as for its HIP-event time.
# Keyed by a digest of the kernel sources the counters were taken on; any
# change nulls it (profiles/surrogate_mech9_256cubed.md,
# profiles/hbm_counters_lsrk_mech9_front1024_stress.md).
_COUNTED = "6d92838f03263d5b"
TRAFFIC = {
    "surrogate256_plain": (_COUNTED, {"lsrk_persistent": 3.7069e+09}),
    "surrogate256_fallback": (_COUNTED, {"lsrk_persistent": 6.8932e+08}),
    "surrogate256_inference": (_COUNTED, {"surr_infer": 2.9144e+09}),
    "front": (_COUNTED, {"lsrk_coop": 1.0697e+07}),
    "stress9": (_COUNTED, {"lsrk_persistent": 3.1985e+09}),
}


def kernel_digest():
    import glob
    import hashlib
    pkg = os.path.join(ROOT, "paper_2506_02602_amd")
    files = sorted(glob.glob(os.path.join(pkg, "csrc", "*.hip")) +
                   glob.glob(os.path.join(pkg, "csrc", "*.h")))
    files += [os.path.join(pkg, "codegen.py"), os.path.join(pkg, "build.py")]
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic(workload, kernel):
    rec = TRAFFIC.get(workload)
    if not rec or rec[0] != kernel_digest():
        return None
    return rec[1].get(kernel)


# Operations per launch of the dominant kernels by hardware counter, from
# rocprofv3 --pmc runs of this bench: FP64 = 64 lanes x (2 FMA + ADD + MUL +
# TRANS) per wave instruction of SQ_INSTS_VALU_{FMA,ADD,MUL,TRANS}_F64 (so
# masked lanes count too); BF16 MFMA = 512 x SQ_INSTS_VALU_MFMA_MOPS_BF16.
# Keyed like TRAFFIC; any kernel change nulls it.
COUNTER_FLOPS = {
    "surrogate256_plain": (_COUNTED, {"lsrk_persistent": 3.4513e+11}),
    "surrogate256_fallback": (_COUNTED, {"lsrk_persistent": 1.9865e+11}),
    "surrogate256_inference": (_COUNTED, {"surr_infer": 1.3057e+12}),
    "front": (_COUNTED, {"lsrk_coop": 2.4618e+10}),
    "stress9": (_COUNTED, {"lsrk_persistent": 1.1582e+12}),
}


def with_counters(roof, workload):
    """The roofline record with the measured HBM traffic and the executed
    (counter) operation rate beside the algorithmic one, where figures taken
    on the current kernels exist; null otherwise."""
    roof["traffic"] = traffic(workload, roof["kernel"])
    rec = COUNTER_FLOPS.get(workload)
    ops = rec[1].get(roof["kernel"]) if rec and rec[0] == kernel_digest() else None
    if ops is None:
        roof["counter_achieved"] = roof["counter_frac"] = None
    else:
        ach = ops / (roof["launch_ms"] * 1e-3) / 1e12
        roof["counter_achieved"] = ach
        roof["counter_frac"] = ach / roof["peak"]
    return roof


WORKLOADS = {
    "surrogate256": "256^3 = 16,777,216 cells: 90% states of held-out stoichiometric H2/O2/N2 "
                    "ignition trajectories in smooth 3-D blobs, 10% reacting-front states (cold "
                    "300 K / 1 atm and hot 1500-3000 K / 5-30 atm) outside the training hull; "
                    "seeded 9-species 21-reaction H/O/N mechanism; dt 1e-7 s, rtol 1e-8, "
                    "atol 1e-10; plain FP64 LSRK vs 12-128-128-128-10 SiLU MLP (BF16 MFMA) with "
                    "FP64 trust test and FP64 fallback",
    "front": "reacting front 1024x1024 (1,048,576 cells), 2% hot band 1500-3000 K / 5-30 atm, "
             "rest 300 K / 1 atm; seeded 9-species 21-reaction H/O/N mechanism; dt 1e-7 s, "
             "rtol 1e-8, atol 1e-10; plain FP64 LSRK with active-cell compaction",
    "front_hot_tiled": "the front field's 21,008 hot cells tiled x48 (1,008,384 stiff cells): "
                       "saturated-throughput probe, same mechanism and tolerances",
    "amr": "3-level AMR hierarchy, ratio 2, 16/32/48 boxes with edges from {16,32,48,64}^3, "
           "hot ellipsoid in each finest box; dt_l = 1e-7/2^l with 2^l sub-calls; one "
           "graph-captured persistent launch, autotuned",
    "stress9": "256x256x64 cells (4,194,304), T ~ U[900,2800] K, p ~ U[1,40] atm i.i.d.; "
               "9-species mechanism",
    "stress32": "256x256x64 cells (4,194,304), T ~ U[900,2800] K, p ~ U[1,40] atm i.i.d.; "
                "seeded 32-species 150-reaction C/H/O/N mechanism",
    "cells": "4096 independent cells, T ~ U[1000,1600] K, 1 atm, stoichiometric H2/O2/N2",
    "diverge_a1": "thread-coherence field: 16x256x16 = 65,536 cells, T(y) of the paper's Eq. 27-28 with "
                  "alpha = 1.0 (T_low 1000 K, T_high 1600 K), H2:O2:N2 = 1:2:7, 1 atm; 100 calls of "
                  "dt = 1e-5 s in one batched launch (one flow step = the 100 calls)",
    "diverge_a01": "thread-divergence field: as diverge_a1 with alpha = 0.1 (T from 515 to 2068 K in "
                   "40 oscillations along y); 100 calls of dt = 1e-5 s in one batched launch",
}


def load_workload(name):
    """Returns (mechanism path, list of boxes as dicts of numpy state/dt/n_sub)."""
    from paper_2506_02602_amd import workloads as wl
    if name == "stress32":
        path = wl.mech_file("mech32")
    else:
        path = wl.mech_file("mech9")
    if name == "front":
        s, _ = wl.front_2d(path)
        return path, [dict(state=s, dt=wl.DT_FLOW, n_sub=1)]
    if name == "front_hot_tiled":
        s, hot = wl.front_2d(path)
        return path, [dict(state=np.ascontiguousarray(np.tile(s[:, hot], (1, 48))),
                           dt=wl.DT_FLOW, n_sub=1)]
    if name == "amr":
        return path, [dict(state=b["state"], dt=b["dt"], n_sub=b["n_sub"], level=b["level"])
                      for b in wl.amr_hierarchy(path)]
    if name in ("diverge_a1", "diverge_a01"):
        alpha = 1.0 if name == "diverge_a1" else 0.1
        return path, [dict(state=wl.diverge_box(path, alpha), dt=wl.DIVERGE_DT,
                           n_sub=wl.DIVERGE_CALLS)]
    if name in ("stress9", "stress32"):
        return path, [dict(state=wl.stress_3d(path), dt=wl.DT_FLOW, n_sub=1)]
    return path, [dict(state=wl.cells_uniform(path), dt=wl.DT_FLOW, n_sub=1)]


# ------------------------------------------------------------ host / oracle
def host_info():
    """lscpu model and core counts of this host, and the CPUs this process may use."""
    info = {"model": None, "sockets": None, "cores_per_socket": None, "threads_per_core": None}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k == "Model name":
                info["model"] = v
            elif k == "Socket(s)":
                info["sockets"] = int(v)
            elif k == "Core(s) per socket":
                info["cores_per_socket"] = int(v)
            elif k == "Thread(s) per core":
                info["threads_per_core"] = int(v)
            elif k == "CPU(s)":
                info["logical_cpus"] = int(v)
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    if info["sockets"] and info["cores_per_socket"]:
        info["physical_cores"] = info["sockets"] * info["cores_per_socket"]
    info["cpus_allowed"] = len(os.sched_getaffinity(0))
    info["omp_num_threads_env"] = os.environ.get("OMP_NUM_THREADS")
    return info


def oracle_threads(host, asked):
    """All physical cores this process may use: the CPUs it is allowed to run
    on, at most one per physical core, at most OMP_NUM_THREADS (the host's
    share for one GPU) when that is set."""
    if asked:
        return asked
    n = host["cpus_allowed"]
    if host.get("physical_cores"):
        n = min(n, host["physical_cores"])
    env = host.get("omp_num_threads_env")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def native_oracle():
    """The oracle built for this host (-O3 -march=native, no FP contraction)
    in a temporary directory; falls back to the portable build."""
    import oracle
    try:
        oracle.use_native_build(tempfile.mkdtemp(prefix="chemgpu_oracle_"))
        return "gcc -O3 -march=native -ffp-contract=off -fno-fast-math -fopenmp"
    except (OSError, subprocess.CalledProcessError, RuntimeError) as e:
        log(f"native oracle build failed ({e}); using the portable build")
        return "gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp (portable build)"


def time_oracle(om, state, dt, n_sub, threads):
    s = np.array(state)
    t0 = time.perf_counter()
    for _ in range(n_sub):
        om.integrate(s, dt, nthreads=threads)
    return time.perf_counter() - t0


def cpu_baseline_strata(path, strata, threads, build, host, one_thread_frac=0.125):
    """The oracle on a stratified sample of a field: strata is a list of
    (name, cells in the field, sampled states [N+3, k], dt, n_sub).  Each
    stratum's sample is timed on `threads` threads and its per-cell time
    weighted back to the whole field; a fixed fraction of every sample is
    timed again on one thread."""
    import oracle
    om = oracle.Mech(path)
    t_all = t_one = 0.0
    total = sampled = 0
    parts = []
    for name, n_field, st, dt, n_sub in strata:
        k = st.shape[1]
        if k == 0:
            continue
        el = time_oracle(om, st, dt, n_sub, threads)
        k1 = max(1, int(k * one_thread_frac))
        el1 = time_oracle(om, st[:, :k1], dt, n_sub, 1)
        t_all += el / k * n_field
        t_one += el1 / k1 * n_field
        total += n_field
        sampled += k
        parts.append(f"{name}: {k} of {n_field} cells, {el:.2f} s on {threads} threads, "
                     f"{k1} cells {el1:.2f} s on 1 thread")
    return {"value": total / t_all, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "value_1_thread": total / t_one,
            "per_core": total / t_all / threads,
            "sample": "stratified sample of the same field, every sampled cell one flow step "
                      "(with its sub-calls); per-stratum time per cell weighted back to the "
                      "whole field (an extrapolation): " + "; ".join(parts),
            "oracle_build": build, "host": host}


# ------------------------------------------------------------- FP64 boxes
def dominant_fp64(kt, total_steps, coop_steps, flops_per_step):
    """The longer of the per-lane kernel (with its resumption launch) and the
    cooperative kernel, with its algorithmic FP64 rate: its RK steps (the
    cooperative kernel counts the steps it takes, chem_tail_stats; the
    per-lane launches take the rest) x flops per step over its HIP-event
    duration."""
    pers_ms = kt["persistent"] + kt["resume"]
    if kt["coop"] > pers_ms:
        dom, dom_ms, dom_steps = "lsrk_coop", kt["coop"], coop_steps
    else:
        dom, dom_ms, dom_steps = "lsrk_persistent", pers_ms, total_steps - coop_steps
    ach = dom_steps * flops_per_step / (dom_ms * 1e-3) / 1e12
    return {"bound": "alu", "kernel": dom, "achieved": ach, "peak": PEAK_FP64_VECTOR_TFLOPS,
            "unit": "TFLOP/s", "frac": ach / PEAK_FP64_VECTOR_TFLOPS, "launch_ms": dom_ms,
            "rk_steps_per_launch": dom_steps}


def timed_kernels(cg, mech, run, reps):
    """Per-kernel HIP-event durations (means over reps calls of run()) and the
    cooperative kernel's step count of the last call."""
    cg.chem_set_kernel_timing(mech, True)
    recs, tail = [], None
    try:
        for _ in range(reps):
            run()
            recs.append(cg.chem_kernel_times(mech))
            tail = cg.chem_tail_stats(mech)
    finally:
        cg.chem_set_kernel_timing(mech, False)
    return {k: float(np.mean([r[k] for r in recs])) for k in recs[0]}, tail


def measure_boxes(args, workload, hboxes=None, path=None, steps=None):
    """One flow step of a field given as boxes, captured in one graph; the
    flow step's HIP-event time, the dominant kernel's FP64 roofline, per-cell
    step counts.  Returns a dict."""
    import torch
    from paper_2506_02602_amd import chemgpu, codegen, workloads as wl
    if hboxes is None:
        path, hboxes = load_workload(workload)
    K = steps or args.steps
    n = int(sum(b["state"].shape[1] for b in hboxes))
    dev = torch.device("cuda:0")
    boxes, pristine = [], []
    for b in hboxes:
        st = b["state"] if torch.is_tensor(b["state"]) else torch.from_numpy(b["state"]).to(dev)
        nb = st.shape[1]
        pristine.append(st.clone())
        boxes.append(dict(state=st, dt=b["dt"], n_sub=b.get("n_sub", 1), level=b.get("level", 0),
                          status=torch.zeros(nb, dtype=torch.int32, device=dev),
                          counts=torch.zeros(2 * nb, dtype=torch.int32, device=dev)))
    mech = chemgpu.chem_mech_load(path, reserve=n)
    base = chemgpu.make_opts(rtol=wl.RTOL, atol=wl.ATOL, chunk_steps=args.chunk,
                             block_size=args.block, tail_steps=args.tail, scheme=args.scheme,
                             tail_cap=args.tail_cap, pool_order=args.pool_order)
    stream = torch.cuda.current_stream()

    def restore():
        for b, p in zip(boxes, pristine):
            b["state"].copy_(p)

    tuned = None
    log(f"{workload}: {n} cells in {len(boxes)} boxes")
    if not args.no_autotune and not (args.chunk or args.block):
        cache = None if args.tune_cache == "none" else args.tune_cache
        tb = chemgpu.chem_autotune(mech, boxes, base, reps=3 if n <= 2_000_000 else 1,
                                   cache_path=cache)
        tuned = {"block_size": tb.block_size, "chunk_steps": tb.chunk_steps,
                 "tail_steps": tb.tail_steps, "tail_cap": tb.tail_cap,
                 "pool_order": tb.pool_order}
    log(f"{workload}: launch {tuned}; untimed pass with per-cell counters")
    restore()
    chemgpu.chem_integrate_batched(mech, boxes, base)
    torch.cuda.synchronize()
    st = np.concatenate([b["status"].cpu().numpy() for b in boxes])
    cn = np.concatenate([b["counts"].cpu().numpy().reshape(2, -1) for b in boxes], axis=1)
    total_steps = int(cn.sum())
    flops_per_step = codegen.step_flops(codegen.parse(path), args.scheme)

    tboxes = [dict(b, status=None, counts=None) for b in boxes]
    graph = chemgpu.chem_graph_capture_batched(mech, tboxes, base)
    for _ in range(max(args.warmup, 1)):
        restore()
        graph.launch()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(K)]
    log(f"{workload}: timing {K} steps")
    t0 = time.perf_counter()
    for k in range(K):
        restore()
        ev[k][0].record(stream)
        graph.launch(stream)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    graph.close()
    kern_all = np.array([a.elapsed_time(b) for a, b in ev])
    kern_ms = float(np.mean(kern_all))

    # the dominant kernel, timed live: the same flow step as plain calls with
    # the library's per-kernel timing (HIP events around each launch, on the
    # launch streams)
    def one():
        restore()
        chemgpu.chem_integrate_batched(mech, tboxes, base)
    kt, tstats = timed_kernels(chemgpu, mech, one, max(3, min(K, 10)))
    roof = dominant_fp64(kt, total_steps, tstats["cooperative_steps"], flops_per_step)
    if args.scheme == "lsrk":
        with_counters(roof, workload)
    else:
        roof["traffic"] = roof["counter_achieved"] = roof["counter_frac"] = None
    achieved = total_steps * flops_per_step / (kern_ms * 1e-3) / 1e12
    nv = mech.n_species + 1
    out = {
        "cells": n, "boxes": len(boxes), "scheme": args.scheme,
        "value": n / (kern_ms * 1e-3),
        "ms_per_step": kern_ms,
        "kernel_ms_p10_p50_p90": [float(np.percentile(kern_all, q)) for q in (10, 50, 90)],
        "wall_ms_per_step_incl_restore": elapsed * 1e3 / K,
        "autotuned": tuned,
        "roofline": roof,
        "roofline_flow_step": {"bound": "alu", "achieved": achieved,
                               "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                               "frac": achieved / PEAK_FP64_VECTOR_TFLOPS},
        "kernel_times_ms": kt,
        "tail_list": tstats,
        # per flow step: read (T, Y, rho, h), write (T, Y, h) of every cell
        "hbm_algorithmic_bytes": n * 8 * ((nv + 2) + (nv + 1)),
        "steps_per_flow_step": {"total_rk_steps": total_steps, "rejected": int(cn[1].sum()),
                                "max_per_cell": int(cn.sum(axis=0).max()),
                                "status_nonzero": int((st != 0).sum())},
        "flops_per_rk_step": flops_per_step,
    }
    sub_calls = int(sum(b["state"].shape[1] * b.get("n_sub", 1) for b in hboxes))
    if sub_calls != n:
        out["cell_subcalls_per_s"] = sub_calls / (kern_ms * 1e-3)
    mech.close()
    return out


def cpu_baseline_boxes(hboxes, path, threads, build, host, target_s=10.0):
    """The oracle on a bounded sample of a field given as boxes: cells drawn
    uniformly (seed 123) from the concatenated boxes, each integrated over its
    box's sub-calls, in chunks of 4096 until about target_s seconds."""
    import oracle
    om = oracle.Mech(path)
    sizes = np.array([b["state"].shape[1] for b in hboxes])
    n = int(sizes.sum())
    rng = np.random.Generator(np.random.PCG64(123))
    pick = rng.permutation(n)[:262144]
    starts = np.concatenate([[0], np.cumsum(sizes)])
    box_of = np.searchsorted(starts, pick, side="right") - 1

    def run(cells, nthreads, budget):
        done, el, t0 = 0, 0.0, time.perf_counter()
        while el < budget:
            for c0 in range(0, len(pick), cells):
                sel, bsel = pick[c0:c0 + cells], box_of[c0:c0 + cells]
                for bi in np.unique(bsel):
                    b = hboxes[bi]
                    s = np.ascontiguousarray(b["state"][:, sel[bsel == bi] - starts[bi]])
                    for _ in range(b.get("n_sub", 1)):
                        om.integrate(s, b["dt"], nthreads=nthreads)
                done += len(sel)
                el = time.perf_counter() - t0
                if el >= budget:
                    break
        return done, el
    done, el = run(4096, threads, target_s)
    done1, el1 = run(256, 1, target_s / 4)
    return {"value": done / el, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "value_1_thread": done1 / el1, "per_core": done / el / threads,
            "sample": f"{done} cells drawn uniformly (seed 123) from the same workload, one flow "
                      f"step each (with the box's sub-calls), in chunks of 4096: {el:.1f} s wall "
                      f"on {threads} host threads; {done1} cells in {el1:.1f} s on 1 thread",
            "oracle_build": build, "host": host}


# ------------------------------------------------------- surrogate field
def surrogate_field(args):
    """The 256^3 field: plain FP64 and surrogate+fallback, each timed from the
    pristine field.  Returns (result dict, field strata for the CPU baseline)."""
    import torch
    from paper_2506_02602_amd import chemgpu as cg, codegen, surrogate as sg, workloads as wl
    path = wl.mech_file("mech9")
    m = cg.chem_mech_load(path)
    sfile = args.surrogate_file
    if sfile and os.path.exists(sfile):
        s = cg.surrogate_load(m, sfile)
        with open(sfile + ".trust.json") as f:
            saved = json.load(f)
        trust, tstats, train_rec = tuple(saved["trust"]), saved["validation"], saved["train"]
        log(f"surrogate: loaded from {sfile}")
    else:
        t0 = time.perf_counter()
        ds = sg.build_dataset(m)
        t_data = time.perf_counter() - t0
        n_pairs = int(ds["X"].shape[0])
        log(f"surrogate: {n_pairs} training pairs in {t_data:.1f} s; training")
        s = cg.Surrogate(m, seed=11)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = cg.surrogate_train(s, ds["X"], ds["Y"], epochs=args.surrogate_epochs, batch=4096,
                                  lr=3e-3, seed=2)
        t_train = time.perf_counter() - t0
        train_flops = (3.0 * SURROGATE_FLOPS_PER_CELL * (n_pairs // 4096) * 4096 *
                       args.surrogate_epochs)
        log("surrogate: tuning trust thresholds")
        trust, tstats = sg.tune_trust(s, m, sg.validation_states(ds))
        if trust is None:
            trust = (0.0, 1e-6, 1e-7, 0.05)
        train_rec = {"pairs": n_pairs, "epochs": args.surrogate_epochs, "batch": 4096,
                     "first_loss": float(loss[0]), "final_loss": float(loss[-1]),
                     "data_s": t_data, "train_s": t_train,
                     "achieved_tflops": train_flops / t_train / 1e12}
        if sfile:
            cg.surrogate_save(s, sfile)
            with open(sfile + ".trust.json", "w") as f:
                json.dump({"trust": list(trust), "validation": tstats, "train": train_rec}, f)
        del ds
        torch.cuda.empty_cache()
    log("surrogate: building the 256^3 evaluation field")
    field, out_mask = sg.inference_field(m)
    n = field.shape[1]
    cg.chem_workspace_reserve(m, n)
    cg.surrogate_reserve(s, n)
    work = torch.empty_like(field)
    base = cg.make_opts(rtol=wl.RTOL, atol=wl.ATOL)
    cache = None if args.tune_cache == "none" else args.tune_cache
    opts = cg.chem_autotune(m, [dict(state=field, dt=wl.DT_FLOW)], base, reps=1, cache_path=cache)
    launch = {"block_size": opts.block_size, "chunk_steps": opts.chunk_steps,
              "tail_steps": opts.tail_steps, "tail_cap": opts.tail_cap,
              "pool_order": opts.pool_order}
    log(f"surrogate: launch {launch}")
    # the fallback's launch, tuned on whole surrogate steps over this field
    fb_opts = cg.surrogate_autotune(s, m, field, wl.DT_FLOW, trust, base, reps=1, cache_path=cache)
    launch_fb = {"block_size": fb_opts.block_size, "chunk_steps": fb_opts.chunk_steps,
                 "tail_steps": fb_opts.tail_steps, "tail_cap": fb_opts.tail_cap,
                 "pool_order": fb_opts.pool_order}
    log(f"surrogate: fallback launch {launch_fb}")
    stream = torch.cuda.current_stream()
    K = args.steps
    flops_per_step = codegen.step_flops(codegen.parse(path), "lsrk")

    def timed(fn, k=K):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(k)]
        for _ in range(max(args.warmup, 1)):
            work.copy_(field)
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for a, b in ev:
            work.copy_(field)
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / k
        ms = np.array([a.elapsed_time(b) for a, b in ev])
        return float(ms.mean()), ms, wall

    # plain FP64: the batched call captured in one graph (as the other fields)
    ref = field.clone()
    stc = torch.zeros(n, dtype=torch.int32, device="cuda")
    cnc = torch.zeros(2 * n, dtype=torch.int32, device="cuda")
    cg.chem_integrate(m, ref, wl.DT_FLOW, opts, status=stc, counts=cnc)
    torch.cuda.synchronize()
    plain_counts = cnc.view(2, n).cpu().numpy()
    graph = cg.chem_graph_capture_batched(m, [dict(state=work, dt=wl.DT_FLOW)], opts)
    log(f"surrogate field: timing {K} plain FP64 steps")
    k_plain, k_plain_all, w_plain = timed(lambda: graph.launch(stream))
    graph.close()
    def plain_once():
        work.copy_(field)
        cg.chem_integrate(m, work, wl.DT_FLOW, opts)
    kt_plain, tail_plain = timed_kernels(cg, m, plain_once, 3)
    per_cell = plain_counts.sum(axis=0)
    roof_plain = dominant_fp64(kt_plain, int(per_cell.sum()), tail_plain["cooperative_steps"],
                               flops_per_step)
    with_counters(roof_plain, "surrogate256_plain")
    plain_ach = int(per_cell.sum()) * flops_per_step / (k_plain * 1e-3) / 1e12

    # surrogate + fallback: the step captured in one graph (as the plain
    # leg), and the same step enqueued call by call
    log(f"surrogate field: timing {K} surrogate+fallback steps")
    sgraph = cg.surrogate_graph_capture(s, m, work, wl.DT_FLOW, trust, fb_opts)
    k_surr, k_surr_all, w_surr = timed(lambda: sgraph.launch(stream))
    sgraph.close()
    k_surr_eager, _, _ = timed(
        lambda: cg.surrogate_infer(s, m, work, wl.DT_FLOW, trust, fallback=True, opts=fb_opts))
    k_inf, k_inf_all, _ = timed(
        lambda: cg.surrogate_infer(s, m, work, wl.DT_FLOW, trust, fallback=False))
    tc = torch.zeros(n, dtype=torch.int32, device="cuda")
    fst = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    fcn = torch.zeros(2 * n, dtype=torch.int32, device="cuda")
    fb_count = [0]

    def surr_once():
        work.copy_(field)
        fb_count[0] = cg.surrogate_infer(s, m, work, wl.DT_FLOW, trust, fallback=True,
                                         opts=fb_opts, trust_code=tc, status=fst, counts=fcn,
                                         want_count=True)
    kt_fb, tail_fb = timed_kernels(cg, m, surr_once, 3)
    n_fb = fb_count[0]
    # the timed FP64 run is the one over the cells outside the hull (code 1)
    tcn = tc.cpu().numpy()
    hull = tcn == 1
    fb_steps = fcn.view(2, n).cpu().numpy().sum(axis=0)
    roof_fb = dominant_fp64(kt_fb, int(fb_steps[hull].sum()), tail_fb["cooperative_steps"],
                            flops_per_step)
    with_counters(roof_fb, "surrogate256_fallback")
    inf_ach = SURROGATE_FLOPS_PER_CELL * n / (k_inf * 1e-3) / 1e12
    roof_inf = {"bound": "mfma", "kernel": "surr_infer", "achieved": inf_ach,
                "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": inf_ach / PEAK_BF16_MFMA_TFLOPS, "launch_ms": k_inf,
                "cells_per_launch": n}
    with_counters(roof_inf, "surrogate256_inference")
    # the surrogate step's dominant kernel: the longer of the FP64 fallback's
    # dominant kernel and the network
    dom = roof_fb if roof_fb["launch_ms"] >= k_inf else roof_inf

    # accuracy of the trusted cells against the plain FP64 result
    ok = torch.from_numpy(tcn == 0).cuda()
    eT, eY = sg.errors(work[:, ok], ref[:, ok], m.n_species)
    idx = torch.randperm(int(ok.sum()), device="cuda")[:2000000]
    q = lambda x: float(torch.quantile(x[idx].float(), 0.999))
    fb = ~ok
    fT, fY = sg.errors(work[:, fb], ref[:, fb], m.n_species)
    neg = int((work[1:m.n_species + 1, ok] < 0).sum())
    res = {
        "cells": n,
        "value": n / (k_surr * 1e-3),
        "ms_per_step": k_surr,
        "kernel_ms_p10_p50_p90": [float(np.percentile(k_surr_all, p)) for p in (10, 50, 90)],
        "wall_ms_per_step_incl_restore": 1e3 * w_surr,
        "ms_per_step_eager_calls": k_surr_eager,
        "speedup_vs_plain_fp64": k_plain / k_surr,
        "fallback_fraction": n_fb / n,
        "roofline": dom,
        "roofline_inference": roof_inf,
        "roofline_fallback_fp64": roof_fb,
        "kernel_times_fallback_ms": kt_fb,
        "tail_list_fallback": tail_fb,
        "fallback_rk_steps": {"hull_cells": int(hull.sum()),
                              "hull_rk_steps": int(fb_steps[hull].sum()),
                              "other_fallback_cells": int((tcn > 1).sum()),
                              "other_rk_steps": int(fb_steps[tcn > 1].sum())},
        "ms_inference_only": k_inf,
        "plain_fp64": {
            "cells_per_s": n / (k_plain * 1e-3), "ms_per_step": k_plain,
            "kernel_ms_p10_p50_p90": [float(np.percentile(k_plain_all, p)) for p in (10, 50, 90)],
            "wall_ms_per_step_incl_restore": 1e3 * w_plain,
            "roofline": roof_plain,
            "roofline_flow_step": {"bound": "alu", "achieved": plain_ach,
                                   "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                                   "frac": plain_ach / PEAK_FP64_VECTOR_TFLOPS},
            "kernel_times_ms": kt_plain,
            "tail_list": tail_plain,
            "steps_per_flow_step": {"total_rk_steps": int(per_cell.sum()),
                                    "rejected": int(plain_counts[1].sum()),
                                    "max_per_cell": int(per_cell.max())},
            "flops_per_rk_step": flops_per_step},
        "launch": launch,
        "launch_fallback": launch_fb,
        "trust": {"hull_margin": trust[0], "elem_tol": trust[1], "pos_tol": trust[2],
                  "energy_tol_K": trust[3], "validation": tstats},
        "trusted_error_vs_fp64": {"max_rel_T": float(eT.max()), "p999_rel_T": q(eT),
                                  "max_abs_Y": float(eY.max()), "p999_abs_Y": q(eY),
                                  "negative_Y_entries": neg},
        "fallback_cells_max_diff_vs_plain": {"rel_T": float(fT.max()) if fb.any() else 0.0,
                                             "abs_Y": float(fY.max()) if fb.any() else 0.0},
        "train": train_rec,
    }
    # strata for the CPU baseline: trajectory states, cold and hot front states
    T = field[0]
    strata_masks = [("trajectory states", ~out_mask), ("front states, cold", out_mask & (T < 1000.0)),
                    ("front states, hot", out_mask & (T >= 1000.0))]
    rng = np.random.Generator(np.random.PCG64(321))
    strata = []
    for name, mk in strata_masks:
        idx_all = torch.nonzero(mk).flatten()
        cnt = int(idx_all.numel())
        # the hot cells carry nearly all the oracle's time: all of them (up
        # to 2^19), a tenth of the rest; about 15 s on the host in all
        k = min(cnt, 1 << 19) if "hot" in name else max(1, cnt // 10)
        pick = torch.from_numpy(np.sort(rng.choice(cnt, k, replace=False))).cuda()
        st = field[:, idx_all[pick]].cpu().numpy()
        strata.append((name, cnt, np.ascontiguousarray(st), wl.DT_FLOW, 1))
    del work, ref, field
    s.close()
    m.close()
    torch.cuda.empty_cache()
    return res, strata, path


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the chemistry path runs on one GPU (asked for --gpus {args.gpus}); "
              "the chemistry step needs no cross-GPU exchange, see the design notes",
              file=sys.stderr)
        sys.exit(2)
    import torch  # noqa: F401
    host = host_info()
    threads = oracle_threads(host, args.cpu_threads)
    build = None if args.no_cpu else native_oracle()
    out = {"metric": METRIC, "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "data": "synthetic"}
    if args.workload == "surrogate256":
        res, strata, path = surrogate_field(args)
        out.update({"value": res["value"], "ms_per_step": res["ms_per_step"],
                    "dtype": "f64+bf16",
                    "config": {"workload": WORKLOADS["surrogate256"], "name": "surrogate256",
                               "cells": res["cells"], "path": "surrogate+fallback",
                               "launch": res["launch"]},
                    "roofline": res["roofline"]})
        out["surrogate_fallback"] = {k: v for k, v in res.items()
                                     if k not in ("plain_fp64", "roofline")}
        out["plain_fp64"] = res["plain_fp64"]
        if not args.no_cpu:
            log(f"oracle on {threads} host threads (stratified sample of the 256^3 field)")
            out["cpu_baseline"] = cpu_baseline_strata(path, strata, threads, build, host)
        if not args.no_front:
            log("front field")
            out["front"] = measure_boxes(args, "front")
    else:
        path, hboxes = load_workload(args.workload)
        res = measure_boxes(args, args.workload, hboxes, path)
        out.update({"value": res["value"], "ms_per_step": res["ms_per_step"],
                    "dtype": "f64",
                    "config": {"workload": WORKLOADS[args.workload], "name": args.workload,
                               "cells": res["cells"], "boxes": res["boxes"],
                               "scheme": res["scheme"], "autotuned": res["autotuned"]},
                    "roofline": res["roofline"]})
        out["detail"] = {k: v for k, v in res.items() if k != "roofline"}
        if not args.no_cpu:
            log(f"oracle on {threads} host threads")
            out["cpu_baseline"] = cpu_baseline_boxes(hboxes, path, threads, build, host)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
