"""Throughput of the per-cell FP64 chemistry integrator on one MI355X.

One step = one flow step of the whole hot path over one workload; the
default is the 1024 x 1024 reacting-front field (1,048,576 cells of the
9-species / 21-reaction mechanism, dt = 1e-7 s, rtol 1e-8, atol 1e-10): every
cell is advanced by dt with the LSRK4(3)5 two-register scheme and WRMS
control, in the persistent compacting kernel, launched as one captured HIP
graph.  Inputs are resident in HBM; each timed step first restores the
pristine field with a device-to-device copy (inside the timed region) so
every step integrates the same input.  --workload selects the other fields
(AMR hierarchy, stress fields, the hot-cell throughput probe).

Prints one JSON line.  --gpus N with N > 1 is refused: the integrator runs on
one GPU per process (cells are independent; sharding them over GPUs is
described in the design notes, not built).
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
                         "(Rosenbrock) comparator")
    ap.add_argument("--tail", type=int, default=0,
                    help="steps after which a cell moves to the cooperative kernel "
                         "(0 = default, < 0 = never)")
    ap.add_argument("--tail-cap", type=int, default=0,
                    help="most handed-over cells per CU the cooperative kernel takes "
                         "(0 = default, < 0 = no limit)")
    ap.add_argument("--pool-order", type=int, default=0,
                    help="deal cells expected to be slow over the first claims (1), keep the "
                         "pool order (-1), or the tuned choice (0)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--workload", default="front",
                    choices=["front", "front_hot_tiled", "amr", "stress9", "stress32", "cells",
                             "diverge_a1", "diverge_a01"])
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2506_02602_amd",
                                                         "tuning_gfx950.json"),
                    help="autotuner cache (JSON, keyed by mechanism hash, size bucket, GPU "
                         "architecture); a hit skips the sweep; 'none' = always sweep")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner (block/chunk/hand-off from the library defaults)")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the surrogate+fallback leg on the 256^3 evaluation field")
    ap.add_argument("--surrogate-epochs", type=int, default=12)
    return ap.parse_args()


# HBM bytes of one flow step (persistent + cooperative kernel, the timed
# launches of this bench with the committed tuning), from two rocprofv3
# --pmc runs, FETCH_SIZE then WRITE_SIZE, each scaled by what the counter
# reads for the restore copy of known size in the same run (FETCH_SIZE
# reports 0.5002 of the copied bytes, WRITE_SIZE 1.000).  Keyed by a digest of
# the kernel sources the counters were taken on; any change nulls it.
TRAFFIC = {"front": ("5c9d19c03c3dbae1", 232.9e6,
                     {"lsrk_persistent": 203.20e6, "lsrk_coop": 29.54e6}),
           "stress9": ("5c9d19c03c3dbae1", 3605.3e6,
                       {"lsrk_persistent": 3518.15e6, "lsrk_coop": 0.04e6})}


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


PEAK_BF16_MFMA_TFLOPS = 2500.0
# algorithmic flops of one surrogate evaluation: 2 (12*128 + 128*128 + 128*128 + 128*10)
SURROGATE_FLOPS_PER_CELL = 2 * (12 * 128 + 2 * 128 * 128 + 128 * 10)


def surrogate_leg(args):
    """Config-5 comparison: train the surrogate on FP64 trajectory pairs, tune
    the trust thresholds on held-out trajectories, then time plain FP64 and
    surrogate+fallback on the 256^3 evaluation field (each timed step restores
    the pristine field first) and judge the trusted cells against FP64."""
    import torch
    from paper_2506_02602_amd import chemgpu as cg, surrogate as sg, workloads as wl
    m = cg.chem_mech_load(wl.mech_file("mech9"))
    t0 = time.perf_counter()
    ds = sg.build_dataset(m)
    t_data = time.perf_counter() - t0
    log(f"surrogate: {int(ds['X'].shape[0])} training pairs in {t_data:.1f} s; training")
    n_pairs = int(ds["X"].shape[0])
    s = cg.Surrogate(m, seed=11)
    t0 = time.perf_counter()
    loss = cg.surrogate_train(s, ds["X"], ds["Y"], epochs=args.surrogate_epochs, batch=4096,
                              lr=3e-3, seed=2)
    t_train = time.perf_counter() - t0
    log("surrogate: tuning trust thresholds")
    trust, tstats = sg.tune_trust(s, m, sg.validation_states(ds))
    if trust is None:
        trust = (0.0, 1e-6, 1e-7, 0.05)
    del ds
    torch.cuda.empty_cache()
    log("surrogate: building the 256^3 evaluation field")
    field, out_mask = sg.inference_field(m)
    n = field.shape[1]
    work = torch.empty_like(field)
    # one launch configuration for both paths: the autotuner's choice on the
    # evaluation field itself (the fallback integrates a subset of it)
    base = cg.make_opts(rtol=wl.RTOL, atol=wl.ATOL)
    cache = None if args.tune_cache == "none" else args.tune_cache
    opts = cg.chem_autotune(m, [dict(state=field, dt=wl.DT_FLOW)], base, reps=1, cache_path=cache)
    log(f"surrogate: launch block {opts.block_size} chunk {opts.chunk_steps} "
        f"hand-off {opts.tail_steps}")
    ref = field.clone()
    cg.chem_integrate(m, ref, wl.DT_FLOW, opts)
    stream = torch.cuda.current_stream()
    K = max(1, min(args.steps, 5))

    def timed(fn):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(K)]
        work.copy_(field)
        fn()                                   # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        for a, b in ev:
            work.copy_(field)
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / K, float(np.mean([a.elapsed_time(b) for a, b in ev]))

    t_plain, k_plain = timed(lambda: cg.chem_integrate(m, work, wl.DT_FLOW, opts))
    t_surr, k_surr = timed(lambda: cg.surrogate_infer(s, m, work, wl.DT_FLOW, trust, fallback=True,
                                                      opts=opts))
    t_inf, k_inf = timed(lambda: cg.surrogate_infer(s, m, work, wl.DT_FLOW, trust, fallback=False))
    tc = torch.zeros(n, dtype=torch.int32, device="cuda")
    work.copy_(field)
    n_fb = cg.surrogate_infer(s, m, work, wl.DT_FLOW, trust, fallback=True, trust_code=tc,
                              want_count=True, opts=opts)
    ok = tc == 0
    eT, eY = sg.errors(work[:, ok], ref[:, ok], m.n_species)
    idx = torch.randperm(int(ok.sum()), device="cuda")[:2000000]
    q = lambda x: float(torch.quantile(x[idx].float(), 0.999))
    fb = ~ok
    fT, fY = sg.errors(work[:, fb], ref[:, fb], m.n_species)
    achieved = SURROGATE_FLOPS_PER_CELL * n / (k_inf * 1e-3) / 1e12
    return {
        "workload": "256^3 = 16,777,216 cells: 90% held-out H2/O2/N2 ignition-trajectory states "
                    "in smooth 3-D blobs, 10% reacting-front states outside the training hull; "
                    "dt 1e-7 s; 9-species mechanism",
        "cells": n,
        "plain_fp64_cells_per_s": n / t_plain, "surrogate_fallback_cells_per_s": n / t_surr,
        "speedup": t_plain / t_surr,
        "launch": {"block_size": opts.block_size, "chunk_steps": opts.chunk_steps,
                   "tail_steps": opts.tail_steps},
        "ms_plain": 1e3 * t_plain, "ms_surrogate_fallback": 1e3 * t_surr,
        "ms_inference_only": k_inf,
        "fallback_fraction": n_fb / n,
        "trust": {"hull_margin": trust[0], "elem_tol": trust[1], "pos_tol": trust[2],
                  "energy_tol_K": trust[3], "validation": tstats},
        "trusted_error_vs_fp64": {"max_rel_T": float(eT.max()), "p999_rel_T": q(eT),
                                  "max_abs_Y": float(eY.max()), "p999_abs_Y": q(eY)},
        "fallback_cells_max_diff_vs_plain": {"rel_T": float(fT.max()) if fb.any() else 0.0,
                                             "abs_Y": float(fY.max()) if fb.any() else 0.0},
        "train": {"pairs": n_pairs, "epochs": args.surrogate_epochs, "batch": 4096,
                  "first_loss": float(loss[0]), "final_loss": float(loss[-1]),
                  "data_s": t_data, "train_s": t_train},
        "roofline_inference": {"bound": "mfma", "achieved": achieved,
                               "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s",
                               "frac": achieved / PEAK_BF16_MFMA_TFLOPS},
    }


WORKLOADS = {
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


def cpu_baseline(boxes, path, threads, target_s=10.0):
    """The oracle, as it stands, on a bounded sample of the same workload:
    cells drawn uniformly (seed 123) from the concatenated boxes, each
    integrated over its box's n_sub sub-calls of dt, in chunks of 4096 until
    about target_s seconds of host time have been spent (the whole sample is
    cycled again if it is used up first)."""
    import oracle
    om = oracle.Mech(path)
    sizes = np.array([b["state"].shape[1] for b in boxes])
    n = int(sizes.sum())
    rng = np.random.Generator(np.random.PCG64(123))
    pick = rng.permutation(n)[:262144]
    starts = np.concatenate([[0], np.cumsum(sizes)])
    box_of = np.searchsorted(starts, pick, side="right") - 1
    done = 0
    t0 = time.perf_counter()
    el = 0.0
    while el < target_s:
        for c0 in range(0, len(pick), 4096):
            sel, bsel = pick[c0:c0 + 4096], box_of[c0:c0 + 4096]
            for bi in np.unique(bsel):
                b = boxes[bi]
                s = np.ascontiguousarray(b["state"][:, sel[bsel == bi] - starts[bi]])
                for _ in range(b.get("n_sub", 1)):
                    om.integrate(s, b["dt"], nthreads=threads)
            done += len(sel)
            el = time.perf_counter() - t0
            if el >= target_s:
                break
    return {"value": done / el, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} cells drawn uniformly (seed 123) from the same workload, one flow "
                      f"step each (with the box's sub-calls), in chunks of 4096: {el:.1f} s wall "
                      f"on {threads} host threads"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the integrator runs on one GPU (asked for --gpus {args.gpus}); "
              "the chemistry step needs no cross-GPU exchange, see the design notes",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2506_02602_amd import chemgpu, codegen, workloads as wl

    path, hboxes = load_workload(args.workload)
    n = int(sum(b["state"].shape[1] for b in hboxes))
    dev = torch.device("cuda:0")
    boxes, pristine = [], []
    for b in hboxes:
        st = torch.from_numpy(b["state"]).to(dev)
        nb = st.shape[1]
        pristine.append(st.clone())
        boxes.append(dict(state=st, dt=b["dt"], n_sub=b.get("n_sub", 1), level=b.get("level", 0),
                          status=torch.zeros(nb, dtype=torch.int32, device=dev),
                          counts=torch.zeros(2 * nb, dtype=torch.int32, device=dev)))
    mech = chemgpu.chem_mech_load(path)
    chemgpu.chem_workspace_reserve(mech, n)
    base = chemgpu.make_opts(rtol=wl.RTOL, atol=wl.ATOL, chunk_steps=args.chunk,
                             block_size=args.block, tail_steps=args.tail, scheme=args.scheme,
                             tail_cap=args.tail_cap, pool_order=args.pool_order)
    stream = torch.cuda.current_stream()

    def restore():
        for b, p in zip(boxes, pristine):
            b["state"].copy_(p)

    tuned = None
    log(f"workload {args.workload}: {n} cells in {len(boxes)} boxes")
    if not args.no_autotune and not (args.chunk or args.block):
        log("autotuning block, chunk and hand-off")
        # small workloads launch in milliseconds: time each candidate 3 times
        cache = None if args.tune_cache == "none" else args.tune_cache
        tb = chemgpu.chem_autotune(mech, boxes, base, reps=3 if n <= 2_000_000 else 1,
                                   cache_path=cache)
        tuned = {"block_size": tb.block_size, "chunk_steps": tb.chunk_steps,
                 "tail_steps": tb.tail_steps, "tail_cap": tb.tail_cap,
                 "pool_order": tb.pool_order}
    log(f"launch {tuned}; untimed pass with per-cell counters")
    # one untimed pass with per-cell counters for the flop count
    restore()
    chemgpu.chem_integrate_batched(mech, boxes, base)
    torch.cuda.synchronize()
    st = np.concatenate([b["status"].cpu().numpy() for b in boxes])
    cn = np.concatenate([b["counts"].cpu().numpy().reshape(2, -1) for b in boxes], axis=1)
    total_steps = int(cn.sum())
    m = codegen.parse(path)
    flops_per_step = codegen.step_flops(m, args.scheme)
    flops_per_launch = total_steps * flops_per_step

    # the timed launches: one graph holding the whole batched call
    tboxes = [dict(b, status=None, counts=None) for b in boxes]
    graph = chemgpu.chem_graph_capture_batched(mech, tboxes, base)
    for _ in range(max(args.warmup, 1)):
        restore()
        graph.launch()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for k in range(args.steps):
        restore()
        ev[k][0].record(stream)
        graph.launch(stream)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    graph.close()
    kern_all = np.array([a.elapsed_time(b) for a, b in ev])
    kern_ms = float(np.mean(kern_all))
    ms_per_step = elapsed * 1e3 / args.steps
    value = n * args.steps / elapsed
    achieved = flops_per_launch / (kern_ms * 1e-3) / 1e12
    rec = TRAFFIC.get(args.workload) if args.scheme == "lsrk" else None
    current = bool(rec) and rec[0] == kernel_digest()

    # The dominant kernel, timed live: the same flow step as plain calls with
    # the library's per-kernel timing (HIP events around each launch, on the
    # launch stream).  Its algorithmic flops: a cell still stepping after
    # the hand-off point takes its remaining steps in the cooperative kernel
    # when the list fits the cap, else in the resumption launch of the
    # per-lane kernel.
    log("per-kernel timing")
    chemgpu.chem_set_kernel_timing(mech, True)
    recs = []
    for _ in range(max(3, min(args.steps, 10))):
        restore()
        chemgpu.chem_integrate_batched(mech, tboxes, base)
        recs.append(chemgpu.chem_kernel_times(mech))
    chemgpu.chem_set_kernel_timing(mech, False)
    kt = {k: float(np.mean([r[k] for r in recs])) for k in recs[0]}
    eff = tuned or {}
    tail = args.tail or eff.get("tail_steps", 0)
    cap = args.tail_cap or eff.get("tail_cap", 0) or 64   # 0: the library's default, 64 per CU
    per_cell = cn.sum(axis=0)
    coop_steps = 0
    if args.scheme == "lsrk" and tail > 0:
        over = per_cell[per_cell > tail]
        n_cu = torch.cuda.get_device_properties(0).multi_processor_count
        if cap < 0 or over.size <= cap * n_cu:
            coop_steps = int((over - tail).sum())
    pers_ms = kt["persistent"] + kt["resume"]
    if kt["coop"] > pers_ms:
        dom, dom_ms, dom_steps = "lsrk_coop", kt["coop"], coop_steps
    else:
        dom, dom_ms, dom_steps = "lsrk_persistent", pers_ms, total_steps - coop_steps
    dom_achieved = dom_steps * flops_per_step / (dom_ms * 1e-3) / 1e12
    dom_traffic = rec[2].get(dom) if current and len(rec) > 2 else None
    nv = mech.n_species + 1
    out = {
        "metric": METRIC, "value": value, "unit": "cells/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "name": args.workload,
                   "cells": n, "boxes": len(boxes),
                   "scheme": args.scheme,
                   "chunk_steps": args.chunk, "block_size": args.block, "tail_steps": args.tail,
                   "tail_cap": args.tail_cap, "pool_order": args.pool_order,
                   "autotuned": tuned},
        # the dominant kernel: its algorithmic flops per launch over its mean
        # launch time (traffic: its HBM bytes per launch from the counters)
        "roofline": {"bound": "alu", "kernel": dom, "achieved": dom_achieved,
                     "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": dom_achieved / PEAK_FP64_VECTOR_TFLOPS, "traffic": dom_traffic,
                     "launch_ms": dom_ms, "rk_steps_per_launch": dom_steps},
        # the whole flow step (all its launches) against the HIP-event time of
        # the graph launch
        "roofline_flow_step": {"bound": "alu", "achieved": achieved,
                               "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                               "frac": achieved / PEAK_FP64_VECTOR_TFLOPS,
                               "traffic": rec[1] if current else None},
        "kernel_times_ms": kt,
        # per flow step: read (T, Y, rho, h), write (T, Y, h) of every cell
        "hbm_algorithmic_bytes": n * 8 * ((nv + 2) + (nv + 1)),
        "kernel_ms": kern_ms,
        "kernel_ms_p10_p50_p90": [float(np.percentile(kern_all, q)) for q in (10, 50, 90)],
        "steps_per_flow_step": {"total_rk_steps": total_steps,
                                "rejected": int(cn[1].sum()),
                                "max_per_cell": int(cn.sum(axis=0).max()),
                                "status_nonzero": int((st != 0).sum())},
        "flops_per_rk_step": flops_per_step,
    }
    sub_calls = int(sum(b["state"].shape[1] * b.get("n_sub", 1) for b in hboxes))
    if sub_calls != n:
        out["cell_subcalls_per_s"] = sub_calls * args.steps / elapsed
    if not args.no_cpu:
        threads = args.cpu_threads or min(os.cpu_count() or 1, 16)
        log(f"oracle on {threads} host threads")
        out["cpu_baseline"] = cpu_baseline(hboxes, path, threads)
    if not args.no_surrogate and args.workload == "front":
        del boxes, pristine, tboxes
        torch.cuda.empty_cache()
        log("surrogate leg")
        out["surrogate"] = surrogate_leg(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
