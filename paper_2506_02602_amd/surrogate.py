"""Surrogate pipeline: training data from the FP64 integrator, training on the
GPU, trust-threshold selection and the evaluation field.

Every numerical step runs in the library's kernels through the C ABI
(``chemgpu``); this module only sequences the calls and moves tensors.

Training data.  Cells of the 4096-cell stoichiometric H2/O2/N2 workload
(T0 ~ U[1000, 1600] K, 1 atm) are integrated by the FP64 path through R
record times spaced logarithmically from 1e-7 s to 1e-2 s, so every
trajectory covers induction, ignition and the approach to equilibrium.  From
each record a pair is made with one flow step of dt drawn log-uniform in
[2.5e-8, 2e-7] s (one dt per record, shared by the cells of that record):
(state, dt) -> increment.  95 % of the trajectories train, 5 % validate.

Evaluation field (256^3 cells).  90 % of the cells take states of held-out
trajectories (a different seed) arranged in smooth 3-D blobs: two smooth
fields pick the trajectory and the record of each cell; the other 10 %, in
a smooth region of their own, take reacting-front states (cold 300 K / 1 atm
and hot 1500-3000 K / 5-30 atm cells), which lie outside the training
hull and exercise the fallback.
"""
from __future__ import annotations

import math

import numpy as np

from . import chemgpu as cg
from . import workloads as wl

DT_LO, DT_HI = 2.5e-8, 2.0e-7


def _torch():
    import torch
    return torch


def trajectories(mech, state0: np.ndarray, times, opts=None):
    """FP64 states of every cell of state0 at each record time (device tensor
    [R, N+3, n]); the step-size hint is carried between records."""
    torch = _torch()
    s = torch.from_numpy(np.ascontiguousarray(state0)).cuda()
    R = len(times)
    snaps = torch.empty((R,) + tuple(s.shape), dtype=torch.float64, device="cuda")
    t_prev = 0.0
    for j, t in enumerate(times):
        cg.chem_integrate(mech, s, float(t - t_prev), opts)
        snaps[j].copy_(s)
        t_prev = float(t)
    torch.cuda.synchronize()
    return snaps


def pairs_from_snapshots(mech, snaps, dts, opts=None):
    """(X, Y) training pairs: one FP64 flow step of dts[j] from every record j."""
    torch = _torch()
    R, nv, n = snaps.shape
    after = snaps.clone()
    boxes = [dict(state=after[j], dt=float(dts[j])) for j in range(R)]
    cg.chem_integrate_batched(mech, boxes, opts)
    X = torch.empty((R * n, mech.n_species + 3), dtype=torch.float32, device="cuda")
    Y = torch.empty((R * n, mech.n_species + 1), dtype=torch.float32, device="cuda")
    for j in range(R):
        cg.surrogate_make_pairs(mech, snaps[j], after[j], dt=float(dts[j]),
                                X=X[j * n:(j + 1) * n], Y=Y[j * n:(j + 1) * n])
    torch.cuda.synchronize()
    return X, Y, after


def build_dataset(mech, n_cells=4096, n_records=2441, t_end=1e-2, seed=1, val_frac=0.05):
    """Returns dict with train/validation tensors and the record layout."""
    torch = _torch()
    state0 = wl.cells_uniform(mech.path, n=n_cells, seed=seed)
    times = np.geomspace(1e-7, t_end, n_records)
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    dts = np.exp(rng.uniform(math.log(DT_LO), math.log(DT_HI), n_records))
    snaps = trajectories(mech, state0, times)
    X, Y, after = pairs_from_snapshots(mech, snaps, dts)
    n_val = max(1, int(round(val_frac * n_cells)))
    cell = torch.arange(n_records * n_cells, device="cuda") % n_cells
    val = cell >= n_cells - n_val
    return dict(X=X[~val].contiguous(), Y=Y[~val].contiguous(), Xv=X[val].contiguous(),
                Yv=Y[val].contiguous(), snaps=snaps, after=after, dts=dts, times=times,
                n_val=n_val, n_cells=n_cells)


def validation_states(ds, n_blocks=64):
    """Held-out (state before, FP64 state after, dt) blocks for n_blocks
    records spread evenly over the trajectories."""
    n, nv = ds["n_cells"], ds["n_val"]
    R = len(ds["dts"])
    js = np.unique(np.linspace(0, R - 1, min(n_blocks, R)).astype(int))
    return [(ds["snaps"][j][:, n - nv:].contiguous(), ds["after"][j][:, n - nv:].contiguous(),
             float(ds["dts"][j])) for j in js]


def errors(result, ref, ns):
    """Per-cell relative T error and max absolute Y error (numpy arrays)."""
    eT = (result[0] - ref[0]).abs() / ref[0].abs()
    eY = (result[1:ns + 1] - ref[1:ns + 1]).abs().max(dim=0).values
    return eT, eY


def tune_trust(surr, mech, blocks, target_T=1e-3, target_Y=1e-4, margins=(0.0, 0.05, 0.2)):
    """Loosest trust thresholds whose trusted validation cells all meet the
    error targets (max relative T error, max absolute Y error); ties go to
    the larger trusted fraction.  Returns (trust tuple, stats)."""
    torch = _torch()
    ns = mech.n_species
    grid = []
    for m in margins:
        for et in (0.05, 0.2, 0.5, 1.0, 2.0, 5.0):
            for el in (1e-6, 1e-5, 1e-4):
                grid.append((m, el, 1e-7, et))
    best, best_stats = None, None
    for tr in grid:
        worst_T = worst_Y = 0.0
        trusted = total = 0
        for before, after, dt in blocks:
            s = before.clone()
            tc = torch.zeros(s.shape[1], dtype=torch.int32, device="cuda")
            cg.surrogate_infer(surr, mech, s, dt, tr, fallback=False, trust_code=tc)
            ok = tc == 0
            total += s.shape[1]
            trusted += int(ok.sum())
            if ok.any():
                eT, eY = errors(s[:, ok], after[:, ok], ns)
                worst_T = max(worst_T, float(eT.max()))
                worst_Y = max(worst_Y, float(eY.max()))
        frac = trusted / total
        good = worst_T <= target_T and worst_Y <= target_Y
        if good and (best is None or frac > best_stats["trusted_frac"]):
            best, best_stats = tr, dict(trusted_frac=frac, max_rel_T=worst_T, max_abs_Y=worst_Y)
    return best, best_stats


def smooth_field(shape, n_blobs, rng):
    """Sum of Gaussian blobs on a periodic-free grid, scaled to [0, 1)."""
    nx, ny, nz = shape
    x = np.linspace(0, 1, nx)[:, None, None]
    y = np.linspace(0, 1, ny)[None, :, None]
    z = np.linspace(0, 1, nz)[None, None, :]
    f = np.zeros(shape, dtype=np.float32)
    for _ in range(n_blobs):
        c = rng.uniform(0, 1, 3)
        r = rng.uniform(0.08, 0.3)
        a = rng.uniform(0.5, 1.5)
        f += (a * np.exp(-(((x - c[0]) ** 2) + ((y - c[1]) ** 2) + ((z - c[2]) ** 2)) /
                         (2 * r * r))).astype(np.float32)
    f -= f.min()
    f /= f.max() * (1 + 1e-6)
    return f.reshape(-1)


def inference_field(mech, shape=(256, 256, 256), n_traj=1024, n_records=1024, t_end=1e-2,
                    seed=5, out_frac=0.10):
    """The evaluation field (device tensor [N+3, prod(shape)]) and its masks."""
    torch = _torch()
    state0 = wl.cells_uniform(mech.path, n=n_traj, seed=seed)
    times = np.geomspace(1e-7, t_end, n_records)
    snaps = trajectories(mech, state0, times)          # [R, N+3, n_traj]
    rng = np.random.Generator(np.random.PCG64(seed))
    ft = smooth_field(shape, 12, rng)
    fr = smooth_field(shape, 12, rng)
    fo = smooth_field(shape, 6, rng)
    ti = torch.from_numpy((ft * n_traj).astype(np.int64)).cuda()
    ri = torch.from_numpy((fr * n_records).astype(np.int64)).cuda()
    flat = snaps.permute(1, 0, 2).reshape(snaps.shape[1], -1)    # [N+3, R * n_traj]
    field = flat[:, ri * n_traj + ti].contiguous()
    out = torch.from_numpy(fo >= np.quantile(fo, 1.0 - out_frac)).cuda()
    n_out = int(out.sum())
    front, hot = wl.front_2d(mech.path, nx=512, ny=512, seed=seed)
    pick = np.concatenate([np.where(hot)[0], np.where(~hot)[0][:3 * int(hot.sum())]])
    src = torch.from_numpy(np.ascontiguousarray(front[:, pick])).cuda()
    field[:, out] = src[:, torch.arange(n_out, device="cuda") % src.shape[1]]
    field[mech.n_species + 2] = 0.0                     # no step hint
    del snaps, flat
    return field, out
