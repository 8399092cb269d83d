"""How far two correct FP64 integrations of one cell may end apart, per
workload: the allowance the GPU parity tests give cells whose adaptive step
path differs from the oracle's.

The parity bar (one flow step from identical inputs, |x_gpu - x_cpu| <=
1e-8 |x_cpu|, + 1e-13 on Y) holds for a cell whose step sequence is the
oracle's.  The controller of Eq. 22 bounds each step's local error, not the
global one, and a step whose WRMS error sits at the accept/reject boundary is
decided by the last bit of the arithmetic; the GPU evaluates the
exponentials, the rate sums and the step factor in other orders than the
oracle, so on such cells it may take another, equally valid, sequence of steps
and end up to a few hundred tolerance units (rtol |x| + atol) away.

This module measures that directly, on the CPU, with the oracle alone: the
oracle against copies of itself that differ by one rounding (``STUDY_MODES``:
k_f one ulp up; the step factor err^(-1/4) taken as 1/sqrt(sqrt(err));
production rates summed in reverse reaction order; k_r from one exponential;
all four together; the initial temperature one ulp up), on seeded samples of
each workload the GPU tests use.  A cell is *flagged* when some copy misses
the parity bar against the unperturbed oracle; ``STUDY`` holds, per workload,
the sample size, the number of cells so flagged and the largest distance of a
flagged cell in tolerance units.  ``tests/test_parity_budget.py`` recomputes
every entry and requires the same numbers, so the figures below are
reproducible from the tree.

Allowances derived from them (the stated margin):
  * flagged cells in a GPU sample of n cells: at most
    floor(1.25 f n + 3 sqrt(1.25 f n) + 2), f = the study's flagged fraction
    (a quarter more than the study, three standard deviations of counting
    noise, and two cells);
  * distance of a flagged cell: at most max(10, 2 u) tolerance units, u = the
    study's largest;
  * every flagged cell must meet the 1e-8 bar when both sides re-run it at
    rtol 1e-11 / atol 1e-14, where the step paths coincide again.
"""
from __future__ import annotations

import math

import numpy as np

RTOL, ATOL = 1e-8, 1e-10

# perturbed copies: oracle perturbation bits (see oracle.set_perturbation),
# and "T0" = the unperturbed oracle started from T one ulp up
STUDY_MODES = (1, 2, 4, 8, 15, "T0")

# workload -> (cells in the study, cells flagged, largest distance of a
# flagged cell in tolerance units); measured by measure(), checked by
# tests/test_parity_budget.py
STUDY = {
    "cells": (4096, 0, 0.0),
    "front_hot": (21008, 0, 0.0),
    "stress9": (20000, 0, 0.0),
    "stress32": (4000, 324, 135.2),
    "amr": (8640, 0, 0.0),
    "diverge_a1": (256, 0, 0.0),
    "diverge_a01": (256, 44, 50.4),
    "front_hot_rkf45": (4202, 0, 0.0),
    "stress32_rkf45": (1000, 4, 0.6),
    "front_hot_ros4": (4202, 0, 0.0),
    "front_hot_ros4_dt1e-5": (106, 0, 0.0),
}


def allowed_flags(workload: str, n: int) -> int:
    n_study, flagged, _ = STUDY[workload]
    mu = 1.25 * flagged / n_study * n
    return int(math.floor(mu + 3.0 * math.sqrt(mu) + 2.0))


def unit_bound(workload: str) -> float:
    return max(10.0, 2.0 * STUDY[workload][2])


def tolerance_units(a, b, ns, rtol=RTOL, atol=ATOL):
    """Per cell: max over T and Y of |a - b| / (rtol |b| + atol), atol 0 on T."""
    sc = rtol * np.abs(b[:ns + 1]) + np.r_[0.0, [atol] * ns][:, None]
    sc[0] = rtol * np.abs(b[0])
    return (np.abs(a[:ns + 1] - b[:ns + 1]) / sc).max(axis=0)


def misses_bar(a, b, ns, rtol=RTOL, floor_y=1e-13):
    dT = np.abs(a[0] - b[0]) > rtol * np.abs(b[0])
    dY = (np.abs(a[1:ns + 1] - b[1:ns + 1]) > rtol * np.abs(b[1:ns + 1]) + floor_y).any(axis=0)
    return dT | dY


# ------------------------------------------------------------ the workloads
def _workloads():
    """name -> (mechanism, state sample, dt, sub-calls, oracle keywords)."""
    from paper_2506_02602_amd import workloads as wl
    p9, p32 = wl.mech_file("mech9"), wl.mech_file("mech32")
    out = {}

    def front_hot():
        s, hot = wl.front_2d(p9)
        return np.ascontiguousarray(s[:, hot])

    def stress(path, n, seed):
        st = wl.stress_3d(path)
        rng = np.random.Generator(np.random.PCG64(seed))
        return np.ascontiguousarray(st[:, rng.choice(st.shape[1], n, replace=False)])

    def amr():
        rng = np.random.Generator(np.random.PCG64(91))
        parts = []
        for b in wl.amr_hierarchy(p9):
            n = b["state"].shape[1]
            hot = np.where(b["hot"])[0]
            pick = np.concatenate([hot[:100], rng.choice(n, 40, replace=False)])
            parts.append((np.ascontiguousarray(b["state"][:, pick]), b["dt"], b["n_sub"]))
        return parts

    def diverge(alpha):
        d = wl.diverge_box(p9, alpha)                          # x fastest, then y, then z
        return np.ascontiguousarray(d[:, 0:16 * 256:16])       # the 256 distinct y rows

    out["cells"] = lambda: (p9, [(wl.cells_uniform(p9), wl.DT_FLOW, 1)], {})
    out["front_hot"] = lambda: (p9, [(front_hot(), wl.DT_FLOW, 1)], {})
    out["stress9"] = lambda: (p9, [(stress(p9, 20000, 5), wl.DT_FLOW, 1)], {})
    out["stress32"] = lambda: (p32, [(stress(p32, 4000, 6), wl.DT_FLOW, 1)], {})
    out["amr"] = lambda: (p9, amr(), {})
    out["diverge_a1"] = lambda: (p9, [(diverge(1.0), wl.DIVERGE_DT, wl.DIVERGE_CALLS)], {})
    out["diverge_a01"] = lambda: (p9, [(diverge(0.1), wl.DIVERGE_DT, wl.DIVERGE_CALLS)], {})
    out["front_hot_rkf45"] = lambda: (p9, [(front_hot()[:, ::5], wl.DT_FLOW, 1)],
                                      {"scheme": "rkf45"})
    out["stress32_rkf45"] = lambda: (p32, [(stress(p32, 1000, 7), wl.DT_FLOW, 1)],
                                     {"scheme": "rkf45"})
    out["front_hot_ros4"] = lambda: (p9, [(front_hot()[:, ::5], wl.DT_FLOW, 1)],
                                     {"scheme": "ros4"})
    out["front_hot_ros4_dt1e-5"] = lambda: (p9, [(front_hot()[:, ::200], 1e-5, 1)],
                                            {"scheme": "ros4"})
    return out


WORKLOADS = tuple(STUDY)


def _run(om, state, dt, n_sub, mode, kw):
    import oracle
    s = np.array(state)
    if mode == "T0":
        s[0] = np.nextafter(s[0], np.inf)
    else:
        oracle.set_perturbation(mode)
    try:
        for _ in range(n_sub):
            om.integrate(s, dt, **kw)
    finally:
        oracle.set_perturbation(0)
    return s


def measure(name: str, nthreads=None):
    """(cells, flagged, largest flagged distance in tolerance units) of one
    workload, and whether every flagged cell meets the bar at rtol 1e-11."""
    import oracle
    path, parts, kw = _workloads()[name]()
    om = oracle.Mech(path)
    ns = om.ns
    n_tot = flagged = 0
    umax = 0.0
    tight_ok = True
    for state, dt, n_sub in parts:
        k = dict(kw, nthreads=nthreads)
        base = _run(om, state, dt, n_sub, 0, k)
        bad = np.zeros(state.shape[1], bool)
        for mode in STUDY_MODES:
            p = _run(om, state, dt, n_sub, mode, k)
            b = misses_bar(p, base, ns)
            if b.any():
                umax = max(umax, float(tolerance_units(p[:, b], base[:, b], ns).max()))
            new = b & ~bad                      # re-run each flagged cell once, tight
            if new.any():
                kt = dict(k, rtol=1e-11, atol=1e-14, max_steps=2000000)
                sub = np.ascontiguousarray(state[:, new])
                t0 = _run(om, sub, dt, n_sub, 0, kt)
                t1 = _run(om, sub, dt, n_sub, mode, kt)
                tight_ok = tight_ok and not misses_bar(t1, t0, ns).any()
            bad |= b
        n_tot += state.shape[1]
        flagged += int(bad.sum())
    return n_tot, flagged, round(umax, 1), tight_ok
