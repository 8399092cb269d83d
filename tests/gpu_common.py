"""Shared helpers for the GPU parity tests (HIP path vs the CPU oracle)."""
import os

import numpy as np

import parity_budget

# Parity bar for one flow step from identical inputs: per component
# |gpu - cpu| <= RTOL_PARITY |cpu| + floor, with the floor 1e-13 (1e-3 atol)
# on Y and 0 on T.
RTOL_PARITY = 1e-8
FLOOR_Y = 1e-13


def to_gpu(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def run_gpu(mech, state, dt, **opt):
    import torch
    from paper_2506_02602_amd import chemgpu
    n = state.shape[1]
    s = to_gpu(state)
    st = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")
    cn = torch.full((2 * max(n, 1),), -7, dtype=torch.int32, device="cuda")
    chemgpu.chem_integrate(mech, s, dt, chemgpu.make_opts(**opt), status=st, counts=cn)
    torch.cuda.synchronize()
    return s.cpu().numpy(), st.cpu().numpy()[:n], cn.cpu().numpy()[:2 * n].reshape(2, n)


def parity_violations(gpu, cpu, ns, rtol=RTOL_PARITY, floor_y=FLOOR_Y):
    """Boolean mask [n] of cells where T or any Y misses the parity bar."""
    dT = np.abs(gpu[0] - cpu[0]) > rtol * np.abs(cpu[0])
    dY = (np.abs(gpu[1:ns + 1] - cpu[1:ns + 1]) >
          rtol * np.abs(cpu[1:ns + 1]) + floor_y).any(axis=0)
    return dT | dY


def max_rel(gpu, cpu, ns, floor_y=FLOOR_Y):
    eT = np.max(np.abs(gpu[0] - cpu[0]) / np.abs(cpu[0]))
    eY = np.max(np.abs(gpu[1:ns + 1] - cpu[1:ns + 1]) / (np.abs(cpu[1:ns + 1]) + floor_y / RTOL_PARITY))
    return float(eT), float(eY)


def check_flagged(gsub, csub, ns, budget, rerun=None, label="", rtol=1e-8, atol=1e-10):
    """Parity of GPU results gsub against oracle results csub (SoA blocks of
    the same cells).  Every cell must meet the 1e-8 bar except cells whose
    adaptive step path differs from the oracle's (see parity_budget): those
    ("flagged") may number at most parity_budget.allowed_flags(budget, n),
    must lie within parity_budget.unit_bound(budget) tolerance units
    (rtol |x| + atol), and, when `rerun` is given, must meet the bar once
    both sides integrate them at rtol 1e-11 / atol 1e-14: rerun(indices)
    returns that (gpu, cpu) pair.  Returns the flagged mask."""
    bad = parity_violations(gsub, csub, ns)
    n, nb = bad.size, int(bad.sum())
    units = 0.0
    if nb:
        units = float(parity_budget.tolerance_units(gsub[:, bad], csub[:, bad], ns, rtol, atol).max())
    allowed = parity_budget.allowed_flags(budget, n)
    bound = parity_budget.unit_bound(budget)
    print(f"[parity] {label}: {n} cells, {nb} flagged (allowed {allowed}, study '{budget}'), "
          f"max {units:.1f} of {bound:.0f} tolerance units", flush=True)
    assert nb <= allowed, f"{label}: {nb} flagged cells, budget {allowed}"
    assert units <= bound, f"{label}: flagged cells {units:.1f} tolerance units apart"
    if nb and rerun is not None:
        g2, c2 = rerun(np.where(bad)[0])
        tb = parity_violations(g2, c2, ns)
        assert not tb.any(), f"{label}: {tb.sum()} flagged cells still differ at rtol 1e-11"
    return bad


def assert_parity(gmech, omech, s_full, dt, idx=None, budget="front_hot", label="", **opt):
    """Parity of one flow step, GPU vs oracle, on the cells `idx` of s_full.

    The GPU integrates the whole block; the oracle integrates the sampled
    cells.  Status codes must be equal everywhere; values must meet the 1e-8
    bar except for the flagged cells check_flagged allows under the
    workload's `budget`, each of which must meet it again when both sides
    re-run it at rtol 1e-11.  Returns the number of flagged cells."""
    ns = omech.ns
    n = s_full.shape[1]
    idx = np.arange(n) if idx is None else np.asarray(idx)
    g, gst, gcn = run_gpu(gmech, s_full, dt, **opt)
    sub = np.ascontiguousarray(s_full[:, idx])
    c = sub.copy()
    kw = {k: v for k, v in opt.items() if k in ("rtol", "atol", "max_steps", "fixed_steps",
                                                 "scheme")}
    cst, ccn = omech.integrate(c, dt, **kw)
    gsub = np.ascontiguousarray(g[:, idx])
    assert np.array_equal(gst[idx], cst), "per-cell status differs"

    def rerun(fi):
        tight = np.ascontiguousarray(sub[:, fi])
        o2 = dict(opt, rtol=1e-11, atol=1e-14, max_steps=2000000)
        g2, _, _ = run_gpu(gmech, tight, dt, **o2)
        c2 = tight.copy()
        omech.integrate(c2, dt, rtol=1e-11, atol=1e-14, max_steps=2000000,
                        scheme=opt.get("scheme", "lsrk"))
        return g2, c2

    bad = check_flagged(gsub, c, ns, budget, rerun, label,
                        rtol=opt.get("rtol", 1e-8) or 1e-8, atol=opt.get("atol", 1e-10) or 1e-10)
    if not bad.any():
        assert np.array_equal(gcn[:, idx], ccn), "accepted/rejected counts differ"
    return int(bad.sum())


def oracle_subcalls(om, state, dt, n_sub, **kw):
    """n_sub oracle calls of dt on a copy of `state`; a cell stops at its
    first non-OK sub-call.  Returns (state, status, counts)."""
    s = state.copy()
    n = s.shape[1]
    status = np.zeros(n, np.int32)
    counts = np.zeros((2, n), np.int32)
    live = np.arange(n)
    for _ in range(n_sub):
        if len(live) == 0:
            break
        sub = np.ascontiguousarray(s[:, live])
        st, cn = om.integrate(sub, dt, **kw)
        s[:, live] = sub
        counts[:, live] += cn
        status[live] = st
        live = live[st == 0]
    return s, status, counts


def tuned_launch(mech, boxes, rtol=1e-8, atol=1e-10, scheme="lsrk"):
    """The launch the committed tuning cache holds for these boxes, read
    through chem_autotune from a copy of the cache that must come back
    unchanged (a hit: nothing is tuned or timed).  Returns make_opts
    keywords with every launch field spelled out."""
    import shutil
    import tempfile
    from paper_2506_02602_amd import chemgpu
    fd, cache = tempfile.mkstemp(suffix=".json")
    os.close(fd)
    try:
        shutil.copy(os.path.join(os.path.dirname(chemgpu.__file__), "tuning_gfx950.json"), cache)
        before = open(cache).read()
        base = chemgpu.make_opts(rtol=rtol, atol=atol, scheme=scheme)
        tb = chemgpu.chem_autotune(mech, boxes, base, reps=1, cache_path=cache)
        assert open(cache).read() == before, "no cached launch for this workload"
    finally:
        os.unlink(cache)
    return dict(rtol=rtol, atol=atol, scheme=scheme, block_size=tb.block_size,
                chunk_steps=tb.chunk_steps, tail_steps=tb.tail_steps, tail_cap=tb.tail_cap,
                pool_order=tb.pool_order)
