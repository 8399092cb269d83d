"""Batched AMR integration, hipGraph replay and the autotuner, on the GPU.

Reference: each box's cells integrated by the oracle as n_sub successive
flow-step calls of the box's dt (the step-size hint carried in the state's h
row), i.e. the chemistry calls of a subcycled AMR coarse step (paper Sec. 3.2,
Algorithm 1)."""
import json
import os
import tempfile

import numpy as np
import pytest

from paper_2506_02602_amd import workloads as wl

from gpu_common import check_flagged, oracle_subcalls, parity_violations, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cg():
    from paper_2506_02602_amd import chemgpu
    return chemgpu


@pytest.fixture(scope="module")
def gm9(cg, mech9_path):
    return cg.chem_mech_load(mech9_path)


def gpu_boxes(hier, with_out=True):
    import torch
    boxes = []
    for b in hier:
        n = b["state"].shape[1]
        d = dict(state=to_gpu(b["state"]), dt=b["dt"], n_sub=b["n_sub"], level=b["level"])
        if with_out:
            d["status"] = torch.full((n,), -7, dtype=torch.int32, device="cuda")
            d["counts"] = torch.full((2 * n,), -7, dtype=torch.int32, device="cuda")
        boxes.append(d)
    return boxes


def small_hierarchy(path, seed=13):
    return wl.amr_hierarchy(path, seed=seed, boxes_per_level=(2, 3, 4), edges=(8, 12, 16))


@pytest.mark.parametrize("tail", [0, 3])
def test_batched_matches_oracle_subcycling(cg, gm9, omech9, mech9_path, tail):
    """tail = 3 hands nearly every hot cell to the cooperative kernel, most of
    them with sub-calls still to run."""
    import torch
    hier = small_hierarchy(mech9_path)
    boxes = gpu_boxes(hier)
    cg.chem_integrate_batched(gm9, boxes, cg.make_opts(tail_steps=tail))
    torch.cuda.synchronize()
    gall, call = [], []
    for hb, gb in zip(hier, boxes):
        c, cst, ccn = oracle_subcalls(omech9, hb["state"], hb["dt"], hb["n_sub"])
        g = gb["state"].cpu().numpy()
        gst = gb["status"].cpu().numpy()
        gcn = gb["counts"].cpu().numpy().reshape(2, -1)
        assert np.array_equal(gst, cst)

        def rerun(idx, hb=hb):
            tight = np.ascontiguousarray(hb["state"][:, idx])
            gt = to_gpu(tight)
            cg.chem_integrate_batched(gm9, [dict(state=gt, dt=hb["dt"], n_sub=hb["n_sub"])],
                                      cg.make_opts(rtol=1e-11, atol=1e-14, max_steps=2000000,
                                                   tail_steps=tail))
            c2, _, _ = oracle_subcalls(omech9, tight, hb["dt"], hb["n_sub"], rtol=1e-11,
                                       atol=1e-14, max_steps=2000000)
            return gt.cpu().numpy(), c2
        bad = check_flagged(g, c, 9, "amr", rerun, f"small AMR box (tail {tail})")
        if not bad.any():
            assert np.array_equal(gcn, ccn)
        gall.append(g)
        call.append(c)
    # the allowance over all boxes together
    check_flagged(np.hstack(gall), np.hstack(call), 9, "amr", None,
                  f"small AMR batch (tail {tail}), all boxes")


def test_batched_equals_per_box_calls(cg, gm9, mech9_path):
    """One batched launch == host-driven per-box sub-calls of chem_integrate,
    bitwise (per-lane kernel only: the cooperative hand-off counts steps over
    all sub-calls of a batched cell, but per call here)."""
    import torch
    hier = small_hierarchy(mech9_path, seed=14)
    boxes = gpu_boxes(hier)
    off = cg.make_opts(tail_steps=-1)
    cg.chem_integrate_batched(gm9, boxes, off)
    for hb, gb in zip(hier, boxes):
        t = to_gpu(hb["state"])
        tot = torch.zeros(2 * t.shape[1], dtype=torch.int32, device="cuda")
        cn = torch.zeros_like(tot)
        for _ in range(hb["n_sub"]):
            cg.chem_integrate(gm9, t, hb["dt"], off, counts=cn)
            tot += cn
        torch.cuda.synchronize()
        assert torch.equal(t, gb["state"])
        assert torch.equal(tot, gb["counts"])


@pytest.mark.parametrize("tail", [0, 3])
def test_graph_replay_matches_eager(cg, gm9, mech9_path, tail):
    """Replays of a captured graph (per-lane and cooperative kernels), with
    eager work and syncs between them, each reproduce the eager batched
    result exactly."""
    import torch
    hier = small_hierarchy(mech9_path, seed=15)
    opts = cg.make_opts(tail_steps=tail)
    eager = gpu_boxes(hier)
    cg.chem_integrate_batched(gm9, eager, opts)
    torch.cuda.synchronize()
    boxes = gpu_boxes(hier)
    pristine = [b["state"].clone() for b in boxes]
    g = cg.chem_graph_capture_batched(gm9, boxes, opts)
    other = to_gpu(wl.cells_uniform(mech9_path, n=3000, seed=3))
    for rep in range(4):
        for b, p in zip(boxes, pristine):
            b["state"].copy_(p)
        g.launch()
        cg.chem_integrate(gm9, other, wl.DT_FLOW)      # unrelated eager work in between
        torch.cuda.synchronize()
        for b, e in zip(boxes, eager):
            assert torch.equal(b["state"], e["state"]), f"replay {rep}"
            assert torch.equal(b["counts"], e["counts"])
    g.close()


def test_autotune_keeps_data_and_caches(cg, mech9_path):
    import torch
    m = cg.chem_mech_load(mech9_path)        # fresh handle: no tuned entries yet
    hier = small_hierarchy(mech9_path, seed=16)
    boxes = gpu_boxes(hier, with_out=False)
    before = [b["state"].clone() for b in boxes]
    fd, cache = tempfile.mkstemp(suffix=".json")
    os.close(fd)
    os.unlink(cache)
    try:
        best = cg.chem_autotune(m, boxes, reps=1, cache_path=cache)
        torch.cuda.synchronize()
        assert best.block_size in (64, 128, 192, 256, 384, 512)
        assert best.chunk_steps in (1, 2, 4, 8, 16, 32, 64)
        for b, p in zip(boxes, before):
            assert torch.equal(b["state"], p)          # caller's data untouched
        entries = json.load(open(cache))["entries"]
        assert len(entries) == 1 and entries[0]["key"].startswith(f"{m.hash:016x}:")
        again = cg.chem_autotune(cg.chem_mech_load(mech9_path), boxes, reps=1, cache_path=cache)
        assert (again.block_size, again.chunk_steps) == (best.block_size, best.chunk_steps)
        # tuned defaults give the same numbers as the explicit choice
        b1 = gpu_boxes(hier, with_out=False)
        b2 = gpu_boxes(hier, with_out=False)
        cg.chem_integrate_batched(m, b1)
        cg.chem_integrate_batched(m, b2, cg.make_opts(block_size=best.block_size,
                                                      chunk_steps=best.chunk_steps))
        torch.cuda.synchronize()
        for x, y in zip(b1, b2):
            assert torch.equal(x["state"], y["state"])
    finally:
        if os.path.exists(cache):
            os.unlink(cache)


@pytest.mark.parametrize("launch", ["default", "tuned"])
def test_full_amr_hierarchy_sampled(cg, gm9, omech9, mech9_path, launch):
    """The full 3-level, 96-box hierarchy in one graph launch, with the
    library's default launch and with the one the committed tuning cache
    holds for it (the benchmark's); the oracle checks up to 400 sampled
    cells per box (all of them hot on level 2)."""
    import torch
    from gpu_common import tuned_launch
    hier = wl.amr_hierarchy(mech9_path)
    ncells = sum(b["state"].shape[1] for b in hier)
    print(f"[amr] {len(hier)} boxes, {ncells} cells", flush=True)
    boxes = gpu_boxes(hier)
    opts = cg.make_opts(**tuned_launch(gm9, boxes)) if launch == "tuned" else None
    g = cg.chem_graph_capture_batched(gm9, boxes, opts)
    g.launch()
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(99))
    gall, call, tight_in = [], [], []
    for hb, gb in zip(hier, boxes):
        n = hb["state"].shape[1]
        hot = np.where(hb["hot"])[0]
        pick = hot[:200] if len(hot) else np.array([], int)
        pick = np.concatenate([pick, rng.choice(n, 200, replace=False)])
        sub = np.ascontiguousarray(hb["state"][:, pick])
        c, cst, _ = oracle_subcalls(omech9, sub, hb["dt"], hb["n_sub"])
        gst = gb["status"].cpu().numpy()[pick]
        assert np.array_equal(gst, cst)
        gall.append(np.ascontiguousarray(gb["state"].cpu().numpy()[:, pick]))
        call.append(c)
        tight_in += [(sub[:, j:j + 1], hb["dt"], hb["n_sub"]) for j in range(len(pick))]
    g.close()

    def rerun(idx):
        gg, cc = [], []
        for j in idx:
            st, dt, n_sub = tight_in[j]
            gt = to_gpu(st)
            cg.chem_integrate_batched(gm9, [dict(state=gt, dt=dt, n_sub=n_sub)],
                                      cg.make_opts(rtol=1e-11, atol=1e-14, max_steps=2000000))
            c2, _, _ = oracle_subcalls(omech9, np.ascontiguousarray(st), dt, n_sub, rtol=1e-11,
                                       atol=1e-14, max_steps=2000000)
            gg.append(gt.cpu().numpy())
            cc.append(c2)
        return np.hstack(gg), np.hstack(cc)
    check_flagged(np.hstack(gall), np.hstack(call), 9, "amr", rerun,
                  f"full AMR ({launch} launch), sampled")


@pytest.mark.parametrize("mode", [1, 2, 3])
@pytest.mark.parametrize("block,chunk,tail", [(512, 8, 32), (256, 2, 16), (128, 1, -1)])
def test_pool_order_changes_no_result(cg, gm9, mech9_path, block, chunk, tail, mode):
    """Dealing the hot cells over the first claims (pool_order 1), grouping
    the cells by NASA-7 range (pool_order 2) or, with a hand-off point,
    leaving the cells below the range switch to the end of the resumption
    (pool_order 3) moves cells between blocks and launches and in time,
    never their arithmetic: state, status and counts are bitwise those of
    the laid-out order, on the first call (order from temperature) and on a
    second call (order from the step hints the first one wrote).  The field
    is larger than one round of claims, so the order is really dealt."""
    import torch
    from gpu_common import run_gpu
    s0, hot = wl.front_2d(mech9_path, nx=512, ny=512, seed=61)
    kw = dict(block_size=block, chunk_steps=chunk, tail_steps=tail)
    off1 = run_gpu(gm9, s0, wl.DT_FLOW, pool_order=-1, **kw)
    on1 = run_gpu(gm9, s0, wl.DT_FLOW, pool_order=mode, **kw)
    assert all(np.array_equal(x, y) for x, y in zip(off1, on1))
    s1 = off1[0]                                   # carries the hints of the first call
    off2 = run_gpu(gm9, s1, wl.DT_FLOW, pool_order=-1, **kw)
    on2 = run_gpu(gm9, s1, wl.DT_FLOW, pool_order=mode, **kw)
    assert all(np.array_equal(x, y) for x, y in zip(off2, on2))


def test_range_order_on_scattered_temperatures(cg, gm9, mech9_path):
    """On a stress field (T scattered over 900-2800 K, so most 64-cell waves
    of the laid-out order straddle the 1000 K range switch and evaluate both
    sets of NASA-7 polynomials) grouping by range gives bitwise the laid-out
    result, also in a captured graph replayed twice; an unknown order mode
    is refused."""
    import torch
    from gpu_common import run_gpu
    s0 = wl.stress_3d(mech9_path, shape=(64, 64, 16), seed=63)
    assert 0.02 < np.mean(s0[0] < 1000.0) < 0.2
    kw = dict(block_size=256, chunk_steps=2, tail_steps=64)
    off = run_gpu(gm9, s0, wl.DT_FLOW, pool_order=-1, **kw)
    on = run_gpu(gm9, s0, wl.DT_FLOW, pool_order=2, **kw)
    assert all(np.array_equal(x, y) for x, y in zip(off, on))
    # the cells below the switch left to the end of the resumption, which
    # takes the whole tail list with a cap of one cell per CU (against the
    # laid-out order with the same cap: the cooperative kernel, which takes
    # shorter lists, sums in another order)
    off1 = run_gpu(gm9, s0, wl.DT_FLOW, pool_order=-1, tail_cap=1, **kw)
    on3 = run_gpu(gm9, s0, wl.DT_FLOW, pool_order=3, tail_cap=1, **kw)
    assert all(np.array_equal(x, y) for x, y in zip(off1, on3))
    st = torch.from_numpy(s0.copy()).cuda()
    g = cg.chem_graph_capture_batched(gm9, [dict(state=st, dt=wl.DT_FLOW)],
                                      cg.make_opts(pool_order=2, **kw))
    for rep in range(2):
        st.copy_(torch.from_numpy(s0))
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(st.cpu().numpy(), off[0]), f"replay {rep}"
    g.close()
    with pytest.raises(cg.ChemError) as e:
        cg.chem_integrate(gm9, st, wl.DT_FLOW, cg.make_opts(pool_order=4))
    assert e.value.code == -1


def test_pool_order_batched_and_graph(cg, gm9, mech9_path):
    """The same with boxes of three levels (sub-calls, own dt) in one batched
    call and in a captured graph replayed several times."""
    import torch
    hier = wl.amr_hierarchy(mech9_path, seed=62, boxes_per_level=(2, 3, 4), edges=(32, 48, 64))
    ncells = sum(b["state"].shape[1] for b in hier)
    assert ncells > 512 * 256
    off = gpu_boxes(hier)
    cg.chem_integrate_batched(gm9, off, cg.make_opts(pool_order=-1))
    on = gpu_boxes(hier)
    cg.chem_integrate_batched(gm9, on, cg.make_opts(pool_order=1))
    torch.cuda.synchronize()
    for x, y in zip(off, on):
        assert torch.equal(x["state"], y["state"]) and torch.equal(x["counts"], y["counts"])
        assert torch.equal(x["status"], y["status"])
    boxes = gpu_boxes(hier)
    pristine = [b["state"].clone() for b in boxes]
    g = cg.chem_graph_capture_batched(gm9, boxes, cg.make_opts(pool_order=1))
    for rep in range(3):
        for b, p in zip(boxes, pristine):
            b["state"].copy_(p)
        g.launch()
        torch.cuda.synchronize()
        for b, e in zip(boxes, off):
            assert torch.equal(b["state"], e["state"]), f"replay {rep}"
    g.close()


def test_kernel_timing_reports_each_launch(cg, gm9, mech9_path):
    """Per-kernel timing: refused before any timed call; after one, the
    persistent, tail-sort, cooperative and resumption durations are reported
    (the cooperative kernel ran, the list being under the cap); timing
    changes no result."""
    from gpu_common import run_gpu
    s0, hot = wl.front_2d(mech9_path, nx=256, ny=256, seed=71)
    kw = dict(block_size=256, chunk_steps=1, tail_steps=8, tail_cap=-1)
    cg.chem_set_kernel_timing(gm9, True)
    with pytest.raises(cg.ChemError):
        cg.chem_kernel_times(gm9)
    on = run_gpu(gm9, s0, wl.DT_FLOW, **kw)
    kt = cg.chem_kernel_times(gm9)
    st = cg.chem_tail_stats(gm9)
    cg.chem_set_kernel_timing(gm9, False)
    off = run_gpu(gm9, s0, wl.DT_FLOW, **kw)
    assert all(np.array_equal(x, y) for x, y in zip(on, off))
    assert set(kt) == {"persistent", "tail_sort", "coop", "resume", "total"}
    assert all(v >= 0.0 for v in kt.values())
    assert kt["persistent"] > 0.0 and kt["coop"] > 0.0
    assert abs(kt["total"] - (kt["persistent"] + kt["tail_sort"] + kt["coop"] + kt["resume"])) < 0.05
    assert st["cooperative"] == st["handed_over"] > 0      # no cap: it takes the whole list
    assert st["cooperative_steps"] > 0


def test_front_field_in_the_timed_launch(cg, omech9, mech9_path):
    """The 1024 x 1024 front field exactly as the benchmark times it: the
    committed launch cache (read from a copy, which must come back
    unchanged: a hit, no tuning), the workspace reserved, the one-box
    batched call captured in a graph and replayed three times from the
    pristine field.  Every replay equals the eager batched call bitwise, the
    eager call equals a plain call with the tuned launch spelled out, and
    that launch meets the parity bar against the oracle on every hot cell
    and a seeded sample of 20,000 cold cells."""
    import shutil
    import torch
    from gpu_common import assert_parity, run_gpu
    s0, hot = wl.front_2d(mech9_path)
    n = s0.shape[1]
    fd, cache = tempfile.mkstemp(suffix=".json")
    os.close(fd)
    shutil.copy(os.path.join(os.path.dirname(cg.__file__), "tuning_gfx950.json"), cache)
    before = open(cache).read()
    m = cg.chem_mech_load(mech9_path)
    try:
        cg.chem_workspace_reserve(m, n)
        base = cg.make_opts(rtol=wl.RTOL, atol=wl.ATOL)
        pristine = to_gpu(s0)
        st = pristine.clone()
        tb = cg.chem_autotune(m, [dict(state=st, dt=wl.DT_FLOW)], base, reps=3, cache_path=cache)
        assert open(cache).read() == before
        assert torch.equal(st, pristine)
        cg.chem_integrate_batched(m, [dict(state=st, dt=wl.DT_FLOW)], base)
        torch.cuda.synchronize()
        eager = st.cpu().numpy()
        g = cg.chem_graph_capture_batched(m, [dict(state=st, dt=wl.DT_FLOW)], base)
        try:
            for rep in range(3):
                st.copy_(pristine)
                g.launch()
                torch.cuda.synchronize()
                assert np.array_equal(st.cpu().numpy(), eager), f"replay {rep}"
        finally:
            g.close()
    finally:
        m.close()
        os.unlink(cache)
    launch = dict(rtol=wl.RTOL, atol=wl.ATOL, block_size=tb.block_size,
                  chunk_steps=tb.chunk_steps, tail_steps=tb.tail_steps,
                  tail_cap=tb.tail_cap, pool_order=tb.pool_order)
    gm = cg.chem_mech_load(mech9_path)
    assert np.array_equal(run_gpu(gm, s0, wl.DT_FLOW, **launch)[0], eager)
    rng = np.random.Generator(np.random.PCG64(79))
    idx = np.concatenate([np.where(hot)[0],
                          rng.choice(np.where(~hot)[0], 20000, replace=False)])
    assert_parity(gm, omech9, s0, wl.DT_FLOW, idx=idx, label="front 1024^2, timed launch",
                  budget="front_hot", **launch)
    gm.close()
