"""GPU parity: the HIP integrator (through the C ABI) against the CPU oracle on
identical seeded inputs.  Bar (one flow step): |gpu - cpu| <= 1e-8 |cpu| on T
and on each Y_k (+1e-13 floor on Y); fixed-step test mode <= 1e-12."""
import os
import tempfile

import numpy as np
import pytest

import oracle
from paper_2506_02602_amd import workloads as wl

from gpu_common import (assert_parity, max_rel, parity_violations, run_gpu, to_gpu,
                        tuned_launch)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def chemgpu():
    from paper_2506_02602_amd import chemgpu as c
    return c


@pytest.fixture(scope="module")
def gmech9(chemgpu, mech9_path):
    return chemgpu.chem_mech_load(mech9_path)


@pytest.fixture(scope="module")
def gmech32(chemgpu, mech32_path):
    return chemgpu.chem_mech_load(mech32_path)


def _oracle_run(om, state, dt, **kw):
    s = state.copy()
    st, cnt = om.integrate(s, dt, **kw)
    return s, st, cnt


def _report(name, gpu, cpu, ns):
    eT, eY = max_rel(gpu, cpu, ns)
    print(f"[parity] {name}: max rel err T {eT:.3e}, Y {eY:.3e}", flush=True)


def test_mech_query(gmech9, gmech32):
    assert (gmech9.n_species, gmech9.n_reactions) == (9, 21)
    assert (gmech32.n_species, gmech32.n_reactions) == (32, 150)


@pytest.mark.parametrize("chunk", [-1, 0, 1, 7])
def test_uniform_cells_all(gmech9, omech9, mech9_path, chunk):
    """4096 independent cells, T ~ U[1000, 1600] K, 1 atm: every cell."""
    s0 = wl.cells_uniform(mech9_path)
    g, gst, gcn = run_gpu(gmech9, s0, wl.DT_FLOW, chunk_steps=chunk)
    c, cst, ccn = _oracle_run(omech9, s0, wl.DT_FLOW)
    _report(f"cells_uniform chunk={chunk}", g, c, 9)
    assert np.array_equal(gst, cst)
    assert np.array_equal(gcn, ccn)
    assert not parity_violations(g, c, 9).any()
    assert np.allclose(g[11], c[11], rtol=1e-6)        # next-step hint
    assert np.array_equal(g[10], s0[10])                # rho untouched


def _hot_cells(path, n, seed):
    s, hot = wl.front_2d(path, nx=256, ny=256, seed=seed, band=10)
    idx = np.where(hot)[0][:n]
    return np.ascontiguousarray(s[:, idx])


@pytest.mark.parametrize("name", ["mech9", "mech32"])
def test_cold_cells_down_to_200K(request, name):
    """Cells from 200 K to 400 K (the low end of the NASA-7 fits, where the
    equilibrium constants are most extreme: the reverse rates' per-species
    factors are range-checked from 200 K up), over one flow step and over a
    thousand flow steps' worth of time: every cell OK and at the parity bar."""
    gm = request.getfixturevalue(f"g{name}")
    om = request.getfixturevalue(f"o{name}")
    path = request.getfixturevalue(f"{name}_path")
    s0 = wl.stress_3d(path, shape=(16, 16, 2), seed=8)
    n = s0.shape[1]
    names, W = wl.read_species(path)
    T = np.linspace(200.0, 400.0, n)
    p = np.full(n, wl.P_ATM)
    s0[0] = T
    s0[len(names) + 1] = wl.density(T, p, s0[1:len(names) + 1], W)
    for dt in (wl.DT_FLOW, 1e-4):
        g, gst, _ = run_gpu(gm, s0, dt)
        c, cst, _ = _oracle_run(om, s0, dt)
        assert (gst == 0).all() and np.array_equal(gst, cst)
        assert np.isfinite(g).all()
        assert not parity_violations(g, c, om.ns).any(), dt


@pytest.mark.parametrize("chunk", [-1, 4])
def test_hot_front_cells(gmech9, omech9, mech9_path, chunk):
    """Stiff front cells (1500-3000 K, 5-30 atm): ~50 adaptive steps each."""
    s0 = _hot_cells(mech9_path, 3000, seed=31)
    assert_parity(gmech9, omech9, s0, wl.DT_FLOW, label=f"hot front chunk={chunk}",
                  budget="front_hot", chunk_steps=chunk)


def test_fixed_step_mode_tight(gmech9, omech9, mech9_path):
    s0 = _hot_cells(mech9_path, 512, seed=32)
    g, gst, gcn = run_gpu(gmech9, s0, wl.DT_FLOW, fixed_steps=400)
    c, _, ccn = _oracle_run(omech9, s0, wl.DT_FLOW, fixed_steps=400)
    _report("fixed 400 steps", g, c, 9)
    assert (gst == 0).all() and (gcn[0] == 400).all()
    assert not parity_violations(g, c, 9, rtol=1e-12, floor_y=1e-15).any()


def test_isomer_closed_form(chemgpu, isomer_path):
    """A <-> B, kf = kr = k = 2e7 /s: c_A - c_B decays as exp(-2 k t), T fixed."""
    m = chemgpu.chem_mech_load(isomer_path)
    n = 300
    rng = np.random.Generator(np.random.PCG64(5))
    YA = rng.uniform(0.0, 1.0, n)
    T = rng.uniform(800.0, 2000.0, n)
    names, W = wl.read_species(isomer_path)
    Y = np.stack([YA, 1.0 - YA])
    rho = wl.density(T, np.full(n, wl.P_ATM), Y, W)
    s0 = wl.pack(T, Y, rho)
    g, gst, _ = run_gpu(m, s0, 1e-7, rtol=1e-12, atol=1e-16)
    assert (gst == 0).all()
    expect = (Y[0] - Y[1]) * np.exp(-2 * 2.0e7 * 1e-7)
    # error budget of an rtol 1e-12 integration on O(1) mass fractions
    assert np.abs((g[1] - g[2]) - expect).max() < 2e-11
    assert np.allclose(g[0], T, rtol=1e-13)


def test_ragged_sizes_and_padding(gmech9, omech9, mech9_path, chemgpu):
    """n not a multiple of any block; ld > n: padding columns untouched."""
    import torch
    s0 = wl.cells_uniform(mech9_path, n=1000, seed=9)
    ld = 1037
    pad = np.full((12, ld), 123.0)
    pad[:, :1000] = s0
    t = torch.from_numpy(pad).cuda()
    st = torch.zeros(1000, dtype=torch.int32, device="cuda")
    chemgpu.chem_integrate(gmech9, t, wl.DT_FLOW, chemgpu.make_opts(block_size=192),
                           status=st, n_cells=1000)
    torch.cuda.synchronize()
    out = t.cpu().numpy()
    assert (out[:, 1000:] == 123.0).all()
    c, cst, _ = _oracle_run(omech9, s0, wl.DT_FLOW)
    assert not parity_violations(np.ascontiguousarray(out[:, :1000]), c, 9).any()
    # n = 0 is a no-op
    chemgpu.chem_integrate(gmech9, t, wl.DT_FLOW, n_cells=0)


def test_status_paths(gmech9, omech9, mech9_path):
    s0 = _hot_cells(mech9_path, 70, seed=33)
    s0[3, 5] = np.nan
    s0[0, 6] = np.inf
    g, gst, gcn = run_gpu(gmech9, s0, wl.DT_FLOW, max_steps=3)
    c, cst, ccn = _oracle_run(omech9, s0, wl.DT_FLOW, max_steps=3)
    assert np.array_equal(gst, cst)
    assert gst[5] == 2 and gst[6] == 2
    assert np.isnan(g[3, 5]) and np.isinf(g[0, 6])
    assert np.array_equal(gcn, ccn)
    ok = np.ones(70, bool)
    ok[[5, 6]] = False
    assert not parity_violations(g[:, ok], c[:, ok], 9).any()


def test_invalid_arguments(gmech9, chemgpu):
    import torch
    s = torch.zeros((12, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(chemgpu.ChemError) as e:
        chemgpu.chem_integrate(gmech9, s, 0.0)
    assert e.value.code == -1
    with pytest.raises(chemgpu.ChemError) as e:
        chemgpu.chem_integrate(gmech9, s, 1e-7, n_cells=9)
    assert e.value.code == -1
    with pytest.raises(chemgpu.ChemError) as e:
        chemgpu.chem_integrate(gmech9, s, 1e-7, chemgpu.make_opts(block_size=100))
    assert e.value.code == -1


def test_unknown_mechanism_rejected(chemgpu, mech9_path):
    txt = open(mech9_path).read().replace("name mech9", "name other")
    fd, p = tempfile.mkstemp(suffix=".mech")
    with os.fdopen(fd, "w") as f:
        f.write(txt)
    try:
        with pytest.raises(chemgpu.ChemError) as e:
            chemgpu.chem_mech_load(p)
        assert e.value.code == -5
    finally:
        os.unlink(p)


def test_front_field_sampled(gmech9, omech9, mech9_path):
    """The full 1024 x 1024 front field in one call; the oracle checks every hot
    cell and a seeded sample of cold cells."""
    s0, hot = wl.front_2d(mech9_path)
    rng = np.random.Generator(np.random.PCG64(77))
    idx = np.concatenate([np.where(hot)[0],
                          rng.choice(np.where(~hot)[0], 20000, replace=False)])
    assert_parity(gmech9, omech9, s0, wl.DT_FLOW, idx=idx, label="front 1024^2 sampled",
                  budget="front_hot")


def test_stress_mech32_sampled(gmech32, omech32, mech32_path):
    """32 species / 150 reactions on a slab of the independent-T,p stress field."""
    s0 = wl.stress_3d(mech32_path, shape=(64, 64, 2), seed=4)
    idx = np.arange(0, s0.shape[1], 7)
    assert_parity(gmech32, omech32, s0, wl.DT_FLOW, idx=idx, label="stress mech32 sampled",
                  budget="stress32")


def test_stress_mech9_sampled(gmech9, omech9, mech9_path):
    """The 9-species mechanism on the same kind of independent-T,p field."""
    s0 = wl.stress_3d(mech9_path, shape=(64, 64, 4), seed=4)
    idx = np.arange(0, s0.shape[1], 5)
    assert_parity(gmech9, omech9, s0, wl.DT_FLOW, idx=idx, label="stress mech9 sampled",
                  budget="stress9")


@pytest.mark.parametrize("name,stride", [("mech9", 997), ("mech32", 4099)])
def test_stress_field_full_size_in_the_tuned_launch(chemgpu, request, name, stride):
    """The whole 256 x 256 x 64 stress field (4,194,304 cells) in one call
    with the launch the committed tuning cache holds for it (read from a
    copy that must come back unchanged: a hit, no tuning); every stride-th
    cell against the oracle."""
    gm = request.getfixturevalue(f"g{name}")
    om = request.getfixturevalue(f"o{name}")
    path = request.getfixturevalue(f"{name}_path")
    s0 = wl.stress_3d(path)
    g = to_gpu(s0)
    launch = tuned_launch(gm, [dict(state=g, dt=wl.DT_FLOW)], wl.RTOL, wl.ATOL)
    del g
    idx = np.arange(0, s0.shape[1], stride)
    assert_parity(gm, om, s0, wl.DT_FLOW, idx=idx,
                  label=f"stress 256x256x64 {name}, tuned launch",
                  budget="stress9" if name == "mech9" else "stress32", **launch)


@pytest.mark.parametrize("tail", [-1, 0, 5])
def test_chunk_and_block_invariance(gmech9, mech9_path, tail):
    """Compaction only moves cells between lanes, and a cell moves to the
    cooperative kernel after exactly tail_steps steps: for a given kernel
    build the results are bitwise identical for any chunk length or block
    size.  Without the cooperative kernel the uncompacted kernel agrees to
    rounding."""
    s0 = _hot_cells(mech9_path, 2000, seed=34)
    ref, rst, rcn = run_gpu(gmech9, s0, wl.DT_FLOW, chunk_steps=8, block_size=128, tail_steps=tail)
    for chunk, block in [(1, 64), (3, 128), (16, 256), (64, 192), (5, 512)]:
        g, gst, gcn = run_gpu(gmech9, s0, wl.DT_FLOW, chunk_steps=chunk, block_size=block,
                              tail_steps=tail)
        assert np.array_equal(g, ref) and np.array_equal(gst, rst) and np.array_equal(gcn, rcn)
    if tail < 0:
        g, gst, gcn = run_gpu(gmech9, s0, wl.DT_FLOW, chunk_steps=-1, block_size=256)
        assert np.array_equal(gst, rst) and np.array_equal(gcn, rcn)
        assert not parity_violations(g, ref, 9, rtol=1e-12, floor_y=1e-16).any()


@pytest.mark.parametrize("tail", [1, 8, 32])
def test_tail_cells_match_oracle(gmech9, omech9, mech9_path, tail):
    """Hot front cells finished by the cooperative kernel (several lanes per
    cell, table-driven rate law) after `tail` per-lane steps."""
    s0 = _hot_cells(mech9_path, 3000, seed=35)
    assert_parity(gmech9, omech9, s0, wl.DT_FLOW, label=f"hot front tail={tail}",
                  budget="front_hot", tail_steps=tail)


@pytest.mark.parametrize("tiles,cap", [(2, 0), (2, 1), (48, 0)])
def test_long_tail_list_resumes_per_lane(chemgpu, gmech9, mech9_path, tiles, cap):
    """More handed-over cells than the cooperative kernel takes (default 64
    per CU, or 1): the list is resumed one cell per lane, bitwise the result
    of never handing over, and the cooperative kernel takes no step.  Two
    copies of the front's hot band (~42,000 cells) leave the longest cell
    far above the work per lane, so the resumption runs with wave
    priorities; 48 copies (~1 M cells) put the work per lane above the
    longest cell, where it runs without them."""
    import torch
    s0, hot = wl.front_2d(mech9_path, nx=1024, ny=1024, seed=37)
    s1 = np.ascontiguousarray(np.tile(s0[:, hot], (1, tiles)))
    ref, rst, rcn = run_gpu(gmech9, s1, wl.DT_FLOW, tail_steps=-1)
    # the two regimes, in actual steps after the hand-off over the lanes of
    # two waves per SIMD
    left = np.maximum(rcn.sum(axis=0).astype(np.int64) - 1, 0)
    lanes = torch.cuda.get_device_properties(0).multi_processor_count * 4 * 2 * 64
    print(f"[resume] {s1.shape[1]} cells: longest {left.max()} steps left, "
          f"{left.sum() / lanes:.1f} per lane", flush=True)
    if tiles == 2:
        assert left.max() > 4 * left.sum() / lanes
    else:
        assert left.sum() / lanes > left.max()
    chemgpu.chem_set_kernel_timing(gmech9, True)
    try:
        g, gst, gcn = run_gpu(gmech9, s1, wl.DT_FLOW, tail_steps=1, tail_cap=cap)
        stats = chemgpu.chem_tail_stats(gmech9)
    finally:
        chemgpu.chem_set_kernel_timing(gmech9, False)
    assert np.array_equal(g, ref) and np.array_equal(gst, rst) and np.array_equal(gcn, rcn)
    assert 0 < stats["handed_over"] <= s1.shape[1]
    assert stats["cooperative"] == 0 and stats["cooperative_steps"] == 0


def test_long_tail_list_without_cap(gmech9, omech9, mech9_path):
    """With no cap the cooperative kernel takes a list of ~42,000 cells (far
    more than the groups resident on the chip, so groups claim cell after
    cell): every cell is finished, and a seeded sample matches the oracle."""
    s0, hot = wl.front_2d(mech9_path, nx=1024, ny=1024, seed=37)
    s1 = np.ascontiguousarray(np.tile(s0[:, hot], (1, 2)))
    g, gst, gcn = run_gpu(gmech9, s1, wl.DT_FLOW, tail_steps=1, tail_cap=-1)
    assert (gst == 0).all() and (gcn[0] >= 1).all()
    rng = np.random.Generator(np.random.PCG64(38))
    idx = rng.choice(s1.shape[1], 1500, replace=False)
    assert_parity(gmech9, omech9, s1, wl.DT_FLOW, idx=idx, label="tail list without cap",
                  budget="front_hot", tail_steps=1, tail_cap=-1)


def test_tail_list_at_the_cap(chemgpu, gmech9, omech9, mech9_path):
    """The finisher of the tail list is chosen by its length alone: with a
    cap of one cell per CU, a list of exactly as many cells as CUs goes to
    the cooperative kernel (checked against the oracle) and one cell more to
    the per-lane resumption (bitwise the result of never handing over)."""
    import torch
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    s0, hot = wl.front_2d(mech9_path, nx=1024, ny=1024, seed=37)
    hs = np.ascontiguousarray(s0[:, hot])
    # cells still stepping after one step are handed over with tail_steps=1
    _, _, cn = run_gpu(gmech9, hs, wl.DT_FLOW, tail_steps=-1)
    long = np.flatnonzero(cn.sum(axis=0) >= 2)
    assert long.size > n_cu + 1
    for extra in (0, 1):
        sel = np.ascontiguousarray(hs[:, long[:n_cu + extra]])
        ref, rst, rcn = run_gpu(gmech9, sel, wl.DT_FLOW, tail_steps=-1)
        chemgpu.chem_set_kernel_timing(gmech9, True)
        try:
            g, gst, gcn = run_gpu(gmech9, sel, wl.DT_FLOW, tail_steps=1, tail_cap=1)
            stats = chemgpu.chem_tail_stats(gmech9)
        finally:
            chemgpu.chem_set_kernel_timing(gmech9, False)
        print(f"[tail cap] {n_cu + extra} cells: {stats}", flush=True)
        assert stats["handed_over"] == n_cu + extra
        assert (gst == 0).all()
        if extra == 0:
            assert stats["cooperative"] == n_cu and stats["cooperative_steps"] > 0
            assert_parity(gmech9, omech9, sel, wl.DT_FLOW, label="tail list at the cap",
                          budget="front_hot", tail_steps=1, tail_cap=1)
        else:
            assert stats["cooperative"] == 0 and stats["cooperative_steps"] == 0
            assert np.array_equal(g, ref) and np.array_equal(gst, rst) and np.array_equal(gcn, rcn)


def test_tail_mech32(gmech32, omech32, mech32_path):
    """32 species / 150 reactions through the cooperative kernel (a full wave
    per cell, three reaction rounds per lane)."""
    s0 = wl.stress_3d(mech32_path, shape=(32, 32, 1), seed=6)
    assert_parity(gmech32, omech32, s0, wl.DT_FLOW, label="stress mech32 tail=2",
                  budget="stress32", tail_steps=2)


def test_tail_status_paths_and_isomer(chemgpu, gmech9, omech9, mech9_path, isomer_path):
    """Step budget exhausted inside the cooperative kernel; non-finite cells
    never reach it; the isomer closed form through it."""
    s0 = _hot_cells(mech9_path, 70, seed=36)
    s0[3, 5] = np.nan
    g, gst, gcn = run_gpu(gmech9, s0, wl.DT_FLOW, max_steps=6, tail_steps=2)
    c, cst, ccn = _oracle_run(omech9, s0, wl.DT_FLOW, max_steps=6)
    assert np.array_equal(gst, cst) and gst[5] == 2 and (gst == 1).sum() > 10
    ok = np.ones(70, bool)
    ok[5] = False
    assert np.array_equal(gcn[:, ok], ccn[:, ok])
    assert not parity_violations(g[:, ok], c[:, ok], 9).any()
    m = chemgpu.chem_mech_load(isomer_path)
    rng = np.random.Generator(np.random.PCG64(6))
    n = 200
    YA = rng.uniform(0.0, 1.0, n)
    T = rng.uniform(800.0, 2000.0, n)
    names, W = wl.read_species(isomer_path)
    Y = np.stack([YA, 1.0 - YA])
    s1 = wl.pack(T, Y, wl.density(T, np.full(n, wl.P_ATM), Y, W))
    g1, gst1, gcn1 = run_gpu(m, s1, 1e-7, rtol=1e-12, atol=1e-16, tail_steps=1)
    assert (gst1 == 0).all() and (gcn1[0] > 1).all()
    expect = (Y[0] - Y[1]) * np.exp(-2 * 2.0e7 * 1e-7)
    assert np.abs((g1[1] - g1[2]) - expect).max() < 2e-11
    assert np.allclose(g1[0], T, rtol=1e-13)


def test_every_cell_of_a_large_field_is_integrated(gmech9, omech9, mech9_path):
    """2,097,152 cells = 512 copies of 4096 distinct cells: every cell takes at
    least one accepted step, every copy ends identical, and equals the oracle
    (regression for a pool-refill bug that stopped blocks after one chunk)."""
    import torch
    from paper_2506_02602_amd import chemgpu
    base = wl.cells_uniform(mech9_path, n=4096, seed=12)
    base[0, :512] = np.linspace(1800.0, 2600.0, 512)          # some cells need many steps
    big = torch.from_numpy(np.ascontiguousarray(np.tile(base, (1, 512)))).cuda()
    n = big.shape[1]
    st = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    cn = torch.zeros(2 * n, dtype=torch.int32, device="cuda")
    chemgpu.chem_integrate(gmech9, big, wl.DT_FLOW, status=st, counts=cn)
    torch.cuda.synchronize()
    assert (st == 0).all()
    assert (cn[:n] >= 1).all()
    out = big.cpu().numpy().reshape(12, 512, 4096)
    assert (out == out[:, :1, :]).all()
    c = base.copy()
    omech9.integrate(c, wl.DT_FLOW)
    assert not parity_violations(np.ascontiguousarray(out[:, 0, :]), c, 9).any()


def test_rate_exponential_within_one_ulp(chemgpu):
    """The device exponential used for k_f and k_r against numpy's (itself
    within an ulp of e^x): at most 1 ulp apart on [-745, 709], exact at 0,
    inf above the overflow threshold, 0 below underflow, NaN through."""
    import torch
    rng = np.random.Generator(np.random.PCG64(11))
    x = np.concatenate([rng.uniform(-745.0, 709.0, 2_000_000), rng.uniform(-60.0, 60.0, 2_000_000),
                        [0.0, 1.0, -1.0, 709.7, -708.0, 800.0, -800.0, np.nan]])
    y = chemgpu.chem_eval_exp(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = np.exp(x)
    fin = np.isfinite(ref) & (ref > 1e-300)
    ulp = np.abs(y[fin] - ref[fin]) / np.spacing(ref[fin])
    print(f"[exp] max {ulp.max():.2f} ulp, mean {ulp.mean():.4f}", flush=True)
    assert ulp.max() <= 2.0 and ulp.mean() < 0.2
    assert y[-8] == 1.0 and y[-3] == np.inf and y[-2] == 0.0 and np.isnan(y[-1])


def _ulps(y, x, fn):
    """|y - fn(x)| in units of the last place of the double nearest the
    extended-precision reference."""
    ref = fn(x.astype(np.longdouble))
    return (np.abs(y.astype(np.longdouble) - ref) / np.spacing(ref.astype(np.float64))).astype(
        np.float64)


def test_table_exponential_within_one_ulp(chemgpu):
    """The cooperative kernel's rate exponential (2^(j/64) from an LDS table,
    degree-6 polynomial) against an extended-precision reference: its error
    is the table entry's rounding plus one final rounding, so at most about
    1 ulp on [-745, 709] (asserted with 5 % slack); exact at 0, inf above the
    overflow threshold, 0 below underflow, NaN through."""
    import torch
    rng = np.random.Generator(np.random.PCG64(14))
    x = np.concatenate([rng.uniform(-708.0, 709.0, 2_000_000), rng.uniform(-60.0, 60.0, 2_000_000),
                        rng.uniform(-0.02, 0.02, 500_000),
                        [0.0, 1.0, -1.0, 709.7, -708.0, 800.0, -800.0, np.nan]])
    y = chemgpu.chem_eval_math("exp_tab", torch.from_numpy(x).cuda()).cpu().numpy()
    fin = np.isfinite(x) & (x > -708.0) & (x < 709.7)
    u = _ulps(y[fin], x[fin], np.exp)
    print(f"[exp_tab] max {u.max():.3f} ulp, mean {u.mean():.4f}", flush=True)
    assert u.max() <= 1.05 and u.mean() < 0.35
    assert y[-8] == 1.0 and y[-3] == np.inf and y[-2] == 0.0 and np.isnan(y[-1])
    assert np.isfinite(y[-5])


def test_log_within_one_ulp(chemgpu):
    """ln T for the rate constants and the Gibbs energies: at most 1 ulp from
    an extended-precision reference over the whole positive range and densely
    over temperatures, exact at 1, NaN for 0, negative and NaN inputs."""
    import torch
    rng = np.random.Generator(np.random.PCG64(13))
    x = np.concatenate([np.exp(rng.uniform(-700.0, 700.0, 2_000_000)),
                        rng.uniform(100.0, 5000.0, 2_000_000),
                        rng.uniform(0.70, 1.45, 500_000),
                        [1.0, 2.0, 0.5, np.sqrt(0.5), 0.0, -1.0, np.nan]])
    y = chemgpu.chem_eval_math("log_atanh", torch.from_numpy(x).cuda()).cpu().numpy()
    u = _ulps(y[:-3], x[:-3], np.log)
    print(f"[log_atanh] max {u.max():.3f} ulp, mean {u.mean():.4f}", flush=True)
    assert u.max() <= 1.0 and u.mean() < 0.3
    assert y[-7] == 0.0 and y[-6] == np.log(2.0) and np.isnan(y[-3:]).all()


def test_eval_math_rejects_unknown_function(chemgpu):
    import torch
    x = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(chemgpu.ChemError):
        chemgpu._check(chemgpu._lib.chem_eval_math(7, x.data_ptr(), x.data_ptr(), 4, None),
                       "chem_eval_math")
