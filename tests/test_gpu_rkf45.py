"""The full-storage comparison scheme (Runge-Kutta-Fehlberg 4(5), all six
stage vectors kept) on the GPU against the oracle's RKF45 path: the same
parity bar as the low-storage scheme.  Its registers, occupancy and speed
against the two-register scheme are the measurement (bench --scheme)."""
import numpy as np
import pytest

from paper_2506_02602_amd import workloads as wl

from gpu_common import assert_parity, parity_violations, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gm9(mech9_path):
    from paper_2506_02602_amd import chemgpu
    return chemgpu.chem_mech_load(mech9_path)


def _hot_cells(path, n, seed):
    s, hot = wl.front_2d(path, nx=256, ny=256, seed=seed, band=10)
    return np.ascontiguousarray(s[:, np.where(hot)[0][:n]])


@pytest.mark.parametrize("chunk", [-1, 4])
def test_rkf45_uniform_cells_all(gm9, omech9, mech9_path, chunk):
    s0 = wl.cells_uniform(mech9_path)
    g, gst, gcn = run_gpu(gm9, s0, wl.DT_FLOW, chunk_steps=chunk, scheme="rkf45")
    c = s0.copy()
    cst, ccn = omech9.integrate(c, wl.DT_FLOW, scheme="rkf45")
    assert np.array_equal(gst, cst) and np.array_equal(gcn, ccn)
    assert not parity_violations(g, c, 9).any()


def test_rkf45_hot_front_cells(gm9, omech9, mech9_path):
    s0 = _hot_cells(mech9_path, 3000, seed=41)
    assert_parity(gm9, omech9, s0, wl.DT_FLOW, label="rkf45 hot front", budget="front_hot_rkf45",
                  scheme="rkf45")


def test_rkf45_fixed_steps_tight(gm9, omech9, mech9_path):
    s0 = _hot_cells(mech9_path, 512, seed=42)
    g, gst, gcn = run_gpu(gm9, s0, wl.DT_FLOW, fixed_steps=600, scheme="rkf45")
    c = s0.copy()
    omech9.integrate(c, wl.DT_FLOW, fixed_steps=600, scheme="rkf45")
    assert (gst == 0).all() and (gcn[0] == 600).all()
    assert not parity_violations(g, c, 9, rtol=1e-12, floor_y=1e-15).any()


def test_rkf45_mech32_sampled(omech32, mech32_path):
    from paper_2506_02602_amd import chemgpu
    m = chemgpu.chem_mech_load(mech32_path)
    s0 = wl.stress_3d(mech32_path, shape=(32, 32, 2), seed=7)
    assert_parity(m, omech32, s0, wl.DT_FLOW, idx=np.arange(0, s0.shape[1], 3),
                  label="rkf45 stress mech32", budget="stress32_rkf45", scheme="rkf45")


def test_rkf45_chunk_and_block_invariance(gm9, mech9_path):
    s0 = _hot_cells(mech9_path, 2000, seed=43)
    ref = run_gpu(gm9, s0, wl.DT_FLOW, chunk_steps=8, block_size=128, scheme="rkf45")
    for chunk, block in [(1, 64), (16, 256), (5, 512)]:
        g = run_gpu(gm9, s0, wl.DT_FLOW, chunk_steps=chunk, block_size=block, scheme="rkf45")
        assert all(np.array_equal(x, y) for x, y in zip(g, ref))


def test_rkf45_front_field_in_its_tuned_launch(gm9, omech9, mech9_path):
    """The full 1024 x 1024 front field in the launch the committed tuning
    cache holds for this scheme (the one the benchmark's scheme comparison
    times); 4,000 hot and 2,000 cold cells, seeded, against the oracle."""
    from gpu_common import to_gpu, tuned_launch
    s0, hot = wl.front_2d(mech9_path)
    g = to_gpu(s0)
    launch = tuned_launch(gm9, [dict(state=g, dt=wl.DT_FLOW)], wl.RTOL, wl.ATOL, scheme="rkf45")
    del g
    rng = np.random.Generator(np.random.PCG64(83))
    idx = np.concatenate([rng.choice(np.where(hot)[0], 4000, replace=False),
                          rng.choice(np.where(~hot)[0], 2000, replace=False)])
    assert_parity(gm9, omech9, s0, wl.DT_FLOW, idx=idx, label="rkf45 front 1024^2, tuned launch",
                  budget="front_hot_rkf45", **launch)
