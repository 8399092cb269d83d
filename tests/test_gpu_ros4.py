"""The implicit comparator (fourth-order Rosenbrock, exact generated Jacobian,
LU with partial pivoting in registers) on the GPU against the oracle's
Rosenbrock path (complex-step Jacobian, its own LU): the same parity bar as
the explicit schemes.  Its speed against the explicit scheme is the
measurement (bench --scheme ros4)."""
import math

import numpy as np
import pytest

from paper_2506_02602_amd import workloads as wl

from gpu_common import assert_parity, parity_violations, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def chemgpu():
    from paper_2506_02602_amd import chemgpu as cg
    return cg


@pytest.fixture(scope="module")
def gm9(mech9_path):
    from paper_2506_02602_amd import chemgpu
    return chemgpu.chem_mech_load(mech9_path)


def _hot_cells(path, n, seed):
    s, hot = wl.front_2d(path, nx=256, ny=256, seed=seed, band=10)
    return np.ascontiguousarray(s[:, np.where(hot)[0][:n]])


def test_ros4_fixed_steps_tight(gm9, omech9, mech9_path):
    """No controller: exactly 40 steps of the same size on both sides, so the
    results differ only by rounding in the Jacobian, the factorisation and
    the stages (1e-11 relative)."""
    s0 = _hot_cells(mech9_path, 512, seed=51)
    g, gst, gcn = run_gpu(gm9, s0, wl.DT_FLOW, fixed_steps=40, scheme="ros4")
    c = s0.copy()
    omech9.integrate(c, wl.DT_FLOW, fixed_steps=40, scheme="ros4")
    assert (gst == 0).all() and (gcn[0] == 40).all()
    assert not parity_violations(g, c, 9, rtol=1e-11, floor_y=1e-15).any()


@pytest.mark.parametrize("chunk", [-1, 4])
def test_ros4_uniform_cells_all(gm9, omech9, mech9_path, chunk):
    s0 = wl.cells_uniform(mech9_path)
    g, gst, gcn = run_gpu(gm9, s0, wl.DT_FLOW, chunk_steps=chunk, block_size=128, scheme="ros4")
    c = s0.copy()
    cst, ccn = omech9.integrate(c, wl.DT_FLOW, scheme="ros4")
    assert np.array_equal(gst, cst)
    assert not parity_violations(g, c, 9).any()


def test_ros4_hot_front_cells(gm9, omech9, mech9_path):
    s0 = _hot_cells(mech9_path, 3000, seed=52)
    assert_parity(gm9, omech9, s0, wl.DT_FLOW, label="ros4 hot front", budget="front_hot_ros4",
                  scheme="ros4", block_size=256)


def test_ros4_long_stiff_interval(gm9, omech9, mech9_path):
    """A flow step 100x longer (1e-5 s, the divergence workload's dt), where
    hot cells reach equilibrium and the explicit scheme is stability-bound:
    parity with the oracle, and fewer steps than the explicit scheme."""
    s0 = _hot_cells(mech9_path, 256, seed=53)
    assert_parity(gm9, omech9, s0, 1e-5, label="ros4 dt 1e-5", budget="front_hot_ros4_dt1e-5",
                  scheme="ros4")
    _, _, c_imp = run_gpu(gm9, s0, 1e-5, scheme="ros4")
    _, _, c_exp = run_gpu(gm9, s0, 1e-5, scheme="lsrk", tail_steps=-1)
    assert c_imp.sum() < c_exp.sum()


def test_ros4_isomer_closed_form(chemgpu, isomer_path):
    """A <-> B, c_A - c_B decays as exp(-2 k t), at k dt = 2e3 (2,000 times
    the explicit scheme's stability limit per step)."""
    m = chemgpu.chem_mech_load(isomer_path)
    names, W = wl.read_species(isomer_path)
    Y = np.array([[0.9], [0.1]])
    rho = wl.density(np.array([1400.0]), np.array([wl.P_ATM]), Y, W)[0]
    s0 = np.zeros((5, 64))
    s0[0], s0[1], s0[2], s0[3] = 1400.0, 0.9, 0.1, rho
    k, dt = 2.0e7, 1.0e-4
    g, gst, gcn = run_gpu(m, s0, dt, rtol=1e-8, atol=1e-16, scheme="ros4")
    assert (gst == 0).all() and gcn.sum(axis=0).max() < 200
    d = (g[1] - g[2]) / 0.8
    assert np.all(np.abs(d - math.exp(-2 * k * dt)) <= 20e-8)
    assert np.all(np.abs(g[0] - 1400.0) < 1e-9)


def test_ros4_rejects_unsupported(chemgpu, mech32_path, gm9, mech9_path):
    """No Jacobian is generated for 32 species (the matrix would not fit in
    registers) and the kernel is built for 256-lane blocks only: both are
    refused before any GPU work."""
    import torch
    m32 = chemgpu.chem_mech_load(mech32_path)
    s = torch.from_numpy(wl.stress_3d(mech32_path, shape=(4, 4, 1), seed=1)).cuda()
    with pytest.raises(chemgpu.ChemError) as e:
        chemgpu.chem_integrate(m32, s, wl.DT_FLOW, chemgpu.make_opts(scheme="ros4"))
    assert e.value.code == -5
    s9 = torch.from_numpy(wl.cells_uniform(mech9_path, n=64)).cuda()
    with pytest.raises(chemgpu.ChemError) as e:
        chemgpu.chem_integrate(gm9, s9, wl.DT_FLOW,
                               chemgpu.make_opts(scheme="ros4", block_size=512))
    assert e.value.code == -1


def test_ros4_batched_boxes_match_single_calls(gm9, mech9_path):
    """Boxes of two levels (own dt and sub-calls) in one batched launch give
    the per-box results of separate calls bitwise."""
    import torch
    from paper_2506_02602_amd import chemgpu
    s0 = _hot_cells(mech9_path, 700, seed=54)
    a, b = np.ascontiguousarray(s0[:, :300]), np.ascontiguousarray(s0[:, 300:])
    ga, gb = torch.from_numpy(a.copy()).cuda(), torch.from_numpy(b.copy()).cuda()
    o = chemgpu.make_opts(scheme="ros4", block_size=128, chunk_steps=2)
    chemgpu.chem_integrate_batched(gm9, [dict(state=ga, dt=1e-7), dict(state=gb, dt=5e-8, n_sub=2)], o)
    torch.cuda.synchronize()
    ra = run_gpu(gm9, a, 1e-7, scheme="ros4", block_size=128, chunk_steps=2)[0]
    hb = torch.from_numpy(b.copy()).cuda()
    chemgpu.chem_integrate(gm9, hb, 5e-8, o)
    chemgpu.chem_integrate(gm9, hb, 5e-8, o)
    torch.cuda.synchronize()
    assert np.array_equal(ga.cpu().numpy(), ra)
    assert np.array_equal(gb.cpu().numpy(), hb.cpu().numpy())


def test_ros4_front_field_in_its_tuned_launch(gm9, omech9, mech9_path):
    """The full 1024 x 1024 front field in the launch the committed tuning
    cache holds for this scheme (the one the benchmark's scheme comparison
    times); 4,000 hot and 2,000 cold cells, seeded, against the oracle."""
    from gpu_common import to_gpu, tuned_launch
    s0, hot = wl.front_2d(mech9_path)
    g = to_gpu(s0)
    launch = tuned_launch(gm9, [dict(state=g, dt=wl.DT_FLOW)], wl.RTOL, wl.ATOL, scheme="ros4")
    del g
    rng = np.random.Generator(np.random.PCG64(83))
    idx = np.concatenate([rng.choice(np.where(hot)[0], 4000, replace=False),
                          rng.choice(np.where(~hot)[0], 2000, replace=False)])
    assert_parity(gm9, omech9, s0, wl.DT_FLOW, idx=idx, label="ros4 front 1024^2, tuned launch",
                  budget="front_hot_ros4", **launch)
