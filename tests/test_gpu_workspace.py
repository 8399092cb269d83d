"""The workspace contract of the C ABI: chem_workspace_reserve (and
surrogate_reserve for the surrogate's fallback) allocate everything the
integration calls use; after them chem_integrate, chem_integrate_batched,
chem_react_conserved and surrogate_infer with fallback take no device memory,
and a call on more cells than the reservation holds returns CHEM_ECAPACITY
(-6) without touching the caller's data.  All calls go through the C ABI with
the binding's automatic reservation switched off."""
import numpy as np
import pytest

from paper_2506_02602_amd import workloads as wl

pytestmark = pytest.mark.gpu

ECAPACITY = -6


@pytest.fixture(scope="module")
def cg():
    from paper_2506_02602_amd import chemgpu
    return chemgpu


def conserved_rows(om, s):
    """Conserved rows (rho, rho u, rho v, rho w, rho E, rho Y, T, h) of a
    primitive block at rest, E from the oracle's internal energy."""
    ns = om.ns
    n = s.shape[1]
    c = np.zeros((ns + 7, n))
    rho = s[ns + 1]
    c[0] = rho
    for i in range(n):
        e, _ = om.energy(s[0, i], s[1:ns + 1, i])
        c[4, i] = rho[i] * e
    c[5:5 + ns] = rho * s[1:ns + 1]
    c[5 + ns] = s[0] * 1.01
    return c


def test_calls_past_the_reservation_fail_and_reserved_calls_allocate_nothing(cg, mech9_path,
                                                                              omech9):
    import torch
    big, small = 131072, 2048
    s0 = wl.cells_uniform(mech9_path, n=big, seed=73)
    s0[0, ::7] += 900.0                       # some stiff cells: tail list in use
    o = cg.make_opts(block_size=256, chunk_steps=2, tail_steps=2, tail_cap=-1, pool_order=2)
    m = cg.Mechanism(mech9_path, auto_reserve=False)
    sur = cg.Surrogate(m, seed=3)
    trust = (0.0, 1e-6, 1e-7, 0.05)
    try:
        st = torch.from_numpy(s0.copy()).cuda()
        cons = torch.from_numpy(conserved_rows(omech9, s0[:, :small])).cuda()
        # nothing reserved yet: every integration call refuses, data untouched
        calls = {
            "integrate": lambda x: cg.chem_integrate(m, x, wl.DT_FLOW, o),
            "batched": lambda x: cg.chem_integrate_batched(
                m, [dict(state=x, dt=wl.DT_FLOW)], o),
            "conserved": lambda x: cg.chem_react_conserved(m, cons, wl.DT_FLOW, o),
        }
        for name, fn in calls.items():
            with pytest.raises(cg.ChemError) as e:
                fn(st)
            assert e.value.code == ECAPACITY, name
        torch.cuda.synchronize()
        assert np.array_equal(st.cpu().numpy(), s0)
        cg.chem_workspace_reserve(m, big)
        # the surrogate's fallback needs its own reservation as well
        with pytest.raises(cg.ChemError) as e:
            cg.surrogate_infer(sur, m, st, wl.DT_FLOW, trust, fallback=True, opts=o)
        assert e.value.code == ECAPACITY
        cg.surrogate_reserve(sur, small)
        # first calls load every kernel
        w = st[:, :small].contiguous()
        cg.chem_integrate(m, w, wl.DT_FLOW, o)
        cg.chem_integrate_batched(m, [dict(state=w, dt=wl.DT_FLOW / 2, n_sub=2)], o)
        cg.chem_react_conserved(m, cons, wl.DT_FLOW, o)
        cg.surrogate_infer(sur, m, w, wl.DT_FLOW, trust, fallback=True, opts=o)
        torch.cuda.synchronize()
        st.copy_(torch.from_numpy(s0))
        free0 = torch.cuda.mem_get_info()[0]
        half = big // 2
        sa, sb = st[:, :half].contiguous(), st[:, half:].contiguous()
        cg.chem_integrate(m, st, wl.DT_FLOW, o)
        cg.chem_integrate_batched(m, [dict(state=sa, dt=wl.DT_FLOW),
                                      dict(state=sb, dt=wl.DT_FLOW / 2, n_sub=2)], o)
        cg.chem_react_conserved(m, cons, wl.DT_FLOW, o)
        ws = sa[:, :small].contiguous()
        cg.surrogate_infer(sur, m, ws, wl.DT_FLOW, trust, fallback=True, opts=o)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        # past the reservations: refused, nothing enqueued
        over = torch.from_numpy(wl.cells_uniform(mech9_path, n=big + 1, seed=5)).cuda()
        ref = over.clone()
        for fn in (lambda: cg.chem_integrate(m, over, wl.DT_FLOW, o),
                   lambda: cg.chem_integrate_batched(m, [dict(state=over[:, :big].contiguous(),
                                                              dt=wl.DT_FLOW),
                                                         dict(state=over[:, big:].contiguous(),
                                                              dt=wl.DT_FLOW)], o),
                   lambda: cg.surrogate_infer(sur, m, over[:, :small + 1].contiguous(),
                                              wl.DT_FLOW, trust, fallback=True, opts=o)):
            with pytest.raises(cg.ChemError) as e:
                fn()
            assert e.value.code == ECAPACITY
        torch.cuda.synchronize()
        assert torch.equal(over, ref)
        # the reserved results equal those of a handle that reserves on demand
        m2 = cg.chem_mech_load(mech9_path)
        st2 = torch.from_numpy(s0.copy()).cuda()
        cg.chem_integrate(m2, st2, wl.DT_FLOW, o)
        torch.cuda.synchronize()
        m2.close()
        full = torch.from_numpy(s0.copy()).cuda()
        cg.chem_integrate(m, full, wl.DT_FLOW, o)
        torch.cuda.synchronize()
        assert torch.equal(full, st2)
    finally:
        sur.close()
        m.close()
    with pytest.raises(cg.ChemError) as e:
        cg.chem_workspace_reserve(cg.chem_mech_load(mech9_path), -1)
    assert e.value.code == -1


def test_box_table_holds_4096_boxes(cg, mech9_path):
    """A batched call takes up to 4096 non-empty boxes (the staging ring's
    slot size); one more is CHEM_ECAPACITY.  Empty boxes do not count."""
    import torch
    m = cg.Mechanism(mech9_path, reserve=8192, auto_reserve=False)
    try:
        s = torch.from_numpy(wl.cells_uniform(mech9_path, n=4097, seed=9)).cuda()
        cols = [s[:, i:i + 1].contiguous() for i in range(4097)]
        empty = torch.zeros((m.n_species + 3, 1), dtype=torch.float64, device="cuda")
        boxes = [dict(state=c, dt=wl.DT_FLOW) for c in cols[:4096]]
        cg.chem_integrate_batched(m, boxes + [dict(state=empty, dt=wl.DT_FLOW, n_cells=0)])
        with pytest.raises(cg.ChemError) as e:
            cg.chem_integrate_batched(m, boxes + [dict(state=cols[4096], dt=wl.DT_FLOW)])
        assert e.value.code == ECAPACITY
        torch.cuda.synchronize()
    finally:
        m.close()
