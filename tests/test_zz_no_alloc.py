"""chem_integrate_noalloc: the flow step on the library's fixed scratch
array, for callers that cannot allocate.  Through the C ABI it must give
bitwise the results of chem_integrate (state, status, counts) on calls in a
row -- the second on fewer cells, the third with the tail list resumed one
cell per lane instead of by the cooperative kernel (the scratch keeps a
handed-over cell's state in its rows, the workspace in its tail record),
the fourth with the cells below the NASA-7 range switch stepped after the
resumed ones --
allocate no device memory, and refuse more than 1,048,576 cells with
CHEM_ECAPACITY."""
import numpy as np
import pytest

from paper_2506_02602_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_noalloc_matches_chem_integrate_twice(mech9_path):
    import torch
    from paper_2506_02602_amd import chemgpu as cg
    print("[noalloc] front sample and config-1 cells, tail list and pool order on", flush=True)
    front, hot = wl.front_2d(mech9_path, nx=256, ny=256, seed=2)
    big = np.ascontiguousarray(front)                                    # 65,536 cells
    small = np.ascontiguousarray(wl.cells_uniform(mech9_path, n=3001, seed=13))
    small[0, :500] += 1200.0
    o = cg.make_opts(rtol=wl.RTOL, atol=wl.ATOL, block_size=256, chunk_steps=2, tail_steps=4,
                     tail_cap=-1, pool_order=1)
    # a cap of one cell per CU sends the tail list to the per-lane resumption
    # (state in tail records for chem_integrate, in the cells' rows here)
    o_res = cg.make_opts(rtol=wl.RTOL, atol=wl.ATOL, block_size=256, chunk_steps=2, tail_steps=4,
                         tail_cap=1, pool_order=1)
    # and with the cells below the NASA-7 range switch left to the end of
    # the resumption
    o_def = cg.make_opts(rtol=wl.RTOL, atol=wl.ATOL, block_size=256, chunk_steps=2, tail_steps=4,
                         tail_cap=1, pool_order=3)
    ref_m = cg.chem_mech_load(mech9_path)
    m = cg.Mechanism(mech9_path, auto_reserve=False)      # no workspace at all
    try:
        outs = []
        for k, (s0, o) in enumerate(((big, o), (small, o), (big, o_res), (big, o_def))):
            n = s0.shape[1]
            res = []
            for which in ("plain", "noalloc"):
                st = torch.from_numpy(s0.copy()).cuda()
                status = torch.full((n,), -7, dtype=torch.int32, device="cuda")
                counts = torch.full((2 * n,), -7, dtype=torch.int32, device="cuda")
                torch.cuda.synchronize()
                free0 = torch.cuda.mem_get_info()[0]
                if which == "plain":
                    cg.chem_integrate(ref_m, st, wl.DT_FLOW, o, status=status, counts=counts)
                else:
                    cg.chem_integrate_noalloc(m, st, wl.DT_FLOW, o, status=status, counts=counts)
                torch.cuda.synchronize()
                if which == "noalloc":
                    assert torch.cuda.mem_get_info()[0] == free0
                res.append((st.cpu().numpy(), status.cpu().numpy(), counts.cpu().numpy()))
            for a, b in zip(res[0], res[1]):
                assert np.array_equal(a, b), f"call {k}"
            assert (res[1][1] == 0).all()
            outs.append(res[1])
            print(f"[noalloc] call {k}: {n} cells bitwise equal to chem_integrate "
                  f"(tail cap {o.tail_cap}), {int(res[1][2].sum())} steps", flush=True)
        # more than the scratch array holds: refused before any work
        over = torch.zeros((m.n_species + 3, cg.NOALLOC_MAX_CELLS + 1), dtype=torch.float64,
                           device="cuda")
        with pytest.raises(cg.ChemError) as e:
            cg.chem_integrate_noalloc(m, over, wl.DT_FLOW, o)
        assert e.value.code == -6
        torch.cuda.synchronize()
        assert not over.any()
    finally:
        m.close()
        ref_m.close()
