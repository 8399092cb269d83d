"""GPU tests of the surrogate kernels (MFMA forward/backward, Adam, fused
inference with trust test and FP64 fallback) against the numpy oracle."""
import os
import tempfile

import numpy as np
import pytest

from oracle import mlp_oracle as mo
from paper_2506_02602_amd import workloads as wl

from gpu_common import to_gpu

pytestmark = pytest.mark.gpu
I, O = 12, 10


@pytest.fixture(scope="module")
def cg():
    from paper_2506_02602_amd import chemgpu
    return chemgpu


@pytest.fixture(scope="module")
def gm9(cg, mech9_path):
    return cg.chem_mech_load(mech9_path)


def _states(path, seed=1):
    a = wl.cells_uniform(path, n=1500, seed=seed)
    s, hot = wl.front_2d(path, nx=128, ny=128, seed=seed, band=6)
    b = s[:, np.where(hot)[0][:400]]
    c = s[:, np.where(~hot)[0][:300]]
    return np.ascontiguousarray(np.hstack([a, b, c]))


def _norm_for(X, sd_out):
    mu = X.mean(axis=0).astype(np.float32)
    sd = X.std(axis=0).astype(np.float32)
    sd[sd == 0] = 1.0
    z = (X - mu.astype(np.float64)) / sd.astype(np.float64)
    return np.concatenate([mu, sd, np.zeros(O, np.float32), np.asarray(sd_out, np.float32),
                           z.min(axis=0).astype(np.float32), z.max(axis=0).astype(np.float32)])


def _split_norm(nm):
    return dict(mu_in=nm[:I].astype(np.float64), sd_in=nm[I:2 * I].astype(np.float64),
                mu_out=nm[2 * I:2 * I + O].astype(np.float64),
                sd_out=nm[2 * I + O:2 * I + 2 * O].astype(np.float64),
                zmin=nm[2 * I + 2 * O:3 * I + 2 * O].astype(np.float64),
                zmax=nm[3 * I + 2 * O:].astype(np.float64))


def _rel_fro(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _output_units(out, ref, cache, theta):
    """Element-wise distance of network outputs from the oracle's, in units of
    the output's BF16 rounding scale S = 2^-7 sum_k |W4_ik| |h3_k|: what the
    output moves by if every last-layer activation h3_k (a BF16 value, so
    one ulp is at most 2^-7 of it) moved by one ulp.  The kernel and the
    oracle round the same quantities to BF16; they differ where an FP32
    activation lies within the kernel's SiLU error of a BF16 rounding
    boundary (one ulp there) and by FP32 summation order, both far below S.
    A wrong weight, index or term moves an output by O(S * 2^7)."""
    p = mo.unpack(theta, I, O)
    S = 2.0 ** -7 * (np.abs(cache["H"][3]) @ np.abs(mo.bf16(p["W4"])).T)
    return np.abs(out - ref) / S


def test_fused_inference_matches_oracle(cg, gm9, omech9, mech9_path):
    """MLP outputs of the fused kernel vs the BF16-emulating oracle; trust
    decisions identical given the same network outputs; trusted cells get
    state + increment, untrusted ones are left alone (no fallback here)."""
    import torch
    state = _states(mech9_path)
    n = state.shape[1]
    names, W = wl.read_species(mech9_path)
    X = mo.features(state, 1e-7, W)
    s = cg.Surrogate(gm9, seed=3)
    sd_out = np.r_[5.0, np.full(9, 2e-4)]
    s.set_params(norm=_norm_for(X, sd_out))
    theta, nm = s.get_params()
    norm = _split_norm(nm)
    g = to_gpu(state)
    tc = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    os_ = torch.zeros((n, O), dtype=torch.float32, device="cuda")
    trust = (0.05, 1e-3, 1e-4, 400.0)
    cg.surrogate_infer(s, gm9, g, 1e-7, trust, fallback=False, trust_code=tc, out_std=os_)
    torch.cuda.synchronize()
    out_gpu = os_.cpu().numpy().astype(np.float64)
    z = (X - norm["mu_in"]) / norm["sd_in"]
    out_ref, cache = mo.forward(theta.astype(np.float64), z, I, O)
    u = _output_units(out_gpu, out_ref, cache, theta.astype(np.float64))
    print(f"[surrogate] fused forward: {u.size} outputs, max {u.max():.3f} rounding units, "
          f"{(u > 0.1).sum()} above 0.1, rel Frobenius {_rel_fro(out_gpu, out_ref):.2e}",
          flush=True)
    assert u.max() <= 1.0
    codes_ref = mo.trust_codes(omech9, state, 1e-7, z, out_gpu.astype(np.float32), norm, trust)
    codes = tc.cpu().numpy()
    assert np.array_equal(codes, codes_ref)
    assert 0 < (codes == 0).sum() < n                   # both outcomes exercised
    new = g.cpu().numpy()
    inc = out_gpu * norm["sd_out"] + norm["mu_out"]
    ok = codes == 0
    want = mo.trusted_update(state[:, ok], inc[ok])
    assert np.allclose(new[0, ok], want[0], rtol=1e-14)
    assert np.allclose(new[1:10, ok], want[1:], rtol=1e-13, atol=1e-18)
    assert (new[1:10, ok] >= 0.0).all()                 # clipped at zero
    assert np.array_equal(new[:, ~ok], state[:, ~ok])


def test_generic_forward_matches_oracle(cg, gm9, mech9_path):
    import torch
    state = _states(mech9_path, seed=2)
    names, W = wl.read_species(mech9_path)
    X = mo.features(state, 1e-7, W)
    s = cg.Surrogate(gm9, seed=4)
    s.set_params(norm=_norm_for(X, np.ones(O)))
    theta, nm = s.get_params()
    Xf = X.astype(np.float32)
    out = cg.surrogate_forward(s, to_gpu(Xf)).cpu().numpy().astype(np.float64)
    z32 = (Xf - nm[:I]) / nm[I:2 * I]                  # the kernel standardises in FP32
    ref, cache = mo.forward(theta.astype(np.float64), z32.astype(np.float64), I, O)
    u = _output_units(out, ref, cache, theta.astype(np.float64))
    print(f"[surrogate] training-path forward: max {u.max():.3f} rounding units, "
          f"rel Frobenius {_rel_fro(out, ref):.2e}", flush=True)
    assert u.max() <= 1.0


def test_gradients_match_oracle(cg, gm9):
    rng = np.random.Generator(np.random.PCG64(7))
    B = 512
    Xn = rng.standard_normal((B, I)).astype(np.float32)
    Yn = rng.standard_normal((B, O)).astype(np.float32)
    s = cg.Surrogate(gm9, seed=5)
    theta, _ = s.get_params()
    grad, loss = cg.surrogate_grad(s, to_gpu(Xn), to_gpu(Yn))
    g_gpu = grad.cpu().numpy().astype(np.float64)
    g_ref, loss_ref = mo.backward(theta.astype(np.float64), Xn.astype(np.float64),
                                  Yn.astype(np.float64), I, O)
    assert loss == pytest.approx(loss_ref, rel=1e-3)
    pg, pr = mo.unpack(g_gpu, I, O), mo.unpack(g_ref, I, O)
    for name in pg:
        rel = _rel_fro(pg[name], pr[name])
        cos = float((pg[name] * pr[name]).sum() / np.linalg.norm(pg[name]) / np.linalg.norm(pr[name]))
        print(f"[surrogate] grad {name}: rel {rel:.2e} cos {cos:.6f}", flush=True)
        assert rel < 1e-2 and cos > 0.9999


def test_one_adam_step_matches_oracle(cg, gm9):
    """One training step equals the oracle's Adam step (FP64) applied to the
    kernel's own gradient of the same batch, for every parameter, to the
    rounding of the FP32 update.  The batch repeats one sample, so the
    epoch's permutation of its rows cannot change the gradient's summation
    (the training step's gradient is then bitwise surrogate_grad's); the
    gradient itself is held to the oracle's in test_gradients_match_oracle."""
    import torch
    rng = np.random.Generator(np.random.PCG64(8))
    B = 256
    X = np.repeat(rng.standard_normal((1, I)), B, axis=0).astype(np.float32)
    Y = np.repeat(rng.standard_normal((1, O)), B, axis=0).astype(np.float32)
    s = cg.Surrogate(gm9, seed=6)
    theta0, _ = s.get_params()
    ident = np.concatenate([np.zeros(I), np.ones(I), np.zeros(O), np.ones(O),
                            np.full(I, -10.0), np.full(I, 10.0)]).astype(np.float32)
    s.set_params(norm=ident)
    g_gpu, _ = cg.surrogate_grad(s, to_gpu(X), to_gpu(Y))
    g_gpu = g_gpu.cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    cg.surrogate_train(s, to_gpu(X), to_gpu(Y), epochs=1, batch=B, lr=1e-3, seed=1)
    theta1, _ = s.get_params()
    # the kernel's decay rates are FP32 numbers (0.9f, 0.999f), used both in
    # the moment updates and in the bias corrections
    th_ref, _, _ = mo.adam_step(theta0.astype(np.float64), g_gpu, np.zeros_like(g_gpu),
                                np.zeros_like(g_gpu), 1, lr=1e-3,
                                beta1=float(np.float32(0.9)), beta2=float(np.float32(0.999)))
    # FP32 master weights: the update is rounded to FP32 once, and the FP32
    # step arithmetic (a few roundings of a value <= lr) adds below 1e-9
    ulp = np.spacing(np.abs(th_ref).astype(np.float32)).astype(np.float64)
    err = np.abs(theta1.astype(np.float64) - th_ref)
    print(f"[surrogate] adam step: max {np.max(err / (ulp + 1e-9)):.3f} (FP32 ulp + 1e-9) "
          f"over {err.size} parameters", flush=True)
    assert (err <= ulp + 1e-9).all()
    d = theta1.astype(np.float64) - theta0
    assert np.abs(d).max() <= 1.001e-3 and np.count_nonzero(d) > err.size // 2


def test_training_reduces_loss(cg, gm9):
    rng = np.random.Generator(np.random.PCG64(9))
    n = 65536
    X = rng.standard_normal((n, I)).astype(np.float32)
    Wt = rng.standard_normal((I, O)) / np.sqrt(I)
    Y = np.sin(X.astype(np.float64) @ Wt).astype(np.float32)
    s = cg.Surrogate(gm9, seed=7)
    loss = cg.surrogate_train(s, to_gpu(X), to_gpu(Y), epochs=8, batch=1024, lr=2e-3, seed=3)
    print(f"[surrogate] losses {loss}", flush=True)
    assert loss[-1] < 0.2 * loss[0]
    assert np.all(np.isfinite(loss))


def test_fallback_cells_equal_fp64_integrator(cg, gm9, mech9_path):
    """Cells that fail the trust test are integrated by the FP64 path from
    their own state: bitwise the same as chem_integrate on those cells."""
    import torch
    state = _states(mech9_path, seed=3)
    n = state.shape[1]
    names, W = wl.read_species(mech9_path)
    X = mo.features(state, 1e-7, W)
    s = cg.Surrogate(gm9, seed=8)
    s.set_params(norm=_norm_for(X, np.r_[5.0, np.full(9, 2e-4)]))
    ref = to_gpu(state)
    rst = torch.zeros(n, dtype=torch.int32, device="cuda")
    rcn = torch.zeros(2 * n, dtype=torch.int32, device="cuda")
    cg.chem_integrate(gm9, ref, 1e-7, status=rst, counts=rcn)
    for trust in [(0.05, 1e-3, 1e-4, -1.0), (0.05, 1e-3, 1e-4, 400.0)]:
        g = to_gpu(state)
        tc = torch.zeros(n, dtype=torch.int32, device="cuda")
        st = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        cn = torch.full((2 * n,), -7, dtype=torch.int32, device="cuda")
        nfb = cg.surrogate_infer(s, gm9, g, 1e-7, trust, fallback=True, trust_code=tc, status=st,
                                 counts=cn, want_count=True)
        torch.cuda.synchronize()
        fb = (tc != 0)
        assert nfb == int(fb.sum())
        if trust[3] < 0:
            assert nfb == n
        assert torch.equal(g[:, fb], ref[:, fb])
        assert torch.equal(st[fb], rst[fb])
        assert torch.equal(cn.view(2, n)[:, fb], rcn.view(2, n)[:, fb])
        assert (st[~fb] == -7).all()


def test_make_pairs_match_oracle_features(cg, gm9, mech9_path):
    import torch
    state = _states(mech9_path, seed=4)
    n = state.shape[1]
    before = to_gpu(state)
    after = before.clone()
    cg.chem_integrate(gm9, after, 1e-7)
    dts = torch.from_numpy(np.geomspace(2.5e-8, 2e-7, n)).cuda()
    Xg, Yg = cg.surrogate_make_pairs(gm9, before, after, dt_cells=dts)
    torch.cuda.synchronize()
    names, W = wl.read_species(mech9_path)
    Xr = mo.features(state, 1e-7, W)
    Xr[:, 2] = np.log(np.geomspace(2.5e-8, 2e-7, n))
    assert np.allclose(Xg.cpu().numpy(), Xr.astype(np.float32), rtol=2e-7, atol=0)
    inc = (after.cpu().numpy() - state)[:10].T
    assert np.allclose(Yg.cpu().numpy(), inc.astype(np.float32), rtol=2e-7, atol=1e-30)


def test_save_load_roundtrip(cg, gm9):
    s = cg.Surrogate(gm9, seed=10)
    th, nm = s.get_params()
    nm[:I] = np.arange(I)
    s.set_params(norm=nm)
    fd, p = tempfile.mkstemp(suffix=".surr")
    os.close(fd)
    try:
        cg.surrogate_save(s, p)
        t = cg.surrogate_load(gm9, p)
        th2, nm2 = t.get_params()
        assert np.array_equal(th, th2) and np.array_equal(nm, nm2)
    finally:
        os.unlink(p)
