"""Pins for the surrogate's CPU oracle (oracle/mlp_oracle.py).  The paper gives
no surrogate design, so these pin the oracle to library routines, finite
differences and closed forms rather than to printed values."""
import numpy as np
import pytest

import oracle
from oracle import mlp_oracle as mo
from paper_2506_02602_amd import workloads as wl

I, O, H = 12, 10, 128


def _net(seed=0, hidden=H):
    rng = np.random.Generator(np.random.PCG64(seed))
    th = mo.he_uniform_init(I, O, hidden, rng)
    th = th + 0.01 * rng.standard_normal(th.shape)     # non-zero biases too
    return th, rng


def test_bf16_matches_torch_round_to_nearest_even():
    import torch
    rng = np.random.Generator(np.random.PCG64(1))
    x = (rng.standard_normal(100000) * 10.0 ** rng.uniform(-6, 6, 100000)).astype(np.float32)
    x[:4] = [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -1.5 - 2.0 ** -8, 0.0]   # exact ties
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mo.bf16(x.astype(np.float64)), ref)


def test_silu_derivative_by_finite_differences():
    z = np.linspace(-8, 8, 101)
    h = 1e-6
    fd = (mo.silu(z + h) - mo.silu(z - h)) / (2 * h)
    assert np.allclose(mo.silu_grad(z), fd, rtol=1e-8, atol=1e-10)


def test_forward_matches_torch_layers_without_rounding():
    import torch
    th, rng = _net(2)
    X = rng.standard_normal((37, I))
    out, _ = mo.forward(th, X, I, O, emulate_bf16=False)
    p = mo.unpack(th, I, O)
    net = torch.nn.Sequential(torch.nn.Linear(I, H), torch.nn.SiLU(), torch.nn.Linear(H, H),
                              torch.nn.SiLU(), torch.nn.Linear(H, H), torch.nn.SiLU(),
                              torch.nn.Linear(H, O)).double()
    with torch.no_grad():
        for li, l in zip((0, 2, 4, 6), (1, 2, 3, 4)):
            net[li].weight.copy_(torch.from_numpy(p[f"W{l}"]))
            net[li].bias.copy_(torch.from_numpy(p[f"b{l}"]))
        ref = net(torch.from_numpy(X)).numpy()
    assert np.allclose(out, ref, rtol=1e-12, atol=1e-12)


def test_backward_matches_central_differences():
    th, rng = _net(3, hidden=16)
    X = rng.standard_normal((9, I))
    Y = rng.standard_normal((9, O))
    g, _ = mo.backward(th, X, Y, I, O, hidden=16, emulate_bf16=False)
    idx = rng.choice(len(th), 60, replace=False)
    eps = 1e-6
    for k in idx:
        tp, tm = th.copy(), th.copy()
        tp[k] += eps
        tm[k] -= eps
        lp = mo.mse(mo.forward(tp, X, I, O, 16, False)[0], Y)
        lm = mo.mse(mo.forward(tm, X, I, O, 16, False)[0], Y)
        fd = (lp - lm) / (2 * eps)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_backward_with_rounding_stays_close():
    th, rng = _net(4)
    X = rng.standard_normal((64, I))
    Y = rng.standard_normal((64, O))
    g0, _ = mo.backward(th, X, Y, I, O, emulate_bf16=False)
    g1, _ = mo.backward(th, X, Y, I, O, emulate_bf16=True)
    cos = g0 @ g1 / np.linalg.norm(g0) / np.linalg.norm(g1)
    assert cos > 0.999


def test_adam_first_step_closed_form():
    """With m = v = 0 the first update is -lr g / (|g| + eps)."""
    rng = np.random.Generator(np.random.PCG64(5))
    th = rng.standard_normal(50)
    g = rng.standard_normal(50) * 10.0 ** rng.uniform(-5, 2, 50)
    new, m, v = mo.adam_step(th, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    assert np.allclose(new, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_minimises_a_quadratic():
    th = np.array([3.0, -2.0])
    m = v = np.zeros(2)
    for t in range(1, 3001):
        g = 2 * (th - np.array([0.5, 0.25]))
        th, m, v = mo.adam_step(th, g, m, v, t, lr=mo.cosine_lr(0.05, t, 3000))
    assert np.allclose(th, [0.5, 0.25], atol=1e-4)


def test_cosine_schedule_endpoints():
    assert mo.cosine_lr(1e-3, 0, 100) == pytest.approx(1e-3)
    assert mo.cosine_lr(1e-3, 50, 100) == pytest.approx(5e-4)
    assert mo.cosine_lr(1e-3, 100, 100) == pytest.approx(0.0, abs=1e-18)


def test_features_pressure_is_the_ideal_gas_input(mech9_path):
    names, W = wl.read_species(mech9_path)
    s = wl.cells_uniform(mech9_path, n=16, seed=2)
    f = mo.features(s, 1e-7, W)
    assert np.allclose(np.exp(f[:, 1]), wl.P_ATM, rtol=1e-12)   # generator set p = 1 atm
    assert np.allclose(f[:, 2], np.log(1e-7))
    assert np.array_equal(f[:, 0], s[0]) and np.array_equal(f[:, 3:], s[1:10].T)


def test_trust_bits_on_hand_built_cells(mech9_path, omech9):
    """An exact FP64 integrator increment passes; each violation raises its bit."""
    s = wl.cells_uniform(mech9_path, n=5, seed=3)
    s[0] = 1900.0
    N = 9
    after = s.copy()
    omech9.integrate(after, 1e-7)
    inc = (after[:N + 1] - s[:N + 1]).T.copy()
    inc[1, 1 + 3] += 1e-3                        # create H atoms from nothing
    inc[2, 1 + 0] = -s[1, 2] - 1e-3              # drive Y_H2 negative (elements broken too)
    inc[3, 0] += 50.0                            # temperature inconsistent with energy
    norm = dict(mu_out=np.zeros(N + 1), sd_out=np.ones(N + 1), zmin=np.full(I, -1.0),
                zmax=np.full(I, 1.0))
    z = np.zeros((5, I))
    z[4, 2] = 1.5                                # outside the hull by 0.5
    codes = mo.trust_codes(omech9, s, 1e-7, z, inc, norm, (0.1, 1e-6, 1e-8, 0.5))
    assert codes[0] == 0
    assert codes[1] & mo.TRUST_ELEM and not codes[1] & mo.TRUST_POS
    assert codes[2] & mo.TRUST_POS
    assert codes[3] == mo.TRUST_ENERGY
    assert codes[4] == mo.TRUST_HULL
    codes = mo.trust_codes(omech9, s, 1e-7, z, inc, norm, (0.6, 1e-6, 1e-8, 0.5))
    assert codes[4] == 0
