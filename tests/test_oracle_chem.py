"""Pins for the oracle's chemistry: NASA-7 thermo (Eq. 10), mass-action rates
(Eq. 15-16), the T closure of the chemistry ODE (Eq. 20) and whole-cell
integration.  Expected values come from identities, closed forms, an
independent Gibbs-equilibrium solver, or brute force -- not from the oracle."""
import math
import os
import tempfile

import numpy as np
import pytest

import oracle
from paper_2506_02602_amd import mechgen, workloads as wl

from equilibrium import uv_equilibrium

R_J = 8.31446261815324
R_CGS = 8.31446261815324e7


# ----------------------------------------------------------- helpers
def _cell(path, T, p_atm, Y=None, seed=0):
    names, W = wl.read_species(path)
    rng = np.random.Generator(np.random.PCG64(seed))
    if Y is None:
        Y = wl.base_mixture(names, W, 1, rng)[:, 0]
    rho = wl.density(np.array([T]), np.array([p_atm * wl.P_ATM]), Y[:, None], W)[0]
    return rho, np.concatenate([[T], Y])


def _energy(m, T, Y):
    """Mixture internal energy per mass, erg/g: sum_k Y_k (H_k - R T)/W_k."""
    _, h, _ = m.thermo(T)
    return float(np.sum(Y * R_CGS * T * (h - 1.0) / m.W))


def _hot_states(path, n, seed):
    s, hot = wl.front_2d(path, nx=256, ny=256, seed=seed, band=6)
    idx = np.where(hot)[0][:n]
    return np.ascontiguousarray(s[:, idx])


def _write_mech(text):
    fd, path = tempfile.mkstemp(suffix=".mech")
    with os.fdopen(fd, "w") as f:
        f.write(text)
    return path


def _isomer_text(A, b, Ea, tb=False, eff=None):
    base = open(wl.mech_file("isomer")).read()
    head = base.split("reactions")[0]
    lines = [head + "reactions 1", f"reaction {A!r} {b!r} {Ea!r} {1 if tb else 0}",
             "reactants 1 A 1", "products 1 B 1"]
    if tb:
        lines.append("efficiencies " + " ".join(repr(x) for x in eff))
    lines.append("end")
    return "\n".join(lines) + "\n"


# ----------------------------------------------------------- thermo
@pytest.mark.parametrize("mechname", ["mech9", "mech32"])
def test_nasa7_identities(mechname):
    """d(H/R)/dT = cp/R and d(S/R)/dT = cp/(R T) in both ranges (central differences)."""
    m = oracle.Mech(wl.mech_file(mechname))
    for T in (450.0, 800.0, 1500.0, 2800.0, 4200.0):
        dT = 1e-2
        cp, _, _ = m.thermo(T)
        _, hp, sp = m.thermo(T + dT)
        _, hm, sm = m.thermo(T - dT)
        dH = ((T + dT) * hp - (T - dT) * hm) / (2 * dT)
        dS = (sp - sm) / (2 * dT)
        assert np.allclose(dH, cp, rtol=1e-7, atol=1e-7)
        assert np.allclose(dS * T, cp, rtol=1e-7, atol=1e-7)


def test_nasa7_reference_values_and_continuity():
    """H(298.15) and S(298.15) equal the drawn formation values; H, S continuous at Tmid."""
    gen = mechgen.build_mech9()
    m = oracle.Mech(wl.mech_file("mech9"))
    _, h, s = m.thermo(298.15)
    for k, sp in enumerate(gen["species"]):
        assert h[k] * R_J * 298.15 == pytest.approx(sp.hf, abs=1e-6 * (abs(sp.hf) + 1e3))
        assert s[k] * R_J == pytest.approx(sp.s0, rel=1e-12)
    _, hl, sl = m.thermo(1000.0 - 1e-9)
    _, hh, sh = m.thermo(1000.0)
    assert np.allclose(hl, hh, rtol=1e-9, atol=1e-9)
    assert np.allclose(sl, sh, rtol=1e-9, atol=1e-9)


# ----------------------------------------------------------- rates
def test_arrhenius_special_values():
    """k_f = A T^b exp(-Ea/RT): Ea = R T0 and b = 1 give A T0 / e at T0 (R in J/mol/K)."""
    T0 = 1200.0
    path = _write_mech(_isomer_text(3.0, 1.0, R_J * T0))
    try:
        m = oracle.Mech(path)
        rho, u = _cell(wl.mech_file("isomer"), T0, 1.0, Y=np.array([0.7, 0.3]))
        kf, kr, q, w = m.rates(rho, u)
        assert kf[0] == pytest.approx(3.0 * T0 / math.e, rel=1e-14)
        assert kr[0] == pytest.approx(kf[0], rel=1e-14)  # identical thermo: Kc = 1
        c = rho * u[1:] / m.W
        assert q[0] == pytest.approx(kf[0] * (c[0] - c[1]), rel=1e-13)
        assert w[0] == -q[0] and w[1] == q[0]
    finally:
        os.unlink(path)


def test_third_body_concentration():
    """Unit efficiencies give [M] = total concentration = p/(RT); [M] is linear in alpha."""
    T0, p = 1500.0, 2.0
    rho, u = _cell(wl.mech_file("isomer"), T0, p, Y=np.array([0.6, 0.4]))
    plain = oracle.Mech(wl.mech_file("isomer"))
    _, _, q0, _ = plain.rates(rho, u)
    paths = [_write_mech(_isomer_text(2.0e7, 0.0, 0.0, True, [1.0, 1.0])),
             _write_mech(_isomer_text(2.0e7, 0.0, 0.0, True, [2.0, 6.0]))]
    try:
        _, _, q1, _ = oracle.Mech(paths[0]).rates(rho, u)
        _, _, q2, _ = oracle.Mech(paths[1]).rates(rho, u)
        ctot = p * wl.P_ATM / (R_CGS * T0)
        assert q1[0] == pytest.approx(ctot * q0[0], rel=1e-12)
        c = rho * u[1:] / plain.W
        assert q2[0] == pytest.approx((2.0 * c[0] + 6.0 * c[1]) * q0[0], rel=1e-12)
    finally:
        for pth in paths:
            os.unlink(pth)


@pytest.mark.parametrize("mechname", ["mech9", "mech32"])
def test_mass_and_element_conservation_of_rates(mechname):
    """sum_k W_k wdot_k = 0 and sum_k a_ek wdot_k = 0 (every reaction is balanced)."""
    path = wl.mech_file(mechname)
    m = oracle.Mech(path)
    s = wl.stress_3d(path, shape=(4, 4, 2), seed=11)
    for i in range(s.shape[1]):
        N = m.ns
        _, _, _, w = m.rates(s[N + 1, i], s[:N + 1, i])
        scale = np.abs(m.W * w).sum() + 1e-300
        assert abs(np.sum(m.W * w)) <= 1e-13 * scale
        for e in range(m.ne):
            sc = np.abs(m.comp[:, e] * w).sum() + 1e-300
            assert abs(np.sum(m.comp[:, e] * w)) <= 1e-13 * sc


@pytest.mark.parametrize("mechname", ["mech9", "mech32"])
def test_detailed_balance_at_gibbs_equilibrium(mechname):
    """At the independent U,V equilibrium every reaction's forward and reverse
    rates agree: pins Kc (sign of g/RT, stoichiometry, the (P/RT)^dnu factor)."""
    path = wl.mech_file(mechname)
    m = oracle.Mech(path)
    s = wl.stress_3d(path, shape=(2, 2, 1), seed=5)
    for i in range(2):
        N = m.ns
        rho, T0, Y0 = s[N + 1, i], s[0, i], s[1:N + 1, i]
        Teq, Yeq, ceq = uv_equilibrium(m, rho, T0, Y0)
        kf, kr, _, _ = m.rates(rho, np.concatenate([[Teq], Yeq]))
        fwd = kf * np.prod(ceq ** np.clip(-m.nu, 0, None), axis=1)
        rev = kr * np.prod(ceq ** np.clip(m.nu, 0, None), axis=1)
        assert np.max(np.abs(np.log(fwd / rev))) < 1e-10


@pytest.mark.parametrize("mechname", ["mech9", "mech32"])
def test_temperature_closure_conserves_energy(mechname):
    """de/dt = sum_k e_k dY_k/dt + (de/dT) dT/dt = 0 with de/dT by finite differences."""
    path = wl.mech_file(mechname)
    m = oracle.Mech(path)
    s = wl.stress_3d(path, shape=(3, 3, 1), seed=6)
    N = m.ns
    for i in range(s.shape[1]):
        rho, u = s[N + 1, i], s[:N + 1, i]
        f = m.rhs(rho, u)
        T, Y = u[0], u[1:]
        dT = 1e-3
        dedT = (_energy(m, T + dT, Y) - _energy(m, T - dT, Y)) / (2 * dT)
        _, h, _ = m.thermo(T)
        ek = R_CGS * T * (h - 1.0) / m.W
        total = np.sum(ek * f[1:]) + dedT * f[0]
        scale = np.sum(np.abs(ek * f[1:])) + abs(dedT * f[0])
        assert abs(total) <= 1e-7 * scale


# ----------------------------------------------------------- integration
def test_isomer_closed_form_adaptive(isomer_path):
    """A <-> B with kf = kr = k: c_A - c_B decays as exp(-2 k t); T stays put."""
    m = oracle.Mech(isomer_path)
    k, dt = 2.0e7, 1.0e-7
    rho, u = _cell(isomer_path, 1400.0, 1.0, Y=np.array([0.9, 0.1]))
    r = m.integrate_cell(rho, u, dt, rtol=1e-12, atol=1e-16)
    d0 = u[1] - u[2]
    d1 = r["u"][1] - r["u"][2]
    assert d1 == pytest.approx(d0 * math.exp(-2 * k * dt), rel=1e-10)
    assert r["u"][1] + r["u"][2] == pytest.approx(1.0, abs=1e-15 * (10 + r["nacc"] + r["nrej"]))
    assert abs(r["u"][0] - 1400.0) < 1e-9


def test_isomer_fixed_steps_match_stability_function(isomer_path):
    """Fixed steps: (c_A - c_B) is multiplied by R(-2 k h) per step exactly."""
    from test_oracle_scheme import _butcher, _load_tableau, _R, _stab_coeffs
    import mpmath as mp
    a, b, _ = _load_tableau()
    gam = _stab_coeffs(_butcher(a, b), b)
    m = oracle.Mech(isomer_path)
    k, dt, n = 2.0e7, 1.0e-7, 16
    rho, u = _cell(isomer_path, 1400.0, 1.0, Y=np.array([0.8, 0.2]))
    r = m.integrate_cell(rho, u, dt, fixed_steps=n)
    mp.mp.dps = 40
    fac = float(_R(gam, mp.mpf(-2 * k) * mp.mpf(dt) / n) ** n)
    assert (r["u"][1] - r["u"][2]) == pytest.approx((u[1] - u[2]) * fac, rel=1e-12)


def test_linear_invariants_preserved(mech9_path, omech9):
    """sum Y and element mass fractions drift only by rounding (no clipping)."""
    s = _hot_states(mech9_path, 16, seed=21)
    N = omech9.ns
    Y0 = s[1:N + 1].copy()
    st, cnt = omech9.integrate(s, 1e-7)
    assert (st == 0).all()
    steps = cnt.sum(axis=0)
    Y1 = s[1:N + 1]
    assert np.all(np.abs(Y1.sum(axis=0) - Y0.sum(axis=0)) <= 1e-15 * (10 + steps))
    aw = omech9.comp * 1.0 / omech9.W[:, None]  # element moles per gram, per species
    el0 = aw.T @ Y0
    el1 = aw.T @ Y1
    assert np.all(np.abs(el1 - el0) <= 1e-15 * (10 + steps) * np.abs(el0).max())


def test_energy_conservation_scales_with_tolerance(mech9_path, omech9):
    """Internal energy is conserved to truncation error, shrinking with tol."""
    s0 = _hot_states(mech9_path, 6, seed=22)
    N = omech9.ns
    drifts = []
    for tol in (1e-6, 1e-8, 1e-10):
        s = s0.copy()
        st, _ = omech9.integrate(s, 1e-7, rtol=tol, atol=1e-12)
        assert (st == 0).all()
        d = []
        for i in range(s.shape[1]):
            e0 = _energy(omech9, s0[0, i], s0[1:N + 1, i])
            e1 = _energy(omech9, s[0, i], s[1:N + 1, i])
            cv = (_energy(omech9, s0[0, i] + 1e-2, s0[1:N + 1, i]) - e0) / 1e-2
            d.append(abs(e1 - e0) / cv)         # as an equivalent temperature error, K
        drifts.append(max(d))
    assert drifts[0] < 1e-6 * 3000 * 10
    assert drifts[2] < drifts[0]


@pytest.mark.parametrize("scheme", ["lsrk", "rkf45"])
def test_fourth_order_convergence_fixed_steps(mech9_path, omech9, scheme):
    """Fixed-step error in Y vs a fine reference falls ~16x per halving (order 4)
    on an igniting 1 atm cell over 0.1 ms (smooth, not stability-limited);
    both the low-storage scheme and the full-storage comparison scheme (whose
    smaller stability region needs at least 1024 steps on the 1600 K cell)."""
    ns = (512, 1024, 2048) if scheme == "lsrk" else (1024, 2048)
    for T0 in (1500.0, 1600.0):
        rho, u = _cell(mech9_path, T0, 1.0)
        ref = omech9.integrate_cell(rho, u, 1e-4, fixed_steps=16384, scheme=scheme)["u"]
        errs = [np.abs(omech9.integrate_cell(rho, u, 1e-4, fixed_steps=n, scheme=scheme)["u"]
                       - ref)[1:].max()
                for n in ns]
        for e0, e1 in zip(errs, errs[1:]):
            assert 14 < e0 / e1 < 18


def _rk4_bruteforce(m, rho, u0, dt, n):
    u = u0.copy()
    h = dt / n
    for _ in range(n):
        k1 = m.rhs(rho, u)
        k2 = m.rhs(rho, u + 0.5 * h * k1)
        k3 = m.rhs(rho, u + 0.5 * h * k2)
        k4 = m.rhs(rho, u + h * k3)
        u = u + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return u


@pytest.mark.slow
def test_bruteforce_classical_rk4(mech9_path, omech9):
    """Adaptive LSRK at tol 1e-8 is within ~10 tol of tiny-step classical RK4
    (an independent integrator), and within 1e-10 at tol 1e-12."""
    s0 = _hot_states(mech9_path, 3, seed=24)
    N = omech9.ns
    for i in range(s0.shape[1]):
        rho, u0 = s0[N + 1, i], s0[:N + 1, i].copy()
        a = _rk4_bruteforce(omech9, rho, u0, 1e-7, 4000)
        b = _rk4_bruteforce(omech9, rho, u0, 1e-7, 8000)
        ref = b + (b - a) / 15.0                 # Richardson
        assert np.abs(b - a)[1:].max() < 1e-12
        r8 = omech9.integrate_cell(rho, u0, 1e-7, rtol=1e-8, atol=1e-10)
        r12 = omech9.integrate_cell(rho, u0, 1e-7, rtol=1e-12, atol=1e-14)
        assert abs(r8["u"][0] - ref[0]) < 10 * 1e-8 * ref[0]
        assert np.abs(r8["u"][1:] - ref[1:]).max() < 10 * (1e-8 * np.abs(ref[1:]).max() + 1e-10)
        assert abs(r12["u"][0] - ref[0]) < 1e-10 * ref[0]
        assert np.abs(r12["u"][1:] - ref[1:]).max() < 1e-10


@pytest.mark.slow
def test_long_integration_reaches_gibbs_equilibrium(mech9_path, omech9):
    """From an igniting 1600 K cell, 2 ms of integration lands on the U,V equilibrium."""
    rho, u = _cell(mech9_path, 1600.0, 1.0)
    Teq, Yeq, _ = uv_equilibrium(omech9, rho, u[0], u[1:])
    r = omech9.integrate_cell(rho, u, 2e-3, max_steps=10 ** 6)
    assert r["status"] == oracle.STATUS_OK
    assert abs(r["u"][0] - Teq) < 1e-4
    assert np.abs(r["u"][1:] - Yeq).max() < 1e-7


def test_status_codes(mech9_path, omech9):
    s = _hot_states(mech9_path, 4, seed=25)
    N = omech9.ns
    s[3, 1] = np.nan                       # a non-finite input
    before = s[:, 1].copy()
    st, cnt = omech9.integrate(s, 1e-7, max_steps=2)
    assert st[1] == oracle.STATUS_NONFINITE
    assert np.array_equal(np.isnan(s[:, 1]), np.isnan(before))
    assert np.allclose(np.nan_to_num(s[:, 1]), np.nan_to_num(before))
    others = [0, 2, 3]
    assert all(st[i] == oracle.STATUS_MAXSTEPS for i in others)
    assert all(cnt[0, i] + cnt[1, i] == 2 for i in others)


def test_h_row_is_next_step_hint(mech9_path, omech9):
    """The h row on return is the controller's proposal; reusing it changes nothing in t."""
    s = _hot_states(mech9_path, 4, seed=26)
    st, cnt = omech9.integrate(s, 1e-7)
    N = omech9.ns
    assert (s[N + 2] > 0).all() and (s[N + 2] <= 5 * 1e-7).all()


def test_divergence_workload_profile(mech9_path):
    """Eq. 27-28 at the midpoint reduce to T_b + A cos(2 pi f y_m / L); the
    far ends approach T_b -+ T_r (tanh saturates, the Gaussian vanishes); the
    field is uniform in x and z with mole fractions H2:O2:N2 = 1:2:7."""
    import math
    from paper_2506_02602_amd import workloads as wl
    for alpha in (1.0, 0.1):
        A, f = 50.0 / alpha, 4.0 / alpha
        assert wl.diverge_temperature(0.5, 1.0, alpha) == pytest.approx(
            1300.0 + A * math.cos(2 * math.pi * f * 0.5), rel=1e-14)
        lo, hi = wl.diverge_temperature(np.array([0.0, 1.0]), 1.0, alpha)
        assert abs(lo - (1300.0 - 300.0 * math.tanh(3.0 / alpha))) < A * math.exp(-2.0) + 1e-9
        assert abs(hi - (1300.0 + 300.0 * math.tanh(3.0 / alpha))) < A * math.exp(-2.0) + 1e-9
    s = wl.diverge_box(mech9_path, 0.1)
    names, W = wl.read_species(mech9_path)
    T = s[0].reshape(16, 256, 16)
    assert (T == T[:1, :, :1]).all() and s.shape[1] == 65536
    X = s[1:10, 0] / W
    X /= X.sum()
    k = {n: i for i, n in enumerate(names)}
    assert X[k["O2"]] / X[k["H2"]] == pytest.approx(2.0, rel=1e-12)
    assert X[k["N2"]] / X[k["H2"]] == pytest.approx(7.0, rel=1e-12)


# ------------------------------------------------ split-scheme coupling

def _mixtures(path, n, seed):
    """Cells with T in [300, 3500] K and random compositions incl. radicals."""
    names, W = wl.read_species(path)
    rng = np.random.Generator(np.random.PCG64(seed))
    Y = rng.dirichlet(np.ones(len(names)), size=n).T
    T = rng.uniform(300.0, 3500.0, n)
    return T, Y


def test_cv_is_the_temperature_derivative_of_e(mech9_path, omech9):
    T, Y = _mixtures(mech9_path, 20, 51)
    for t, y in zip(T, Y.T):
        if abs(t - 1000.0) < 5.0:
            continue                          # the fits' range change at Tmid
        e1, _ = omech9.energy(t - 1e-3, y)
        e2, _ = omech9.energy(t + 1e-3, y)
        _, cv = omech9.energy(t, y)
        assert (e2 - e1) / 2e-3 == pytest.approx(cv, rel=1e-7)


def test_calculate_T_round_trip(mech9_path, omech9):
    """Newton recovers the temperature that produced e, from poor guesses."""
    T, Y = _mixtures(mech9_path, 200, 52)
    for t, y in zip(T, Y.T):
        e, _ = omech9.energy(t, y)
        for t0 in (0.0, 300.0, 3500.0):
            tt, it = omech9.calculate_T(y, e, t0)
            assert it > 0 and tt == pytest.approx(t, rel=1e-11)


def _conserved(om, path, state, rng):
    """Conserved rows from a primitive SoA block, with random velocities."""
    N = om.ns
    n = state.shape[1]
    T, Y, rho, h = state[0], state[1:N + 1], state[N + 1], state[N + 2]
    vel = rng.uniform(-5e4, 5e4, (3, n))                # cm/s
    e = np.array([om.energy(T[i], Y[:, i])[0] for i in range(n)])
    cons = np.empty((N + 7, n))
    cons[0] = rho
    cons[1:4] = rho * vel
    cons[4] = rho * (e + 0.5 * (vel ** 2).sum(axis=0))
    cons[5:5 + N] = rho * Y
    cons[5 + N] = 1000.0                                 # initial guess only
    cons[6 + N] = h
    return np.ascontiguousarray(cons), e


def test_react_conserved_is_newton_then_the_chemistry_step(mech9_path, omech9):
    """The conserved-variable step equals the primitive step from the Newton
    temperature, keeps rho, momentum and rho E, conserves mass and (to the
    integration tolerance) internal energy, and does not depend on the flow
    velocity except through e."""
    rng = np.random.Generator(np.random.PCG64(53))
    s, hot = wl.front_2d(mech9_path, nx=128, ny=128, seed=5, band=6)
    prim = np.ascontiguousarray(s[:, np.where(hot)[0][:60]])
    cons, e0 = _conserved(omech9, mech9_path, prim, rng)
    before = cons.copy()
    st, cn = omech9.react_conserved(cons, wl.DT_FLOW)
    assert (st == 0).all()
    ref = prim.copy()
    rho = before[0]
    ref[1:10] = before[5:14] / rho                        # the composition the step sees
    e_in = before[4] / rho - 0.5 * (before[1:4] ** 2).sum(axis=0) / (rho * rho)
    ref[0] = [omech9.calculate_T(ref[1:10, i], e_in[i], 1000.0)[0] for i in range(60)]
    rst, rcn = omech9.integrate(ref, wl.DT_FLOW)
    assert np.array_equal(cons[5:14], rho * ref[1:10])
    assert np.array_equal(cons[14], ref[0]) and np.array_equal(cn, rcn)
    assert np.array_equal(cons[:5], before[:5])
    assert np.allclose(cons[5:14].sum(axis=0), cons[0], rtol=1e-14)
    e1 = np.array([omech9.energy(cons[14, i], cons[5:14, i] / cons[0, i])[0] for i in range(60)])
    cv = np.array([omech9.energy(cons[14, i], cons[5:14, i] / cons[0, i])[1] for i in range(60)])
    assert np.abs((e1 - e0) / cv).max() < 1e-3            # kelvin, integration error only
    still = before.copy()
    still[1:4] = 0.0
    still[4] = cons[0] * e0                               # same e, no motion
    omech9.react_conserved(still, wl.DT_FLOW)
    # equal up to the rounding of E - |u|^2/2 carried through one flow step
    assert np.allclose(still[5:15], cons[5:15], rtol=1e-8, atol=1e-16)
