"""Pins of the oracle's implicit comparator: the Rosenbrock step (Shampine's
fourth-order parameter set in the Kaps-Rentrop form, embedded third order)
with the exact Jacobian by complex-step differentiation.

Each check is independent of the oracle's own arithmetic: finite
differences of the RHS, the exponential as the stability function's target,
convergence rates, the isomer's closed form, conservation laws and agreement
with the independently pinned explicit scheme."""
import math

import numpy as np
import pytest

import oracle
from paper_2506_02602_amd import workloads as wl


def _cell(path, T, p_atm, Y=None, seed=0):
    names, W = wl.read_species(path)
    rng = np.random.Generator(np.random.PCG64(seed))
    if Y is None:
        Y = wl.base_mixture(names, W, 1, rng)[:, 0]
    rho = wl.density(np.array([T]), np.array([p_atm * wl.P_ATM]), Y[:, None], W)[0]
    return rho, np.concatenate([[T], Y])


def _hot_states(path, n, seed):
    s, hot = wl.front_2d(path, nx=256, ny=256, seed=seed, band=6)
    return np.ascontiguousarray(s[:, np.where(hot)[0][:n]])


def _fd_jacobian(m, rho, u, rel, floor):
    """Central differences with one Richardson extrapolation (error O(d^4));
    the step is rel * max(|u_k|, floor), large enough that rounding in the
    temperature row's quotient stays below the truncation error."""
    n = len(u)
    J = np.zeros((n, n))
    for k in range(n):
        d = rel * max(abs(u[k]), floor)

        def D(dd):
            up, um = u.copy(), u.copy()
            up[k] += dd
            um[k] -= dd
            return (m.rhs(rho, up) - m.rhs(rho, um)) / (2 * dd)

        J[:, k] = (4 * D(d / 2) - D(d)) / 3
    return J


@pytest.mark.parametrize("mechname", ["mech9", "mech32"])
def test_jacobian_matches_finite_differences(mechname):
    """Complex-step df/du against extrapolated central differences at a cold,
    an igniting and a hot state (both NASA-7 ranges), column by column
    relative to the column's size."""
    path = wl.mech_file(mechname)
    m = oracle.Mech(path)
    s = _hot_states(path, 1, seed=31)
    N = m.ns
    states = [_cell(path, 300.0, 1.0), _cell(path, 1200.0, 2.0),
              (s[N + 1, 0], np.r_[s[0, 0], s[1:N + 1, 0]])]
    for rho, u in states:
        u = u.copy()
        u[1:] = np.maximum(u[1:], 1e-6)          # every species present: all columns live
        J = m.jacobian(rho, u)
        Jf = _fd_jacobian(m, rho, u, 1e-3, 1e-2)
        scale = np.abs(Jf).max(axis=0) + 1e-300
        assert np.all(np.abs(J - Jf) / scale <= 1e-7), np.max(np.abs(J - Jf) / scale)


def test_stability_function_approximates_exp_to_fourth_order():
    """One step on y' = lambda y gives y1 = R(z) y0, z = h lambda: R(z) - e^z
    = O(z^5) (local error falls 32x per halving of z), |R(iy)| <= 1 on the
    imaginary axis (A-stability) and |R| stays below 1 far into the left
    half-plane, where explicit schemes blow up."""
    def R(z):
        return oracle.integrate_linear(np.array([[z]]), [1.0], 1.0, fixed_steps=1,
                                       scheme="ros4")["u"][0]

    for z0 in (-0.4, 0.3):
        # z from 0.05 down to 0.006: past the higher-order terms, above rounding
        errs = [abs(R(z0 / 2 ** i) - math.exp(z0 / 2 ** i)) for i in range(3, 7)]
        for e0, e1 in zip(errs, errs[1:]):
            assert 29 < e0 / e1 < 35
    for y in np.logspace(-3, 4, 50):
        A = np.array([[0.0, -y], [y, 0.0]])          # eigenvalues +-iy
        r = oracle.integrate_linear(A, [1.0, 0.0], 1.0, fixed_steps=1, scheme="ros4")["u"]
        assert np.hypot(*r) <= 1.0 + 1e-13
    for z in (-10.0, -1e3, -1e8):
        assert abs(R(z)) < 1.0


def test_fourth_order_convergence_fixed_steps(mech9_path, omech9):
    """Fixed steps on the chemistry (nonlinear, exact Jacobian): the error in Y
    against a fine reference falls ~16x per halving."""
    for T0 in (1500.0, 1600.0):
        rho, u = _cell(mech9_path, T0, 1.0)
        ref = omech9.integrate_cell(rho, u, 1e-4, fixed_steps=8192, scheme="ros4")["u"]
        errs = [np.abs(omech9.integrate_cell(rho, u, 1e-4, fixed_steps=n, scheme="ros4")["u"]
                       - ref)[1:].max() for n in (256, 512, 1024)]
        for e0, e1 in zip(errs, errs[1:]):
            assert 13 < e0 / e1 < 19


def test_error_estimate_is_third_order(mech9_path, omech9):
    """The embedded error estimate of one step of size h scales as h^4 (the
    local error of a third-order solution): halving h divides it by ~16."""
    rho, u = _cell(mech9_path, 1500.0, 1.0)
    u = omech9.integrate_cell(rho, u, 2e-5)["u"]            # into the ignition transient
    errs = []
    for h in (4e-7, 2e-7, 1e-7, 5e-8):
        r = omech9.integrate_cell(rho, u, h, rtol=1.0, atol=1.0, trace_cap=1, scheme="ros4")
        errs.append(r["trace"][0, 2])
    for e0, e1 in zip(errs, errs[1:]):
        assert 13 < e0 / e1 < 19


def test_isomer_closed_form(isomer_path):
    """A <-> B with kf = kr = k: c_A - c_B decays as exp(-2 k t), T constant,
    including far beyond the explicit stability limit (k dt = 2e3)."""
    m = oracle.Mech(isomer_path)
    k = 2.0e7
    rho, u = _cell(isomer_path, 1400.0, 1.0, Y=np.array([0.9, 0.1]))
    for dt, rtol in ((1e-7, 1e-12), (1e-4, 1e-8)):
        r = m.integrate_cell(rho, u, dt, rtol=rtol, atol=1e-16, scheme="ros4")
        assert r["status"] == 0
        d0, d1 = u[1] - u[2], r["u"][1] - r["u"][2]
        assert abs(d1 - d0 * math.exp(-2 * k * dt)) <= 20 * rtol * abs(d0)
        assert abs(r["u"][0] - 1400.0) < 1e-9
    # the stiff interval takes few steps: the method is not stability-limited
    assert r["nacc"] + r["nrej"] < 200


def test_linear_invariants_preserved(mech9_path, omech9):
    """sum Y and element mass fractions are conserved up to the rounding of
    the linear solves: every conserved linear combination c annihilates f
    and the Jacobian, so c W = c / (gamma h) and each stage increment keeps
    c g = 0 exactly in exact arithmetic.  In floating point the LU solve's
    rounding, amplified by the condition number of W (~1e4-1e5 on hot
    cells), leaves a drift of ~1e-11 per step in the element fractions
    (sum Y stays at plain rounding); a dropped or wrong term would move
    them by ~1e-3."""
    s = _hot_states(mech9_path, 16, seed=21)
    N = omech9.ns
    Y0 = s[1:N + 1].copy()
    st, cnt = omech9.integrate(s, 1e-7, scheme="ros4")
    assert (st == 0).all()
    steps = cnt.sum(axis=0)
    Y1 = s[1:N + 1]
    assert np.all(np.abs(Y1.sum(axis=0) - Y0.sum(axis=0)) <= 1e-15 * (10 + steps))
    aw = omech9.comp * 1.0 / omech9.W[:, None]
    el0, el1 = aw.T @ Y0, aw.T @ Y1
    assert np.all(np.abs(el1 - el0) <= 1e-10 * (10 + steps) * np.abs(el0).max())


def test_agrees_with_the_explicit_scheme(mech9_path, omech9):
    """Two independent integrators converge to the same flow-step result: the
    Rosenbrock and the low-storage explicit scheme at rtol 1e-11 agree to
    1e-9 relative in T and 1e-11 absolute in Y on hot front cells, and at
    the working tolerance to a few tolerance units."""
    s0 = _hot_states(mech9_path, 24, seed=33)
    N = omech9.ns
    a, b = s0.copy(), s0.copy()
    omech9.integrate(a, 1e-7, rtol=1e-11, atol=1e-14, max_steps=1000000, scheme="ros4")
    omech9.integrate(b, 1e-7, rtol=1e-11, atol=1e-14, max_steps=1000000, scheme="lsrk")
    assert np.max(np.abs(a[0] - b[0]) / b[0]) < 1e-9
    assert np.max(np.abs(a[1:N + 1] - b[1:N + 1])) < 1e-11
    c = s0.copy()
    omech9.integrate(c, 1e-7, scheme="ros4")
    assert np.max(np.abs(c[0] - b[0]) / b[0]) < 2e-7
    assert np.max(np.abs(c[1:N + 1] - b[1:N + 1])) < 2e-7


def test_linear_step_is_the_stability_function_of_the_matrix():
    """On u' = A u one step is u1 = R(hA) u0 with R the scalar stability
    function; with A = V D V^-1 that is V R(hD) V^-1 u0 (numpy's eigenvalue
    routine, R from one-component steps).  At h = 1 the matrix W = 2I - A is
    dominated by off-diagonal entries, so the LU factorisation pivots, also
    after the first column: a pin of the row swaps and the solve."""
    rng = np.random.Generator(np.random.PCG64(41))
    n = 7
    lam = -np.logspace(0, 2.5, n) * rng.uniform(0.8, 1.2, n)
    V = rng.normal(size=(n, n))
    A = V @ np.diag(lam) @ np.linalg.inv(V)
    u0 = rng.normal(size=n)
    W = 2.0 * np.eye(n) - A
    # the pivot column changes after the first step of elimination
    assert np.argmax(np.abs(W[:, 0])) != 0

    def R(z):
        return oracle.integrate_linear(np.array([[z]]), [1.0], 1.0, fixed_steps=1,
                                       scheme="ros4")["u"][0]

    expect = V @ np.diag([R(x) for x in lam]) @ np.linalg.solve(V, u0)
    got = oracle.integrate_linear(A, u0, 1.0, fixed_steps=1, scheme="ros4")["u"]
    assert np.allclose(got, expect, rtol=1e-9, atol=1e-9 * np.abs(expect).max())
