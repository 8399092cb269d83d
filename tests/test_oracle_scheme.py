"""Pins for the oracle's integrator core: the LSRK scheme (Eq. 21), its
embedded error register and the WRMS step control (Eq. 22).

Every expected value here comes from exact rational arithmetic on the
published tableau, from mpmath, or from the paper's stated constants -- never
from the code under test."""
import os
from fractions import Fraction as Fr

import mpmath as mp
import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load_tableau():
    vals = {}
    with open(os.path.join(GOLD, "lsrk_rk4_3_5_2rplus.txt")) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            name, num, den = ln.split()
            vals[name] = Fr(int(num), int(den))
    a = [vals[k] for k in ("a21", "a32", "a43", "a54")]
    b = [vals[f"b{i}"] for i in range(1, 6)]
    bh = [vals[f"bh{i}"] for i in range(1, 6)]
    return a, b, bh


def _load_control():
    out = {}
    with open(os.path.join(GOLD, "paper_step_control.txt")) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            k, v = ln.split()
            out[k] = float(v)
    return out


def _butcher(a, b):
    """Full Butcher matrix of a 2R scheme: a_ij = b_j for j < i-1."""
    s = len(b)
    A = [[Fr(0)] * s for _ in range(s)]
    for i in range(1, s):
        for j in range(i - 1):
            A[i][j] = b[j]
        A[i][i - 1] = a[i - 1]
    return A


def _dot(x, y):
    return sum(p * q for p, q in zip(x, y))


def _mv(M, v):
    return [_dot(r, v) for r in M]


def _order_residuals(A, w):
    one = [Fr(1)] * len(w)
    c = _mv(A, one)
    return [
        _dot(w, one) - 1,
        _dot(w, c) - Fr(1, 2),
        _dot(w, [x * x for x in c]) - Fr(1, 3),
        _dot(w, _mv(A, c)) - Fr(1, 6),
        _dot(w, [x ** 3 for x in c]) - Fr(1, 4),
        _dot(w, [ci * y for ci, y in zip(c, _mv(A, c))]) - Fr(1, 8),
        _dot(w, _mv(A, [x * x for x in c])) - Fr(1, 12),
        _dot(w, _mv(A, _mv(A, c))) - Fr(1, 24),
    ]


def _stab_coeffs(A, w):
    """gamma_k of R(z) = sum_k gamma_k z^k, gamma_k = w^T A^(k-1) 1."""
    s = len(w)
    v = [Fr(1)] * s
    g = [Fr(1)]
    for _ in range(s):
        g.append(_dot(w, v))
        v = _mv(A, v)
    return g


def test_order_conditions_exact():
    a, b, bh = _load_tableau()
    A = _butcher(a, b)
    rb = _order_residuals(A, b)
    assert max(abs(float(r)) for r in rb) < 1e-24          # order 4 (rational approximations)
    rbh = _order_residuals(A, bh)
    assert max(abs(float(r)) for r in rbh[:4]) < 1e-24      # embedded: order 3
    assert max(abs(float(r)) for r in rbh[4:]) > 1e-3       # ... and not order 4


def test_oracle_coefficients_are_correctly_rounded():
    a, b, bh = _load_tableau()
    oa, ob, obh = oracle.lsrk_coeffs()
    assert list(oa) == [float(x) for x in a]
    assert list(ob) == [float(x) for x in b]
    assert list(obh) == [float(x) for x in bh]


def test_stability_polynomial():
    a, b, _ = _load_tableau()
    g = _stab_coeffs(_butcher(a, b), b)
    for k, exact in enumerate([1, 1, Fr(1, 2), Fr(1, 6), Fr(1, 24)]):
        assert abs(float(g[k] - exact)) < 1e-24
    assert abs(float(1 / g[5]) - 206.0) < 1e-6


def _R(gam, z):
    return sum(mp.mpf(gk.numerator) / gk.denominator * z ** k for k, gk in enumerate(gam))


@pytest.mark.parametrize("lam,h,n", [(-3.0, 0.1, 10), (-1.0, 1.0, 7), (-40.0, 0.1, 5),
                                     (2.0, 0.05, 20)])
def test_dahlquist_fixed_steps(lam, h, n):
    """y' = lam y in n fixed steps gives R(h lam)^n y0 (R from the tableau)."""
    a, b, _ = _load_tableau()
    gam = _stab_coeffs(_butcher(a, b), b)
    mp.mp.dps = 40
    expect = float(_R(gam, mp.mpf(lam) * mp.mpf(h)) ** n)
    r = oracle.integrate_linear(np.array([[lam]]), [1.0], h * n, fixed_steps=n)
    assert r["u"][0] == pytest.approx(expect, rel=1e-13, abs=1e-300)


def test_dahlquist_complex_eigenvalue():
    """A 2x2 rotation-dilation block stands for lam = alpha + i beta."""
    a, b, _ = _load_tableau()
    gam = _stab_coeffs(_butcher(a, b), b)
    al, be, h, n = -0.5, 3.0, 0.2, 15
    mp.mp.dps = 40
    z = mp.mpc(al, be) * h
    Rn = _R(gam, z) ** n
    A = np.array([[al, -be], [be, al]])
    r = oracle.integrate_linear(A, [1.0, 0.0], h * n, fixed_steps=n)
    assert r["u"][0] == pytest.approx(float(mp.re(Rn)), abs=1e-13)
    assert r["u"][1] == pytest.approx(float(mp.im(Rn)), abs=1e-13)


def test_real_stability_boundary():
    """|R(z)| < 1 just inside z = -4.8, > 1 just outside (degree-5 term matters)."""
    inside = oracle.integrate_linear(np.array([[-4.75]]), [1.0], 200.0, fixed_steps=200)
    outside = oracle.integrate_linear(np.array([[-4.90]]), [1.0], 200.0, fixed_steps=200)
    assert abs(inside["u"][0]) < 1.0
    assert abs(outside["u"][0]) > 1.0


def test_error_register_first_step():
    """First-step WRMS error equals |R(z) - Rhat(z)| |y0| / (rtol |y0| + atol)."""
    a, b, bh = _load_tableau()
    A = _butcher(a, b)
    g, gh = _stab_coeffs(A, b), _stab_coeffs(A, bh)
    mp.mp.dps = 40
    lam, y0, dt, rtol, atol = -2.0, 3.0, 0.3, 1e-6, 1e-10
    z = mp.mpf(lam) * mp.mpf(dt)
    est = abs(_R(g, z) - _R(gh, z)) * y0 / (rtol * y0 + atol)
    r = oracle.integrate_linear(np.array([[lam]]), [y0], dt, rtol=rtol, atol=atol,
                                trace_cap=50)
    assert r["trace"][0, 1] == dt
    assert r["trace"][0, 2] == pytest.approx(float(est), rel=1e-9)


def test_step_factor_constants_from_paper():
    """Eq. 22: factor = clamp(beta * err^(-1/4), 1/5, 5); accept iff err <= 1."""
    k = _load_control()
    lam = -1.0
    # a huge first step: error >> 1, so the factor hits the 1/5 floor
    r = oracle.integrate_linear(np.array([[lam]]), [1.0], 1e3, rtol=1e-6, atol=1e-10,
                                h0=1e3, trace_cap=10)
    tr = r["trace"]
    assert tr[0, 3] == 0 and tr[0, 2] > 1
    assert tr[1, 1] == pytest.approx(tr[0, 1] * k["factor_min"], rel=1e-15)
    # a tiny first step: error << 1, so the factor hits the 5x ceiling
    r = oracle.integrate_linear(np.array([[lam]]), [1.0], 1.0, rtol=1e-6, atol=1e-10,
                                h0=1e-9, trace_cap=10)
    tr = r["trace"]
    assert tr[0, 3] == 1
    assert tr[1, 1] == pytest.approx(tr[0, 1] * k["factor_max"], rel=1e-15)
    # unclamped region: next h = h * beta * err^(-exponent)
    for i in range(len(tr) - 1):
        fac = k["beta"] * tr[i, 2] ** (-k["exponent"])
        if k["factor_min"] < fac < k["factor_max"] and tr[i + 1, 1] != 1.0 - tr[i + 1, 0]:
            assert tr[i + 1, 1] == pytest.approx(tr[i, 1] * fac, rel=1e-14)
    # accepted iff err <= 1
    assert all((row[2] <= 1.0) == bool(row[3]) for row in tr)


def test_adaptive_accuracy_and_tolerance_proportionality():
    """y' = -y on [0, 1]: error of the order of tol and shrinking with tol."""
    errs = []
    for tol in (1e-6, 1e-8, 1e-10):
        r = oracle.integrate_linear(np.array([[-1.0]]), [1.0], 1.0, rtol=tol, atol=1e-14)
        assert r["status"] == oracle.STATUS_OK
        errs.append(abs(r["u"][0] - np.exp(-1.0)))
    assert errs[0] < 20 * 1e-6 and errs[1] < 20 * 1e-8 and errs[2] < 20 * 1e-10
    assert errs[1] < errs[0] / 10 and errs[2] < errs[1] / 10


def test_last_step_lands_on_dt_and_steps_counted():
    r = oracle.integrate_linear(np.array([[-1.0]]), [1.0], 1.0, rtol=1e-8, atol=1e-12,
                                trace_cap=1000)
    tr = r["trace"]
    acc = tr[tr[:, 3] == 1]
    assert acc[-1, 0] + acc[-1, 1] == pytest.approx(1.0, rel=1e-15)
    assert r["nacc"] == len(acc) and r["nrej"] == len(tr) - len(acc)


def test_embedded_local_error_order():
    """Local error estimate scales like h^4 (embedded order 3) on a smooth problem."""
    e = []
    for h in (0.08, 0.04, 0.02):
        r = oracle.integrate_linear(np.array([[-1.0]]), [1.0], h, rtol=1.0, atol=1.0,
                                    trace_cap=2)
        e.append(r["trace"][0, 2])
    assert e[0] / e[1] == pytest.approx(16.0, rel=0.05)
    assert e[1] / e[2] == pytest.approx(16.0, rel=0.03)


# ------------------------------------------- full-storage comparison scheme

def _load_rkf45():
    vals = {}
    with open(os.path.join(GOLD, "rkf45_fehlberg.txt")) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            name, num, den = ln.split()
            vals[name] = Fr(int(num), int(den))
    A = [[vals.get(f"a{i}{j}", Fr(0)) for j in range(1, 7)] for i in range(1, 7)]
    b4 = [vals[f"b4_{i}"] for i in range(1, 7)]
    b5 = [vals[f"b5_{i}"] for i in range(1, 7)]
    return A, b4, b5


def _order5_residuals(A, w):
    one = [Fr(1)] * len(w)
    c = _mv(A, one)
    Ac = _mv(A, c)
    c2 = [x * x for x in c]
    return [
        _dot(w, [x ** 4 for x in c]) - Fr(1, 5),
        _dot(w, [ci * ci * y for ci, y in zip(c, Ac)]) - Fr(1, 10),
        _dot(w, [ci * y for ci, y in zip(c, _mv(A, c2))]) - Fr(1, 15),
        _dot(w, [ci * y for ci, y in zip(c, _mv(A, Ac))]) - Fr(1, 30),
        _dot(w, [y * y for y in Ac]) - Fr(1, 20),
        _dot(w, _mv(A, [x ** 3 for x in c])) - Fr(1, 20),
        _dot(w, _mv(A, [ci * y for ci, y in zip(c, Ac)])) - Fr(1, 40),
        _dot(w, _mv(A, _mv(A, c2))) - Fr(1, 60),
        _dot(w, _mv(A, _mv(A, Ac))) - Fr(1, 120),
    ]


def test_rkf45_order_conditions_exact():
    """Fourth-order weights satisfy the 8 order-4 conditions exactly, the
    fifth-order ones also the 9 order-5 conditions; the fourth-order weights
    do not."""
    A, b4, b5 = _load_rkf45()
    assert all(r == 0 for r in _order_residuals(A, b4))
    assert all(r == 0 for r in _order_residuals(A, b5))
    assert all(r == 0 for r in _order5_residuals(A, b5))
    assert any(r != 0 for r in _order5_residuals(A, b4))


def test_rkf45_oracle_coefficients_are_correctly_rounded():
    A, b4, b5 = _load_rkf45()
    oa, ob4, ob5 = oracle.rkf45_coeffs()
    for i in range(6):
        for j in range(i):
            assert oa[i, j] == float(A[i][j])
    assert list(ob4) == [float(x) for x in b4]
    assert list(ob5) == [float(x) for x in b5]


@pytest.mark.parametrize("lam,h,n", [(-3.0, 0.1, 10), (-1.0, 1.0, 7), (2.0, 0.05, 20)])
def test_rkf45_dahlquist_fixed_steps(lam, h, n):
    """y' = lam y with the full-storage scheme: R4(h lam)^n from its tableau."""
    A, b4, _ = _load_rkf45()
    gam = _stab_coeffs(A, b4)
    mp.mp.dps = 40
    expect = float(_R(gam, mp.mpf(lam) * mp.mpf(h)) ** n)
    r = oracle.integrate_linear(np.array([[lam]]), [1.0], h * n, fixed_steps=n, scheme="rkf45")
    assert r["u"][0] == pytest.approx(expect, rel=1e-13)


def test_rkf45_error_estimate_and_exponent():
    """First-step error = |R5(z) - R4(z)| |y0| / (rtol |y0| + atol); the next
    step is h * clamp(0.9 err^(-1/5), 1/5, 5) (fourth-order estimate)."""
    A, b4, b5 = _load_rkf45()
    g4, g5 = _stab_coeffs(A, b4), _stab_coeffs(A, b5)
    mp.mp.dps = 40
    lam, y0, dt, rtol, atol = -2.0, 3.0, 0.3, 1e-6, 1e-10
    z = mp.mpf(lam) * mp.mpf(dt)
    est = float(abs(_R(g5, z) - _R(g4, z)) * y0 / (rtol * y0 + atol))
    r = oracle.integrate_linear(np.array([[lam]]), [y0], dt, rtol=rtol, atol=atol,
                                trace_cap=50, scheme="rkf45")
    tr = r["trace"]
    assert tr[0, 2] == pytest.approx(est, rel=1e-9)
    assert tr[0, 3] == 0                                   # rejected (err >> 1)
    fac = min(max(0.9 * est ** -0.2, 0.2), 5.0)
    assert tr[1, 1] == pytest.approx(dt * fac, rel=1e-12)
