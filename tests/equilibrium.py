"""Independent constant-(U, V) chemical equilibrium by element potentials.

Used only by tests to pin the oracle's kinetics to thermodynamics: at the
equilibrium of a closed constant-volume adiabatic cell every reversible
reaction is in detailed balance, so a correct mass-action model with reverse
rates from equilibrium constants must relax to this state.

Method (textbook element-potential formulation): for fixed T the ideal-gas
equilibrium concentrations are c_k = (P_std/(R T)) exp(-g_k/RT + sum_e a_ek l_e),
with l_e found by minimising the convex dual
    F(l) = sum_k c_k(l) - sum_e b_e l_e        (grad = A c - b, Hess = A diag(c) A^T)
by damped Newton.  T is then found by bisection-safe root finding on the
internal-energy balance sum_k c_k U_k(T) = rho * e.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq

R_CGS = 8.31446261815324e7


def _conc(lnc0, Amat, lam):
    return np.exp(lnc0 + Amat.T @ lam)


def element_potentials(lnc0, Amat, b, lam0=None, iters=200):
    """Minimise sum_k exp(lnc0_k + a_k.l) - b.l; returns (l, c)."""
    E = Amat.shape[0]
    if lam0 is None:
        target = np.log(max(b.sum(), 1e-300) / len(lnc0))
        lam, *_ = np.linalg.lstsq(Amat.T, target - lnc0, rcond=None)
    else:
        lam = lam0.copy()

    def F(l):
        return np.exp(lnc0 + Amat.T @ l).sum() - b @ l

    f = F(lam)
    for _ in range(iters):
        c = _conc(lnc0, Amat, lam)
        g = Amat @ c - b
        H = (Amat * c) @ Amat.T
        step = np.linalg.lstsq(H, -g, rcond=None)[0]
        t = 1.0
        while True:
            nl = lam + t * step
            nf = F(nl)
            if nf <= f or t < 1e-12:
                break
            t *= 0.5
        lam, f = nl, nf
        if np.max(np.abs(g) / np.maximum(b, 1e-300)) < 1e-14 and t == 1.0:
            break
    c = _conc(lnc0, Amat, lam)
    return lam, c


def uv_equilibrium(mech, rho, T0, Y0, pstd=1.01325e6, Tbounds=None):
    """Equilibrium (T, Y) at fixed density and internal energy of (T0, Y0).

    ``mech`` is an ``oracle.Mech`` (used only for NASA-7 thermo and the
    species/element tables)."""
    W = mech.W
    Amat = mech.comp.T.astype(float)             # [E, N]
    c_init = rho * Y0 / W
    b = Amat @ c_init
    keep = b > 0
    Amat = Amat[keep]
    b = b[keep]

    def U_molar(T):
        _, h, _ = mech.thermo(T)
        return R_CGS * T * (h - 1.0)             # erg/mol

    e_vol = float(c_init @ U_molar(T0))          # rho * e, erg/cm^3

    def solve_T(T):
        _, h, s = mech.thermo(T)
        lnc0 = np.log(pstd / (R_CGS * T)) - (h - s)
        lam, c = element_potentials(lnc0, Amat, b, None)
        lam, c = element_potentials(lnc0, Amat, b, lam)
        return c

    def resid(T):
        c = solve_T(T)
        return float(c @ U_molar(T)) - e_vol

    if Tbounds is None:
        Tbounds = (0.5 * T0, 6000.0)
    T = brentq(resid, *Tbounds, xtol=1e-12, rtol=1e-15, maxiter=500)
    c = solve_T(T)
    return T, c * W / rho, c
