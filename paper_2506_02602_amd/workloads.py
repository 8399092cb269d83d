"""Seeded synthetic input fields (inputs only; none of the method's arithmetic).

Every generator returns a state block in the library's SoA layout,
``state[v, i]`` with rows ``0: T [K]``, ``1..N: Y_k``, ``N+1: rho [g/cm^3]``,
``N+2: h`` (step hint, 0 = use dt).  Density comes from the ideal-gas law
``rho = p / (R T sum_k Y_k/W_k)`` so that the fields are specified, as in the
paper's chemistry benchmark (Sec. 4.2.2), by temperature, pressure and
composition.  All randomness is ``numpy.random.Generator(PCG64(seed))``.

Workloads (the paper's 13-species mechanism and its benchmark geometry are not
available; these seeded fields stand in for its reacting-front workloads):

* ``cells_uniform``   4096 independent cells, T ~ U[1000, 1600] K, 1 atm,
                      stoichiometric H2/O2/N2 (2 : 1 : 3.76) with +-5 % jitter;
* ``front_2d``        1024 x 1024 field with a sinusoidal hot band of ~2 % of
                      the cells (T ~ U[1500, 3000] K, p ~ U[5, 30] atm), the rest
                      at 300 K, 1 atm, Gaussian mass-fraction noise 1e-3;
* ``amr_hierarchy``   3 levels, ratio 2, 16/32/48 boxes with edges drawn from
                      {16, 32, 48, 64}^3, a hot ellipsoid in each finest box;
* ``stress_3d``       256 x 256 x 64 cells, T ~ U[900, 2800] K,
                      p ~ U[1, 40] atm, independent per cell.
"""
from __future__ import annotations

import math
import os

import numpy as np

R_CGS = 8.31446261815324e7
P_ATM = 1.01325e6
DT_FLOW = 1.0e-7
RTOL = 1.0e-8
ATOL = 1.0e-10


def read_species(path: str):
    """Species names and molecular weights from a ``.mech`` file."""
    names, W = [], []
    with open(path) as f:
        lines = [ln for ln in f if ln.strip() and not ln.lstrip().startswith("#")]
    i = 0
    while i < len(lines):
        tok = lines[i].split()
        if tok[0] == "species":
            n = int(tok[1])
            for ln in lines[i + 1:i + 1 + n]:
                t = ln.split()
                names.append(t[0])
                W.append(float(t[1]))
            break
        i += 1
    return names, np.array(W)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def density(T, p, Y, W):
    """Ideal-gas density for arrays T[n], p[n], Y[N, n]."""
    inv_w = (Y / W[:, None]).sum(axis=0)
    return p / (R_CGS * T * inv_w)


def base_mixture(names, W, n, rng, jitter=0.05):
    """Stoichiometric H2/O2/N2 mole fractions 2 : 1 : 3.76, each x (1 + U[-j, j])."""
    N = len(names)
    X = np.zeros((N, n))
    for sp, x in (("H2", 2.0), ("O2", 1.0), ("N2", 3.76)):
        X[names.index(sp)] = x * (1.0 + rng.uniform(-jitter, jitter, size=n))
    X /= X.sum(axis=0, keepdims=True)
    Y = X * W[:, None]
    Y /= Y.sum(axis=0, keepdims=True)
    return Y


def pack(T, Y, rho, h=None):
    N, n = Y.shape
    s = np.empty((N + 3, n), dtype=np.float64)
    s[0] = T
    s[1:N + 1] = Y
    s[N + 1] = rho
    s[N + 2] = 0.0 if h is None else h
    return s


def cells_uniform(mech_path, n=4096, seed=1):
    names, W = read_species(mech_path)
    rng = _rng(seed)
    T = rng.uniform(1000.0, 1600.0, size=n)
    Y = base_mixture(names, W, n, rng)
    p = np.full(n, P_ATM)
    return pack(T, Y, density(T, p, Y, W))


def _noisy(Y, rng, sigma=1e-3):
    Y = Y + rng.normal(0.0, sigma, size=Y.shape)
    Y = np.clip(Y, 0.0, None)
    return Y / Y.sum(axis=0, keepdims=True)


def front_2d(mech_path, nx=1024, ny=1024, seed=2, band=None):
    """Reacting-front field; cell i = y * nx + x.  Returns (state, hot_mask)."""
    names, W = read_species(mech_path)
    rng = _rng(seed)
    n = nx * ny
    x = np.tile(np.arange(nx), ny)
    y = np.repeat(np.arange(ny), nx)
    half = 0.01 * ny if band is None else band
    yc = ny / 2 + (ny / 16) * np.sin(2 * math.pi * x / nx)
    hot = np.abs(y - yc) < half
    T = np.full(n, 300.0)
    p = np.full(n, P_ATM)
    nh = int(hot.sum())
    T[hot] = rng.uniform(1500.0, 3000.0, size=nh)
    p[hot] = rng.uniform(5.0, 30.0, size=nh) * P_ATM
    Y = _noisy(base_mixture(names, W, n, rng), rng)
    return pack(T, Y, density(T, p, Y, W)), hot


def amr_hierarchy(mech_path, seed=3, boxes_per_level=(16, 32, 48),
                  edges=(16, 32, 48, 64), dt0=DT_FLOW):
    """Boxes of a 3-level hierarchy (ratio 2, dt halved per level).

    Returns a list of dicts: state (SoA block), level, dt, n_sub, hot_mask."""
    names, W = read_species(mech_path)
    rng = _rng(seed)
    out = []
    for lev, nb in enumerate(boxes_per_level):
        for _ in range(nb):
            ex, ey, ez = (int(rng.choice(edges)) for _ in range(3))
            n = ex * ey * ez
            T = np.full(n, 300.0)
            p = np.full(n, P_ATM)
            hot = np.zeros(n, dtype=bool)
            if lev == len(boxes_per_level) - 1:
                # hot ellipsoid holding ~25 % of the box's cells
                gx, gy, gz = np.meshgrid(np.arange(ex), np.arange(ey), np.arange(ez),
                                         indexing="ij")
                c = [rng.uniform(0.3, 0.7) * e for e in (ex, ey, ez)]
                r = [0.391 * e for e in (ex, ey, ez)]  # (4/3)pi r^3 = 0.25 box
                d = (((gx - c[0]) / r[0]) ** 2 + ((gy - c[1]) / r[1]) ** 2 +
                     ((gz - c[2]) / r[2]) ** 2)
                hot = (d < 1.0).reshape(-1)
                nh = int(hot.sum())
                T[hot] = rng.uniform(1500.0, 3000.0, size=nh)
                p[hot] = rng.uniform(5.0, 30.0, size=nh) * P_ATM
            Y = _noisy(base_mixture(names, W, n, rng), rng)
            out.append(dict(state=pack(T, Y, density(T, p, Y, W)), level=lev,
                            dt=dt0 / 2 ** lev, n_sub=2 ** lev, hot=hot,
                            shape=(ex, ey, ez)))
    return out


def stress_3d(mech_path, shape=(256, 256, 64), seed=4):
    """Independent per-cell T ~ U[900, 2800] K, p ~ U[1, 40] atm.

    Composition: the stoichiometric H2/O2/N2 base; if the mechanism has
    carbon species, 10 % of the fuel moles go to CH4 (else nothing); every
    other species gets a log-uniform trace in [1e-6, 1e-3]; renormalised."""
    names, W = read_species(mech_path)
    rng = _rng(seed)
    n = int(np.prod(shape))
    T = rng.uniform(900.0, 2800.0, size=n)
    p = rng.uniform(1.0, 40.0, size=n) * P_ATM
    Y = base_mixture(names, W, n, rng)
    if "CH4" in names:
        k = names.index("H2")
        Y[names.index("CH4")] = 0.1 * Y[k]
        Y[k] *= 0.9
    base = {"H2", "O2", "N2", "CH4"}
    for k, nm in enumerate(names):
        if nm not in base:
            Y[k] = 10.0 ** rng.uniform(-6.0, -3.0, size=n)
    Y /= Y.sum(axis=0, keepdims=True)
    return pack(T, Y, density(T, p, Y, W))


def diverge_temperature(y, L, alpha, T_low=1000.0, T_high=1600.0, y_m=None):
    """The paper's test temperature profile (Sec. 4.2.2, Eq. 27) with the
    parameters of Eq. 28: T_b + T_r tanh(k (y - y_m)/L) +
    A exp(-8 ((y - y_m)/L)^2) cos(2 pi f y / L), k = 6/alpha, f = 4/alpha,
    A = 50/alpha.  T_low, T_high and y_m are not given there; the readings
    are 1000 K, 1600 K and L/2."""
    y = np.asarray(y, dtype=np.float64)
    y_m = 0.5 * L if y_m is None else y_m
    k, f, A = 6.0 / alpha, 4.0 / alpha, 50.0 / alpha
    T_b, T_r = 0.5 * (T_high + T_low), 0.5 * (T_high - T_low)
    z = (y - y_m) / L
    return T_b + T_r * np.tanh(k * z) + A * np.exp(-8.0 * z * z) * np.cos(2.0 * np.pi * f * y / L)


def diverge_box(mech_path, alpha, shape=(16, 256, 16), p=P_ATM):
    """The thread-coherence (alpha = 1) / thread-divergence (alpha = 0.1)
    workload of Sec. 4.2.2: 16 x 256 x 16 = 65,536 cells on a unit box, T
    varying in y only (cell centres, Eq. 27-28), uniform composition
    H2 : O2 : N2 = 1 : 2 : 7 by mole, 1 atm (the pressure is not given).
    Cells are ordered x fastest, then y, then z.  Integrated as 100 calls of
    dt = 1e-5 s (Tables 4-5)."""
    names, W = read_species(mech_path)
    nx, ny, nz = shape
    L = 1.0
    y = (np.arange(ny) + 0.5) * (L / ny)
    Ty = diverge_temperature(y, L, alpha)
    T = np.broadcast_to(Ty[None, :, None], (nz, ny, nx)).reshape(-1).copy()
    n = T.size
    X = np.zeros(len(names))
    for sp, x in (("H2", 1.0), ("O2", 2.0), ("N2", 7.0)):
        X[names.index(sp)] = x
    Y1 = X * W / np.sum(X * W)
    Y = np.repeat(Y1[:, None], n, axis=1)
    rho = density(T, np.full(n, p), Y, W)
    return pack(T, Y, rho)


DIVERGE_DT = 1.0e-5
DIVERGE_CALLS = 100


def mech_file(name: str) -> str:
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "mech", name + ".mech")
