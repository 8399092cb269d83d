"""CPU FP64 oracle for the per-cell chemistry path -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never links or calls it, and it
shares no code with the GPU path: the chemistry is a plain C program
(``chem_oracle.c``) that interprets the ``.mech`` table at run time, and the
surrogate oracle (``mlp_oracle.py``) is plain numpy.

``build()`` compiles the C oracle into ``liboracle.so`` beside this file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "chem_oracle.c")

STATUS_OK, STATUS_MAXSTEPS, STATUS_NONFINITE, STATUS_H_UNDERFLOW = 0, 1, 2, 3


def build() -> str:
    """Compile the oracle (portable x86-64 code, no FP contraction)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", LIB_PATH + ".tmp", SRC_PATH, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None
_lib_path = LIB_PATH


def use_native_build(out_dir: str) -> str:
    """Compile the oracle for the host that runs it (-O3 -march=native; still
    no FP contraction and no fast-math, so it computes the same numbers as
    the portable build) into out_dir and make it the library this module
    loads.  Must be called before the library is first used.  For timing the
    oracle on the machine it runs on; the tests use the portable build."""
    global _lib_path
    if _lib is not None:
        raise RuntimeError("oracle library already loaded")
    path = os.path.join(out_dir, f"liboracle_native_{os.getpid()}.so")
    cmd = ["gcc", "-O3", "-march=native", "-std=c99", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-fPIC", "-shared", "-o", path, SRC_PATH, "-lm"]
    subprocess.run(cmd, check=True)
    _lib_path = path
    return path


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_lib_path):
            build()
        L = C.CDLL(_lib_path)
        P, D, I = C.c_void_p, C.c_double, C.c_int
        L.or_mech_load.argtypes = [C.c_char_p, C.POINTER(C.c_void_p)]
        L.or_mech_load.restype = I
        L.or_mech_free.argtypes = [P]
        L.or_mech_dims.argtypes = [P, C.POINTER(I), C.POINTER(I), C.POINTER(I)]
        L.or_mech_species.argtypes = [P, P, P]
        L.or_mech_elements.argtypes = [P, P]
        L.or_mech_stoich.argtypes = [P, P]
        L.or_thermo.argtypes = [P, D, P, P, P]
        L.or_rates.argtypes = [P, D, P, P, P, P, P]
        L.or_rhs.argtypes = [P, D, P, P]
        L.or_jacobian.argtypes = [P, D, P, P]
        L.or_lsrk_coeffs.argtypes = [P, P, P]
        L.or_integrate_cell.argtypes = [P, D, P, D, D, D, I, I, C.POINTER(D), C.POINTER(I),
                                        C.POINTER(I), P, I, C.POINTER(I)]
        L.or_integrate_cell.restype = I
        L.or_integrate.argtypes = [P, P, C.c_int64, C.c_int64, D, D, D, I, I, I, P, P]
        L.or_integrate.restype = I
        L.or_integrate_linear.argtypes = [I, P, P, D, D, D, I, I, C.POINTER(D), C.POINTER(I),
                                          C.POINTER(I), P, I, C.POINTER(I)]
        L.or_integrate_linear.restype = I
        L.or_rkf45_coeffs.argtypes = [P, P, P]
        L.or_energy.argtypes = [P, D, P, C.POINTER(D), C.POINTER(D)]
        L.or_calculate_T.argtypes = [P, P, D, D, C.POINTER(D)]
        L.or_calculate_T.restype = I
        L.or_react_conserved.argtypes = [P, P, C.c_int64, C.c_int64, D, D, D, I, P, P]
        L.or_react_conserved.restype = I
        L.or_integrate_cell_scheme.argtypes = [I] + L.or_integrate_cell.argtypes
        L.or_integrate_cell_scheme.restype = I
        L.or_integrate_scheme.argtypes = [I] + L.or_integrate.argtypes
        L.or_integrate_scheme.restype = I
        L.or_integrate_linear_scheme.argtypes = [I] + L.or_integrate_linear.argtypes
        L.or_integrate_linear_scheme.restype = I
        L.or_set_perturbation.argtypes = [I]
        L.or_set_perturbation.restype = None
        _lib = L
    return _lib


def set_perturbation(mode: int) -> None:
    """Last-bit perturbations of the oracle (bits: 1 k_f one ulp up, 2 the
    step factor via two square roots, 4 production rates summed in reverse
    reaction order, 8 k_r from one exponential); 0 = off.  For the parity
    budget study only; process-wide, set while nothing integrates."""
    lib().or_set_perturbation(int(mode))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def lsrk_coeffs():
    a, b, bh = np.zeros(4), np.zeros(5), np.zeros(5)
    lib().or_lsrk_coeffs(_ptr(a), _ptr(b), _ptr(bh))
    return a, b, bh


SCHEMES = {"lsrk": 0, "rkf45": 1, "ros4": 2}


def rkf45_coeffs():
    """Fehlberg 4(5): A[6][5] (row i: a_i1..a_i5), fourth- and fifth-order weights."""
    a, b4, b5 = np.zeros(30), np.zeros(6), np.zeros(6)
    lib().or_rkf45_coeffs(_ptr(a), _ptr(b4), _ptr(b5))
    return a.reshape(6, 5), b4, b5


class Mech:
    """A parsed mechanism (table form) on the CPU."""

    def __init__(self, path: str):
        h = C.c_void_p()
        rc = lib().or_mech_load(path.encode(), C.byref(h))
        if rc != 0:
            raise ValueError(f"oracle: cannot parse {path} (line {rc})")
        self._h = h
        ne, ns, nr = C.c_int(), C.c_int(), C.c_int()
        lib().or_mech_dims(h, C.byref(ne), C.byref(ns), C.byref(nr))
        self.ne, self.ns, self.nr = ne.value, ns.value, nr.value
        self.W = np.zeros(self.ns)
        self.comp = np.zeros((self.ns, self.ne), dtype=np.int32)
        lib().or_mech_species(h, _ptr(self.W), _ptr(self.comp))
        self.ew = np.zeros(self.ne)
        lib().or_mech_elements(h, _ptr(self.ew))
        self.nu = np.zeros((self.nr, self.ns))
        lib().or_mech_stoich(h, _ptr(self.nu))

    def __del__(self):
        try:
            lib().or_mech_free(self._h)
        except Exception:
            pass

    def thermo(self, T: float):
        cp, h, s = np.zeros(self.ns), np.zeros(self.ns), np.zeros(self.ns)
        lib().or_thermo(self._h, float(T), _ptr(cp), _ptr(h), _ptr(s))
        return cp, h, s

    def rates(self, rho: float, u: np.ndarray):
        u = np.ascontiguousarray(u, dtype=np.float64)
        kf, kr, q, w = (np.zeros(self.nr), np.zeros(self.nr), np.zeros(self.nr),
                        np.zeros(self.ns))
        lib().or_rates(self._h, float(rho), _ptr(u), _ptr(kf), _ptr(kr), _ptr(q), _ptr(w))
        return kf, kr, q, w

    def rhs(self, rho: float, u: np.ndarray) -> np.ndarray:
        u = np.ascontiguousarray(u, dtype=np.float64)
        f = np.zeros(self.ns + 1)
        lib().or_rhs(self._h, float(rho), _ptr(u), _ptr(f))
        return f

    def jacobian(self, rho: float, u: np.ndarray) -> np.ndarray:
        """df/du of the RHS at u = (T, Y) by complex-step differentiation."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        J = np.zeros((self.ns + 1, self.ns + 1))
        lib().or_jacobian(self._h, float(rho), _ptr(u), _ptr(J))
        return J

    def integrate_cell(self, rho, u, dt, rtol=1e-8, atol=1e-10, max_steps=100000,
                       fixed_steps=0, h0=0.0, trace_cap=0, scheme="lsrk"):
        u = np.array(u, dtype=np.float64)
        h = C.c_double(h0)
        na, nr, tl = C.c_int(), C.c_int(), C.c_int()
        tr = np.zeros(4 * max(trace_cap, 1)) if trace_cap else None
        st = lib().or_integrate_cell_scheme(SCHEMES[scheme], self._h, float(rho), _ptr(u),
                                     float(dt), float(rtol),
                                     float(atol), int(max_steps), int(fixed_steps), C.byref(h),
                                     C.byref(na), C.byref(nr),
                                     _ptr(tr) if tr is not None else None, int(trace_cap),
                                     C.byref(tl))
        out = dict(u=u, status=st, h=h.value, nacc=na.value, nrej=nr.value)
        if tr is not None:
            out["trace"] = tr[: 4 * tl.value].reshape(-1, 4)
        return out

    def integrate(self, state: np.ndarray, dt: float, rtol=1e-8, atol=1e-10,
                  max_steps=100000, fixed_steps=0, nthreads=None, scheme="lsrk"):
        """In-place on an SoA block state[(N+3), n] (rows T, Y.., rho, h).

        Returns (status[n], counts[2, n]) with counts = (n_acc, n_rej)."""
        assert state.dtype == np.float64 and state.flags.c_contiguous
        assert state.shape[0] == self.ns + 3
        n = state.shape[1]
        status = np.zeros(n, dtype=np.int32)
        counts = np.zeros((2, n), dtype=np.int32)
        if nthreads is None:
            nthreads = os.cpu_count() or 1
        lib().or_integrate_scheme(SCHEMES[scheme], self._h, _ptr(state), n, n, float(dt),
                                  float(rtol), float(atol), int(max_steps), int(fixed_steps),
                                  int(nthreads), _ptr(status), _ptr(counts))
        return status, counts


def _mech_energy(self, T, Y):
    """(e [erg/g], c_v [erg/(g K)]) of a mixture."""
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    e, cv = C.c_double(), C.c_double()
    lib().or_energy(self._h, float(T), _ptr(Y), C.byref(e), C.byref(cv))
    return e.value, cv.value


def _mech_calculate_T(self, Y, e, T0=0.0):
    """Newton temperature for internal energy e; returns (T, iterations or -1)."""
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    T = C.c_double()
    it = lib().or_calculate_T(self._h, _ptr(Y), float(e), float(T0), C.byref(T))
    return T.value, it


def _mech_react_conserved(self, cons, dt, rtol=1e-8, atol=1e-10, nthreads=None):
    """In place on conserved SoA rows (rho, rho u, rho v, rho w, rho E,
    rho Y_1..rho Y_N, T, h); returns (status, counts[2, n])."""
    assert cons.dtype == np.float64 and cons.flags.c_contiguous
    assert cons.shape[0] == self.ns + 7
    n = cons.shape[1]
    status = np.zeros(n, dtype=np.int32)
    counts = np.zeros((2, n), dtype=np.int32)
    lib().or_react_conserved(self._h, _ptr(cons), n, n, float(dt), float(rtol), float(atol),
                             int(nthreads or os.cpu_count() or 1), _ptr(status), _ptr(counts))
    return status, counts


Mech.energy = _mech_energy
Mech.calculate_T = _mech_calculate_T
Mech.react_conserved = _mech_react_conserved


def integrate_linear(A, u0, dt, rtol=1e-8, atol=1e-10, max_steps=100000, fixed_steps=0,
                     h0=0.0, trace_cap=0, scheme="lsrk"):
    """u' = A u through the oracle's own step/controller/driver."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    u = np.array(u0, dtype=np.float64)
    h = C.c_double(h0)
    na, nr, tl = C.c_int(), C.c_int(), C.c_int()
    tr = np.zeros(4 * max(trace_cap, 1)) if trace_cap else None
    st = lib().or_integrate_linear_scheme(SCHEMES[scheme], n, _ptr(A), _ptr(u), float(dt),
                                   float(rtol), float(atol),
                                   int(max_steps), int(fixed_steps), C.byref(h), C.byref(na),
                                   C.byref(nr), _ptr(tr) if tr is not None else None,
                                   int(trace_cap), C.byref(tl))
    out = dict(u=u, status=st, h=h.value, nacc=na.value, nrej=nr.value)
    if tr is not None:
        out["trace"] = tr[: 4 * tl.value].reshape(-1, 4)
    return out
