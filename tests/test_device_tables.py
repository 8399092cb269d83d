"""Host-side checks of constants the device code is built with (no GPU):
the per-lane exponential's polynomial, the 2^(j/64) table of the
cooperative kernel's exponential, its reduction constants, the NASA-7 range
switch the code generator emits for the pool order by range, and the
range check of the factorised reverse rates."""
import math
import os
import re
from decimal import Decimal, getcontext

from paper_2506_02602_amd import codegen
from paper_2506_02602_amd import workloads as wl

CSRC = os.path.join(os.path.dirname(codegen.__file__), "csrc")


def _source(name):
    with open(os.path.join(CSRC, name)) as f:
        return f.read()


def test_exp2_table_entries_are_correctly_rounded():
    """Each kExp2Frac entry is the double nearest 2^(j/64) (60-digit decimal
    reference), so the table adds at most half an ulp to exp_tab."""
    src = _source("lsrk.hip.h")
    body = src[src.index("kExp2Frac[64] = {"):]
    body = body[:body.index("};")]
    vals = [float.fromhex(t) for t in re.findall(r"0x[0-9a-f.]+p[+-]\d+", body)]
    assert len(vals) == 64
    getcontext().prec = 60
    for j, v in enumerate(vals):
        exact = Decimal(2) ** (Decimal(j) / 64)
        assert abs(Decimal(v) - exact) <= Decimal(math.ulp(v)) / 2, j


def test_exp_tab_reduction_constants():
    """K = 64 / ln 2, and L_HI + L_LO = ln 2 / 64 to far below an ulp of
    L_HI (the two-part Cody-Waite reduction)."""
    src = _source("lsrk.hip.h")
    fn = src[src.index("double exp_tab("):]
    k = float(re.search(r"constexpr double K = ([0-9.e+-]+);", fn).group(1))
    hi = float(re.search(r"constexpr double L_HI = ([0-9.e+-]+);", fn).group(1))
    lo = float(re.search(r"constexpr double L_LO = ([0-9.e+-]+);", fn).group(1))
    getcontext().prec = 60
    ln2 = Decimal(2).ln()
    assert abs(Decimal(k) - 64 / ln2) <= Decimal(math.ulp(k))
    assert abs(Decimal(hi) + Decimal(lo) - ln2 / 64) < Decimal(math.ulp(hi)) * Decimal("1e-6")


def test_range_switch_is_the_most_shared_tmid():
    """T_SPLIT is the T_mid most species share (the generated RHS branches
    per wave on each distinct T_mid; the pool order by range splits on this
    one); on a tie the first in species order."""
    for name in ("mech9", "mech32", "isomer"):
        m = codegen.parse(wl.mech_file(name))
        tm = [s["Tmid"] for s in m["species"]]
        assert codegen.t_split(m) == max(tm, key=lambda t: (tm.count(t), -tm.index(t)))
    m = codegen.parse(wl.mech_file("mech9"))
    m["species"] = [dict(s, Tmid=(1200.0 if i < 5 else 1000.0)) for i, s in enumerate(m["species"])]
    assert codegen.t_split(m) == 1200.0
    m["species"] = [dict(s, Tmid=(1200.0 if i < 4 else 1000.0)) for i, s in enumerate(m["species"])]
    assert codegen.t_split(m) == 1000.0


def _exp_cw_coefficients():
    src = _source("lsrk.hip.h")
    fn = src[src.index("double exp_cw("):]
    fn = fn[:fn.index("return ldexp")]
    c = [float.fromhex(t) for t in re.findall(r"0x[0-9a-f.]+p[+-]\d+", fn)]
    return c + [1.0, 1.0]        # the last two Horner steps add the literal 1.0


def test_exp_cw_polynomial_error():
    """The degree-11 polynomial of exp_cw (highest coefficient first) against
    e^r in 40-digit arithmetic on [-ln2/2, ln2/2]: relative error below
    1.7e-17 with exact arithmetic, and at most 0.8 ulp when every Horner step
    is an FMA rounded to double (as on the device)."""
    import mpmath as mp
    from fractions import Fraction
    import numpy as np
    mp.mp.dps = 40
    c = _exp_cw_coefficients()
    assert len(c) == 12
    a = float(mp.log(2) / 2)
    rng = np.random.Generator(np.random.PCG64(17))
    rs = np.concatenate([np.linspace(-a, a, 801), rng.uniform(-a, a, 1200)])
    worst_exact = worst_ulp = 0.0
    for r in rs:
        ex = mp.exp(mp.mpf(r))
        p = mp.mpf(0)
        q = c[0]
        for cc in c:
            p = p * mp.mpf(r) + mp.mpf(cc)
        for cc in c[1:]:
            q = float(Fraction(q) * Fraction(r) + Fraction(cc))
        worst_exact = max(worst_exact, float(abs(p / ex - 1)))
        worst_ulp = max(worst_ulp, float(abs(mp.mpf(q) - ex) / mp.mpf(np.spacing(float(ex)))))
    assert worst_exact < 1.7e-17
    assert worst_ulp <= 0.8


def test_factorised_reverse_rates_stay_in_range():
    """Every reverse rate the generator writes as k_f times per-species
    factors multiplies them in an order whose partial products stay within
    e^+-650 for every T on the check grid (200 K to 6000 K and both sides
    of each NASA-7 range switch), re-evaluated here in double from the
    mechanism's own fits; the 9-species mechanism factorises every reaction."""
    for name in ("mech9", "mech32", "isomer"):
        m = codegen.parse(wl.mech_file(name))
        inv = len(m["species"]) <= codegen.FACTOR_INVERSES_MAX_N
        ts = codegen._check_temperatures(m)
        lnP = math.log(m["pstd"] / codegen.R_CGS)
        n_fact = 0
        for rx in m["reactions"]:
            o = codegen._reverse_factors(m, rx, inv)
            if o is None:
                continue
            n_fact += 1
            chains = [o] if inv else [o[0], o[1]]
            for ci, chain in enumerate(chains):
                for T in ts:
                    run = (math.log(rx["A"]) + rx["b"] * math.log(T) - rx["Ea"] / (codegen.R_J * T)
                           if ci == 0 else 0.0)
                    for f in chain:
                        if f == "PRT":
                            run += lnP - math.log(T)
                        elif f == "RTP":
                            run -= lnP - math.log(T)
                        elif f.startswith("Ei"):
                            run -= codegen._g_rt(m["species"][int(f[2:])], T)
                        else:
                            run += codegen._g_rt(m["species"][int(f[1:])], T)
                        assert abs(run) <= 650.0, (name, f, T)
            # the factors are exactly the reaction's net stoichiometry
            nu = codegen._nu(rx)
            got = {}
            for f in (o if inv else o[0]):
                if f.startswith("Ei"):
                    got[int(f[2:])] = got.get(int(f[2:]), 0) - 1
                elif f.startswith("E"):
                    got[int(f[1:])] = got.get(int(f[1:]), 0) + 1
            if not inv:
                for f in o[1]:
                    got[int(f[1:])] = got.get(int(f[1:]), 0) - 1
            assert got == nu
        if name == "mech9":
            assert n_fact == len(m["reactions"])
