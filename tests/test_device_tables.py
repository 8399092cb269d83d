"""Host-side checks of constants the device code is built with (no GPU):
the 2^(j/64) table of the cooperative kernel's exponential, its reduction
constants, and the NASA-7 range switch the code generator emits for the
pool order by range."""
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
