"""Seeded synthetic reaction-mechanism generator (input data, not part of the method).

The paper's chemistry runs use a 13-species hydrogen mechanism that is not
available here, so every workload runs on seeded synthetic mechanisms with the
same structure as the paper's reaction model (Sec. 2.1.2, Eq. 15-16):

* reversible elementary reactions, forward rate in Arrhenius form, reverse rate
  from the equilibrium constant;
* NASA 7-coefficient thermodynamic fits per species (Eq. 10);
* optional third-body enhancement [M] = sum_k alpha_k c_k.

Two mechanisms are produced: ``mech9`` (9 H/O/N species, 21 reactions, 5 of them
third-body, N2 a pure collider) and ``mech32`` (those 9 plus 23 synthetic
C/H/O/N species, 150 reactions).  A two-species isomer mechanism A <-> B with
identical thermodynamics is written for closed-form tests.

Parameter draws (cgs units, activation energy in J/mol): A log-uniform in
[1e8, 1e17], b uniform in [-1.5, 2], Ea uniform in [0, 2.5e5], third-body
efficiencies uniform in [0.5, 12].  Each reaction is written in its exothermic
direction at 298.15 K before its rate is drawn, and a draw whose forward or
reverse pseudo-first-order rate exceeds ``lambda_cap`` anywhere on
300-3000 K at the 30 atm total concentration is redrawn from the same stream.
That filter is an acceptance rule on the input, not part of the integrator;
it keeps the problem inside what an explicit method can step through.

Seed choice for ``mech9``: with these ranges most draws give a mixture that
stays frozen for tens of milliseconds, so no flow step of 1e-7 s does any
chemistry worth integrating.  The seed used, 3312, is the first seed from 2506
upward whose mechanism ignites a stoichiometric H2-air cell at 1300 K, 1 atm
within 1 ms (temperature above 1400 K at 1 ms).  That scan was run once,
offline, with a general-purpose stiff ODE solver; only its result is recorded
here.  ``mech32`` uses seed 2602 as drawn.

The output is a line-oriented text file (the ``.mech`` format documented in
``write_mech``); every number is printed with ``repr`` so that any conforming
decimal-to-double parser recovers the same doubles.
"""
from __future__ import annotations

import itertools
import math
import os
from dataclasses import dataclass, field

import numpy as np

R_J = 8.31446261815324          # J/(mol K), exact SI-2019 value
R_CGS = 8.31446261815324e7      # erg/(mol K)
P_ATM = 1.01325e6               # dyn/cm^2

ATOMIC_WEIGHTS = {"H": 1.008, "O": 15.999, "N": 14.007, "C": 12.011}

SPECIES9 = ["H2", "O2", "H2O", "H", "O", "OH", "HO2", "H2O2", "N2"]
EXTRA23 = ["CH4", "CH3", "CH2", "CH", "CO", "CO2", "HCO", "CH2O", "CH3O",
           "CH3OH", "C2H2", "C2H3", "C2H4", "C2H5", "C2H6", "HCCO", "NO",
           "NO2", "N2O", "HNO", "NH3", "NH2", "HCN"]

# The 21 reaction topologies of the 9-species set: 16 two-sided reactions and
# 5 third-body reactions (entries are (reactants, products, third_body)).
REACTIONS9 = [
    (["H", "O2"], ["O", "OH"], False),
    (["O", "H2"], ["H", "OH"], False),
    (["H2", "OH"], ["H2O", "H"], False),
    (["O", "H2O"], ["OH", "OH"], False),
    (["HO2", "H"], ["H2", "O2"], False),
    (["HO2", "H"], ["OH", "OH"], False),
    (["HO2", "H"], ["O", "H2O"], False),
    (["HO2", "O"], ["O2", "OH"], False),
    (["HO2", "OH"], ["H2O", "O2"], False),
    (["HO2", "HO2"], ["H2O2", "O2"], False),
    (["H2O2", "H"], ["H2O", "OH"], False),
    (["H2O2", "H"], ["HO2", "H2"], False),
    (["H2O2", "O"], ["OH", "HO2"], False),
    (["H2O2", "OH"], ["HO2", "H2O"], False),
    (["H2O2"], ["OH", "OH"], False),
    (["H2O2", "O"], ["H2O", "O2"], False),
    (["H2"], ["H", "H"], True),
    (["O", "O"], ["O2"], True),
    (["O", "H"], ["OH"], True),
    (["H", "OH"], ["H2O"], True),
    (["H", "O2"], ["HO2"], True),
]


def parse_formula(f: str) -> dict:
    """'CH3OH' -> {'C': 1, 'H': 4, 'O': 1}."""
    out: dict = {}
    i = 0
    while i < len(f):
        el = f[i]
        i += 1
        j = i
        while j < len(f) and f[j].isdigit():
            j += 1
        n = int(f[i:j]) if j > i else 1
        out[el] = out.get(el, 0) + n
        i = j
    return out


@dataclass
class Species:
    name: str
    comp: dict
    W: float
    lo: list          # a1..a7 for T < Tmid
    hi: list          # a1..a7 for T >= Tmid
    Tlow: float = 300.0
    Tmid: float = 1000.0
    Thigh: float = 5000.0
    hf: float = 0.0   # J/mol at 298.15 K (record only)
    s0: float = 0.0   # J/(mol K) at 298.15 K (record only)


@dataclass
class Reaction:
    reac: dict        # species name -> stoichiometric coefficient
    prod: dict
    tb: bool
    A: float = 0.0
    b: float = 0.0
    Ea: float = 0.0
    eff: list = field(default_factory=list)


# --------------------------------------------------------------------- thermo
def _natoms(comp):
    return sum(comp.values())


def _cp_class(n):
    """(cp/R at 300 K, cp/R limit at 5000 K) by total atom count."""
    table = {1: (2.5, 2.5), 2: (3.5, 4.5), 3: (4.0, 6.5), 4: (5.0, 9.5),
             5: (5.5, 12.5), 6: (6.0, 15.5)}
    if n in table:
        return table[n]
    return (6.5, 3.0 * n - 2.5)


def _hf_class(name, comp, rng):
    """Formation enthalpy [J/mol] drawn in a physical sign/magnitude class."""
    if name in ("H2", "O2", "N2"):
        return 0.0
    fixed = {"H2O": (-260e3, -220e3), "H2O2": (-150e3, -120e3),
             "H": (200e3, 240e3), "O": (230e3, 270e3),
             "OH": (20e3, 50e3), "HO2": (0.0, 25e3)}
    if name in fixed:
        lo, hi = fixed[name]
        return float(rng.uniform(lo, hi))
    # synthetic extra species: H-count parity decides "stable" vs "radical"
    valence = {"H": 1, "O": 2, "N": 3, "C": 4}
    unpaired = sum(valence[e] * n for e, n in comp.items()) % 2
    if unpaired or _natoms(comp) <= 2 and name not in ("CO", "NO"):
        return float(rng.uniform(30e3, 350e3))
    return float(rng.uniform(-400e3, 60e3))


def _s0_class(comp, rng):
    n = _natoms(comp)
    rngs = {1: (110.0, 165.0), 2: (125.0, 215.0), 3: (180.0, 240.0),
            4: (200.0, 260.0)}
    lo, hi = rngs.get(n, (220.0 + 8.0 * (n - 5), 300.0 + 8.0 * (n - 5)))
    return float(rng.uniform(lo, hi))


def _fit_range(Tlo, Thi, cpfun):
    """Least-squares quartic cp/R(T) on [Tlo, Thi]; returns a1..a5."""
    T = np.linspace(Tlo, Thi, 241)
    x = T / 1000.0
    V = np.vander(x, 5, increasing=True)
    c, *_ = np.linalg.lstsq(V, cpfun(T), rcond=None)
    return [float(c[k] / 1000.0 ** k) for k in range(5)]


def _H_R_poly(a, T):      # H/R without a6
    return a[0] * T + a[1] * T**2 / 2 + a[2] * T**3 / 3 + a[3] * T**4 / 4 + a[4] * T**5 / 5


def _S_R_poly(a, T):      # S/R without a7
    return a[0] * math.log(T) + a[1] * T + a[2] * T**2 / 2 + a[3] * T**3 / 3 + a[4] * T**4 / 4


def make_species(name, rng, Tmid=1000.0):
    comp = parse_formula(name)
    W = sum(ATOMIC_WEIGHTS[e] * n for e, n in comp.items())
    c0, c1 = _cp_class(_natoms(comp))
    scale = 1.0 + rng.uniform(-0.03, 0.03)
    c0 *= scale
    c1 *= scale * (1.0 + rng.uniform(-0.03, 0.03)) if c1 != c0 else scale
    theta = rng.uniform(800.0, 1500.0)

    def cpfun(T):
        return c0 + (c1 - c0) * (1.0 - np.exp(-(np.asarray(T) - 300.0) / theta))

    lo5 = _fit_range(300.0, Tmid, cpfun)
    hi5 = _fit_range(Tmid, 5000.0, cpfun)
    hf = _hf_class(name, comp, rng)
    s0 = _s0_class(comp, rng)
    T0 = 298.15
    a6lo = hf / R_J - _H_R_poly(lo5, T0)
    a7lo = s0 / R_J - _S_R_poly(lo5, T0)
    a6hi = _H_R_poly(lo5, Tmid) + a6lo - _H_R_poly(hi5, Tmid)
    a7hi = _S_R_poly(lo5, Tmid) + a7lo - _S_R_poly(hi5, Tmid)
    return Species(name, comp, W, lo5 + [a6lo, a7lo], hi5 + [a6hi, a7hi],
                   Tmid=Tmid, hf=hf, s0=s0)


def _g_RT(sp: Species, T):
    a = sp.lo if T < sp.Tmid else sp.hi
    h = (_H_R_poly(a, T) + a[5]) / T
    s = _S_R_poly(a, T) + a[6]
    return h - s


def _H_R(sp: Species, T):
    a = sp.lo if T < sp.Tmid else sp.hi
    return _H_R_poly(a, T) + a[5]


# ------------------------------------------------------------------ reactions
def _orient_exothermic(rx: Reaction, spmap):
    dH = sum(n * _H_R(spmap[s], 298.15) for s, n in rx.prod.items()) - \
        sum(n * _H_R(spmap[s], 298.15) for s, n in rx.reac.items())
    if dH > 0:
        rx.reac, rx.prod = rx.prod, rx.reac


def _max_pseudo_rate(rx: Reaction, spmap, A, b, Ea, eff_max):
    """Largest forward/reverse pseudo-first-order rate on 300..3000 K at 30 atm."""
    worst = 0.0
    m_f = sum(rx.reac.values())
    m_r = sum(rx.prod.values())
    nu_f = max(rx.reac.values())
    nu_r = max(rx.prod.values())
    for T in np.linspace(300.0, 3000.0, 55):
        T = float(T)
        ctot = 30.0 * P_ATM / (R_CGS * T)
        kf = A * T**b * math.exp(-Ea / (R_J * T))
        dg = sum(n * _g_RT(spmap[s], T) for s, n in rx.prod.items()) - \
            sum(n * _g_RT(spmap[s], T) for s, n in rx.reac.items())
        dnu = m_r - m_f
        lnKc = -dg + dnu * math.log(P_ATM / (R_CGS * T))
        kr = kf * math.exp(-lnKc) if lnKc > -700 else math.inf
        mfac = eff_max * ctot if rx.tb else 1.0
        lf = nu_f * kf * ctot ** (m_f - 1) * mfac
        lr = nu_r * kr * ctot ** (m_r - 1) * mfac
        worst = max(worst, lf, lr)
    return worst


def draw_rates(rxns, spmap, species_order, rng, lambda_cap, orient=True):
    redraws = 0
    for rx in rxns:
        if orient:
            _orient_exothermic(rx, spmap)
        if rx.tb:
            rx.eff = [float(v) for v in rng.uniform(0.5, 12.0, size=len(species_order))]
        emax = max(rx.eff) if rx.tb else 1.0
        for attempt in range(200000):
            A = float(10.0 ** rng.uniform(8.0, 17.0))
            b = float(rng.uniform(-1.5, 2.0))
            Ea = float(rng.uniform(0.0, 2.5e5))
            if _max_pseudo_rate(rx, spmap, A, b, Ea, emax) <= lambda_cap:
                rx.A, rx.b, rx.Ea = A, b, Ea
                break
            redraws += 1
        else:
            raise RuntimeError("rate draw did not meet the stiffness cap")
    return redraws


# ---------------------------------------------------------------- mechanisms
def _element_list(names):
    els = []
    for n in names:
        for e in parse_formula(n):
            if e not in els:
                els.append(e)
    order = ["H", "O", "N", "C"]
    return [e for e in order if e in els]


def build_mech9(seed=3312, lambda_cap=1e10, orient=True):
    rng = np.random.Generator(np.random.PCG64(seed))
    sp = [make_species(n, rng) for n in SPECIES9]
    spmap = {s.name: s for s in sp}
    rxns = []
    for r, p, tb in REACTIONS9:
        rd, pd = {}, {}
        for s in r:
            rd[s] = rd.get(s, 0) + 1
        for s in p:
            pd[s] = pd.get(s, 0) + 1
        rxns.append(Reaction(rd, pd, tb))
    redraws = draw_rates(rxns, spmap, SPECIES9, rng, lambda_cap, orient)
    return dict(name="mech9", seed=seed, lambda_cap=lambda_cap, redraws=redraws,
                elements=_element_list(SPECIES9), species=sp, reactions=rxns)


def _comp_key(names):
    tot: dict = {}
    for n in names:
        for e, c in parse_formula(n).items():
            tot[e] = tot.get(e, 0) + c
    return tuple(sorted(tot.items()))


def _stoich_rank(rxns, names):
    idx = {n: i for i, n in enumerate(names)}
    M = np.zeros((len(rxns), len(names)))
    for j, rx in enumerate(rxns):
        for s, n in rx.reac.items():
            M[j, idx[s]] -= n
        for s, n in rx.prod.items():
            M[j, idx[s]] += n
    return np.linalg.matrix_rank(M)


def build_mech32(seed=2602, lambda_cap=1e10, n_reactions=150, n_tb=36):
    rng = np.random.Generator(np.random.PCG64(seed))
    names = SPECIES9 + EXTRA23
    sp = [make_species(n, rng) for n in names]
    spmap = {s.name: s for s in sp}
    # enumerate element-balanced topologies
    pairs = list(itertools.combinations_with_replacement(names, 2))
    by_comp2: dict = {}
    for pr in pairs:
        by_comp2.setdefault(_comp_key(pr), []).append(pr)
    by_comp1 = {}
    for n in names:
        by_comp1.setdefault(_comp_key([n]), []).append((n,))
    two_two = []
    for key, lst in by_comp2.items():
        for a, b in itertools.combinations(lst, 2):
            two_two.append((a, b))
    two_one = []
    for key, lst in by_comp2.items():
        for single in by_comp1.get(key, []):
            for pr in lst:
                two_one.append((pr, single))
    base = [(tuple(r), tuple(p), tb) for r, p, tb in REACTIONS9]
    n_base_tb = sum(1 for b in base if b[2])

    def canon(r, p):
        return tuple(sorted([tuple(sorted(r)), tuple(sorted(p))]))
    seen = {canon(r, p) for r, p, _ in base}
    idx_tt = rng.permutation(len(two_two))
    idx_to = rng.permutation(len(two_one))
    chosen = list(base)
    want_tb = n_tb - n_base_tb
    want_tt = n_reactions - len(base) - want_tb
    for i in idx_to:
        if want_tb == 0:
            break
        pr, single = two_one[int(i)]
        c = canon(pr, single)
        if c in seen:
            continue
        seen.add(c)
        chosen.append((pr, single, True))
        want_tb -= 1
    # prefer two-two reactions that touch species not yet covered
    for i in idx_tt:
        if want_tt == 0:
            break
        a, b = two_two[int(i)]
        c = canon(a, b)
        if c in seen:
            continue
        covered = {s for r, p, _ in chosen for s in r + p}
        new = [s for s in a + b if s not in covered]
        if not new and want_tt <= len(set(names) - covered) * 2:
            continue
        seen.add(c)
        chosen.append((a, b, False))
        want_tt -= 1
    rxns = []
    for r, p, tb in chosen:
        rd, pd = {}, {}
        for s in r:
            rd[s] = rd.get(s, 0) + 1
        for s in p:
            pd[s] = pd.get(s, 0) + 1
        rxns.append(Reaction(rd, pd, tb))
    covered = {s for rx in rxns for s in list(rx.reac) + list(rx.prod)}
    missing = set(names) - covered - {"N2"}
    if missing:
        raise RuntimeError(f"species not covered: {missing}")
    n_el = len(_element_list(names))
    rank = _stoich_rank(rxns, names)
    if rank != len(names) - n_el:
        raise RuntimeError(f"stoichiometric rank {rank} != {len(names) - n_el}")
    redraws = draw_rates(rxns, spmap, names, rng, lambda_cap)
    return dict(name="mech32", seed=seed, lambda_cap=lambda_cap, redraws=redraws,
                elements=_element_list(names), species=sp, reactions=rxns)


def build_isomer(k=2.0e7):
    """A <-> B with identical thermo and weight: Kc = 1 and kr = kf = k."""
    base = np.random.Generator(np.random.PCG64(7))
    s = make_species("H2O", base)
    a = Species("A", {"H": 2, "O": 1}, s.W, list(s.lo), list(s.hi), hf=s.hf, s0=s.s0)
    b = Species("B", {"H": 2, "O": 1}, s.W, list(s.lo), list(s.hi), hf=s.hf, s0=s.s0)
    rx = Reaction({"A": 1}, {"B": 1}, False, A=float(k), b=0.0, Ea=0.0)
    return dict(name="isomer", seed=7, lambda_cap=0.0, redraws=0,
                elements=["H", "O"], species=[a, b], reactions=[rx])


# ------------------------------------------------------------------- writer
def write_mech(m: dict, path: str) -> None:
    """Write the line-oriented ``.mech`` text format.

    Grammar (one record per line, '#' starts a comment line)::

        MECH 1
        name <word>
        pstd <float>                       standard-state pressure, dyn/cm^2
        elements <E>
        <symbol> <atomic weight g/mol>     (E lines)
        species <N>
        <name> <W> <n_el_1..n_el_E> <Tlow> <Tmid> <Thigh> <a1..a7 low> <a1..a7 high>
        reactions <J>
        reaction <A> <b> <Ea J/mol> <third_body 0|1>
        reactants <n> <species> <nu> ...
        products <n> <species> <nu> ...
        efficiencies <alpha_1..alpha_N>    (only when third_body is 1)
        end
    """
    r = repr
    lines = ["MECH 1",
             f"# seeded synthetic mechanism; seed {m['seed']}, lambda_cap {m['lambda_cap']!r}, "
             f"rate redraws {m['redraws']}",
             f"name {m['name']}", f"pstd {r(P_ATM)}",
             f"elements {len(m['elements'])}"]
    for e in m["elements"]:
        lines.append(f"{e} {r(ATOMIC_WEIGHTS[e])}")
    lines.append(f"species {len(m['species'])}")
    for s in m["species"]:
        cnt = " ".join(str(s.comp.get(e, 0)) for e in m["elements"])
        lines.append(" ".join([s.name, r(s.W), cnt, r(s.Tlow), r(s.Tmid), r(s.Thigh)]
                              + [r(float(v)) for v in s.lo] + [r(float(v)) for v in s.hi]))
    lines.append(f"reactions {len(m['reactions'])}")
    for rx in m["reactions"]:
        lines.append(f"reaction {r(rx.A)} {r(rx.b)} {r(rx.Ea)} {1 if rx.tb else 0}")
        lines.append("reactants " + str(len(rx.reac)) + "".join(
            f" {s} {n}" for s, n in rx.reac.items()))
        lines.append("products " + str(len(rx.prod)) + "".join(
            f" {s} {n}" for s, n in rx.prod.items()))
        if rx.tb:
            lines.append("efficiencies " + " ".join(r(v) for v in rx.eff))
    lines.append("end")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


MECH_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mech")


def mech_path(name: str) -> str:
    return os.path.join(MECH_DIR, name + ".mech")


def generate_all(out_dir: str = MECH_DIR) -> None:
    os.makedirs(out_dir, exist_ok=True)
    write_mech(build_mech9(), os.path.join(out_dir, "mech9.mech"))
    write_mech(build_mech32(), os.path.join(out_dir, "mech32.mech"))
    write_mech(build_isomer(), os.path.join(out_dir, "isomer.mech"))


if __name__ == "__main__":
    generate_all()
