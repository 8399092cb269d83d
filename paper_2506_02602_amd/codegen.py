"""Build-time code generator: ``.mech`` text -> fully unrolled FP64 HIP RHS.

For one mechanism it emits a struct with the species count, the content hash
of the file (FNV-1a 64 over its bytes, the key ``chem_mech_load`` binds by) and
a ``__device__`` right-hand side of the chemistry ODE (paper Eq. 20 with the
source of Eq. 14-16) in which every stoichiometric coefficient, Arrhenius
parameter and NASA-7 coefficient is a literal:

* thermo (Eq. 10 fits): per species cp/R, h/RT and g/RT = h/RT - s/R as sums
  over the shared powers T, T^2, T^3, T^4 (each multiply-add takes one
  coefficient from a scalar register; a Horner chain costs two vector moves
  per coefficient for its accumulator), with a wave-coherent branch on
  T < Tmid (one branch per distinct Tmid);
* forward rate k_f = exp(ln A + b ln T - Ea/(R T)); reverse rate
  k_r = k_f / K_c = k_f prod_k exp(g_k/RT)^nu_k (R T/P)^dnu, from one
  exponential per species, E_k = exp(g_k/RT), and its reciprocal, shared by
  every reaction (N exponentials instead of one per reaction); the factors
  of each reaction are multiplied in an order whose partial products stay
  within the double range for every T from 200 K to 6000 K, checked here
  on the NASA-7 fits; a reaction for which no such order is found keeps
  exp(ln k_f + sum_k nu_k g_k/RT - dnu ln(P/(R T))).  The choice is made
  per reaction at build time, so every lane runs the same arithmetic
  whatever its neighbours hold.  Below 200 K (outside the fits' validity)
  a factorised product may overflow: the step then has a non-finite error
  and is rejected (the exponential is the device's own ``exp_cw``, within
  1 ulp);
* progress q_j = [M]_j (k_f prod c^nu' - k_r prod c^nu''), integer powers as
  products; production rates accumulated straight into N registers;
* dY_k/dt = W_k wdot_k / rho and the constant-volume adiabatic dT/dt.

This parser is the GPU side's own; it shares nothing with the CPU oracle.
"""
from __future__ import annotations

import math
import os

R_J = 8.31446261815324
R_CGS = 8.31446261815324e7


def fnv1a64(data: bytes) -> int:
    h = 0xCBF29CE484222325
    for b in data:
        h ^= b
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def parse(path: str) -> dict:
    raw = open(path, "rb").read()
    lines = [ln.strip() for ln in raw.decode().splitlines()]
    lines = [ln for ln in lines if ln and not ln.startswith("#")]
    if not lines or lines[0] != "MECH 1":
        raise ValueError(f"{path}: not a MECH 1 file")
    m = {"hash": fnv1a64(raw), "name": "mech", "pstd": 1.01325e6, "elements": [],
         "species": [], "reactions": []}
    i = 1
    while i < len(lines):
        tok = lines[i].split()
        key = tok[0]
        if key == "name":
            m["name"] = tok[1]
            i += 1
        elif key == "pstd":
            m["pstd"] = float(tok[1])
            i += 1
        elif key == "elements":
            ne = int(tok[1])
            m["elements"] = [lines[i + 1 + e].split()[0] for e in range(ne)]
            m["element_weights"] = [float(lines[i + 1 + e].split()[1]) for e in range(ne)]
            i += 1 + ne
        elif key == "species":
            ns = int(tok[1])
            ne = len(m["elements"])
            for k in range(ns):
                t = lines[i + 1 + k].split()
                vals = [float(x) for x in t[2 + ne:]]
                m["species"].append(dict(name=t[0], W=float(t[1]), Tmid=vals[1],
                                         comp=[int(x) for x in t[2:2 + ne]],
                                         lo=vals[3:10], hi=vals[10:17]))
            i += 1 + ns
        elif key == "reactions":
            nr = int(tok[1])
            names = [s["name"] for s in m["species"]]
            i += 1
            for _ in range(nr):
                t = lines[i].split()
                rx = dict(A=float(t[1]), b=float(t[2]), Ea=float(t[3]), tb=int(t[4]) == 1,
                          reac={}, prod={}, eff=None)
                for side, key2 in ((lines[i + 1], "reac"), (lines[i + 2], "prod")):
                    st = side.split()
                    n = int(st[1])
                    for q in range(n):
                        rx[key2][names.index(st[2 + 2 * q])] = int(st[3 + 2 * q])
                i += 3
                if rx["tb"]:
                    rx["eff"] = [float(x) for x in lines[i].split()[1:]]
                    i += 1
                m["reactions"].append(rx)
        elif key == "end":
            break
        else:
            raise ValueError(f"{path}: unexpected record {key}")
    return m


def lit(x: float) -> str:
    """A C double literal that round-trips exactly."""
    if x == 0.0:
        return "0.0"
    r = repr(float(x))
    if "e" not in r and "." not in r and "inf" not in r and "nan" not in r:
        r += ".0"
    return r


def _horner(coefs, var):
    """coefs[0] + var*(coefs[1] + var*(...)) as a C expression."""
    expr = lit(coefs[-1])
    for c in reversed(coefs[:-1]):
        expr = f"{lit(c)} + {var} * ({expr})"
    return expr


def _powsum(coefs):
    """coefs[0] + coefs[1] T + coefs[2] T^2 + ... from the shared powers
    T, T2, T3, T4, accumulated from the highest power down with the constant
    term last: every multiply-add takes one coefficient (a scalar register)
    and one power, so no coefficient has to be copied into a vector
    register as the running accumulator of a Horner chain would need."""
    pw = ["", "T", "T2", "T3", "T4"]
    terms = [f"{lit(c)} * {pw[i]}" for i, c in reversed(list(enumerate(coefs))) if i > 0]
    return " + ".join(terms + [lit(coefs[0])])


def _thermo_block(species, idx, rng, suffix="", den="den"):
    out = []
    for k in idx:
        a = species[k][rng]
        # h/RT = a1 + a2 T/2 + a3 T^2/3 + a4 T^3/4 + a5 T^4/5 + a6/T
        h = _powsum([a[0], a[1] / 2, a[2] / 3, a[3] / 4, a[4] / 5])
        # g/RT = h/RT - s/R = a1 (1 - ln T) - (a2 T/2 + a3 T^2/6 + a4 T^3/12 + a5 T^4/20) + a6/T - a7
        gp = _powsum([a[1] / 2, a[2] / 6, a[3] / 12, a[4] / 20])
        # c_k (cp_k/R - 1), cp/R = a1 + a2 T + a3 T^2 + a4 T^3 + a5 T^4
        out.append(f"    {den} += c{k} * ({_powsum([a[0] - 1.0] + list(a[1:5]))});")
        decl = "const double " if suffix else ""
        out.append(f"    {decl}h{k}{suffix} = {h} + {lit(a[5])} * invT;")
        out.append(f"    {decl}g{k}{suffix} = {lit(a[0])} * omlnT - T * ({gp}) + {lit(a[5])} * invT - {lit(a[6])};")
    return out


def _thermo(species):
    """Range selection made wave-uniform: waves whose lanes all sit in one
    NASA-7 range evaluate that range with literal coefficients; a wave that
    straddles T_mid evaluates both ranges and selects per lane."""
    groups: dict = {}
    for k, s in enumerate(species):
        groups.setdefault(s["Tmid"], []).append(k)
    L = []
    for gi, (tm, idx) in enumerate(groups.items()):
        L.append(f"    const bool lo{gi} = T < {lit(tm)};")
        L.append(f"    if (__all(lo{gi})) {{")
        L += ["  " + x for x in _thermo_block(species, idx, "lo")]
        L.append(f"    }} else if (!__any(lo{gi})) {{")
        L += ["  " + x for x in _thermo_block(species, idx, "hi")]
        L.append("    } else {")
        L.append("      double dlo = 0.0, dhi = 0.0;")
        for k in idx:
            L.append("      {")
            L += ["    " + x for x in _thermo_block(species, [k], "lo", "_l", "dlo")]
            L += ["    " + x for x in _thermo_block(species, [k], "hi", "_h", "dhi")]
            L.append(f"        h{k} = lo{gi} ? h{k}_l : h{k}_h;")
            L.append(f"        g{k} = lo{gi} ? g{k}_l : g{k}_h;")
            L.append("      }")
        L.append(f"      den += lo{gi} ? dlo : dhi;")
        L.append("    }")
    return L


# Lowest temperature for which the factorised reverse rates are range-checked.
T_FACTOR_MIN = 200.0
# Largest |ln| a partial product of a reverse rate may reach (the double
# range ends near e^709).
LN_PARTIAL_MAX = 650.0


def _g_rt(s: dict, T: float) -> float:
    """g/RT of one species from its NASA-7 fit (the range T < Tmid is low)."""
    a = s["lo"] if T < s["Tmid"] else s["hi"]
    return (a[0] * (1.0 - math.log(T)) - (a[1] * T / 2 + a[2] * T * T / 6 + a[3] * T ** 3 / 12 +
                                          a[4] * T ** 4 / 20) + a[5] / T - a[6])


def _check_temperatures(m: dict) -> list:
    """T grid for the range check: log-spaced over [T_FACTOR_MIN, 6000 K] plus
    both sides of every NASA-7 range switch."""
    ts = list(T_FACTOR_MIN * (6000.0 / T_FACTOR_MIN) ** (i / 400.0) for i in range(401))
    for sp in m["species"]:
        ts += [sp["Tmid"] * (1 - 1e-9), sp["Tmid"] * (1 + 1e-9)]
    return sorted(ts)


def _nu(rx: dict) -> dict:
    nu = {}
    for k, v in rx["reac"].items():
        nu[k] = nu.get(k, 0) - v
    for k, v in rx["prod"].items():
        nu[k] = nu.get(k, 0) + v
    return {k: v for k, v in nu.items() if v != 0}


def _chain(start: list, factors: list, ts: list):
    """Greedy multiplication order of `factors` (C name, per-T ln function)
    onto a running product whose ln is `start` on the grid `ts`: at each step
    the factor that keeps the running ln nearest zero at the grid's coldest
    point (the largest magnitudes).  None if a partial product leaves
    e^+-LN_PARTIAL_MAX anywhere on the grid."""
    order, run, rest = [], list(start), list(factors)
    while rest:
        j = min(range(len(rest)), key=lambda i: abs(run[0] + rest[i][1](ts[0])))
        f = rest.pop(j)
        run = [r + f[1](T) for r, T in zip(run, ts)]
        if max(abs(r) for r in run) > LN_PARTIAL_MAX:
            return None
        order.append(f[0])
    return order


def _reverse_factors(m: dict, rx: dict, inverses: bool):
    """The factors of k_r = k_f prod_k E_k^nu_k (RT/P)^dnu, E_k = exp(g_k/RT),
    in multiplication orders whose partial products stay within
    e^+-LN_PARTIAL_MAX on the check grid; None if none passes.  With
    `inverses` the factors of species with nu_k < 0 are reciprocals Ei_k
    (shared, one per species) and the result is one product chain [names];
    without, those factors form a second chain and k_r = first * rcp(second):
    (names, names)."""
    sp = m["species"]
    lnP = math.log(m["pstd"] / R_CGS)
    ts = _check_temperatures(m)
    lkf = [math.log(rx["A"]) + rx["b"] * math.log(T) - rx["Ea"] / (R_J * T) for T in ts]
    num, den = [], []
    for k, v in sorted(_nu(rx).items()):
        if v > 0:
            num += [(f"E{k}", (lambda T, k=k: _g_rt(sp[k], T)))] * v
        elif inverses:
            num += [(f"Ei{k}", (lambda T, k=k: -_g_rt(sp[k], T)))] * (-v)
        else:
            den += [(f"E{k}", (lambda T, k=k: _g_rt(sp[k], T)))] * (-v)
    dnu = sum(_nu(rx).values())
    if dnu:
        # (RT/P)^dnu: RTP = RT/P for dnu > 0, PRT = P/RT for dnu < 0
        name, sign = ("RTP", -1.0) if dnu > 0 else ("PRT", 1.0)
        num += [(name, (lambda T, sg=sign: sg * (lnP - math.log(T))))] * abs(dnu)
    a = _chain(lkf, num, ts)
    if inverses:
        return a
    b = _chain([0.0] * len(ts), den, ts) if den else []
    return None if a is None or b is None else (a, b)


# Mechanisms with more species than this keep only E_k live through the
# reaction section and divide once per reaction (register pressure); smaller
# ones also keep the reciprocals Ei_k and only multiply.
FACTOR_INVERSES_MAX_N = 16


def _prod_expr(coef: str, side: dict) -> str:
    terms = [coef]
    for k, nu in sorted(side.items()):
        terms += [f"c{k}"] * nu
    return " * ".join(terms)


def _rate_lines(m: dict, orders: list) -> list:
    """Rates of progress and their accumulation into w_k; reaction j's k_r
    from its factor order (see _reverse_factors), or through its own
    exponential when orders[j] is None."""
    L = []
    for j, rx in enumerate(m["reactions"]):
        L.append(f"    {{  // reaction {j}")
        e = [lit(math.log(rx["A"]))]
        if rx["b"] != 0.0:
            e.append(f"{lit(rx['b'])} * lnT")
        if rx["Ea"] != 0.0:
            e.append(f"- {lit(rx['Ea'] / R_J)} * invT")
        L.append(f"      const double lkf = {' + '.join(e).replace('+ -', '-')};")
        L.append("      const double kf = exp_cw(lkf);")
        nu = _nu(rx)
        dnu = sum(nu.values())
        if isinstance(orders[j], tuple):
            num, den = orders[j]
            d = f" * rcp_nr({' * '.join(den)})" if den else ""
            L.append(f"      const double kr = {' * '.join(['kf'] + num)}{d};")
        elif orders[j] is not None:
            L.append(f"      const double kr = {' * '.join(['kf'] + orders[j])};")
        else:
            gterms = []
            for k, v in sorted(nu.items()):
                sign = "+" if v > 0 else "-"
                mag = abs(v)
                gterms.append(f" {sign} {'' if mag == 1 else lit(float(mag)) + ' * '}g{k}")
            if dnu != 0:
                sign = "-" if dnu > 0 else "+"
                mag = abs(dnu)
                gterms.append(f" {sign} {'' if mag == 1 else lit(float(mag)) + ' * '}lnPRT")
            L.append(f"      const double kr = exp_cw(lkf{''.join(gterms)});")
        q = f"{_prod_expr('kf', rx['reac'])} - {_prod_expr('kr', rx['prod'])}"
        if rx["tb"]:
            mt = " + ".join(f"{lit(a)} * c{k}" for k, a in enumerate(rx["eff"]))
            L.append(f"      const double q = ({mt}) * ({q});")
        else:
            L.append(f"      const double q = {q};")
        for k, v in sorted(nu.items()):
            if v == 1:
                L.append(f"      w{k} += q;")
            elif v == -1:
                L.append(f"      w{k} -= q;")
            else:
                L.append(f"      w{k} += {lit(float(v))} * q;")
        L.append("    }")
    return L


def gen_rhs(m: dict) -> str:
    sp = m["species"]
    N = len(sp)
    L = []
    L.append("  __device__ __forceinline__ static void rhs(const double* __restrict__ u, double rho,")
    L.append("                                             double inv_rho, double* __restrict__ f) {")
    L.append("    // Hide rho's loop invariance from the optimiser: otherwise every")
    L.append("    // rho-dependent product (rho/W_k, third-body alpha_k rho/W_k, ...) is")
    L.append("    // hoisted out of the step loop and pinned in registers.")
    L.append("    asm volatile(\"\" : \"+v\"(rho), \"+v\"(inv_rho));")
    L.append("    const double T = u[0];")
    L.append("    const double lnT = log_atanh(T);")
    L.append("    const double invT = rcp_nr(T);")
    L.append("    const double omlnT = 1.0 - lnT;")
    L.append("    const double T2 = T * T, T3 = T2 * T, T4 = T2 * T2;")
    L.append(f"    const double lnPRT = {lit(math.log(m['pstd'] / R_CGS))} - lnT;")
    for k, s in enumerate(sp):
        L.append(f"    const double c{k} = u[{k + 1}] * (rho * {lit(1.0 / s['W'])});")
    L.append("    double " + ", ".join(f"h{k}, g{k}" for k in range(N)) + ";")
    L.append("    double den = 0.0;  // sum_k c_k (cp_k/R - 1)")
    L += _thermo(sp)
    L.append("    double " + ", ".join(f"w{k} = 0.0" for k in range(N)) + ";")
    inv = N <= FACTOR_INVERSES_MAX_N
    orders = [_reverse_factors(m, rx, inv) for rx in m["reactions"]]
    need = sorted({f for o in orders if o for f in (o if inv else o[0] + o[1])})
    for k in range(N):
        if f"E{k}" in need or f"Ei{k}" in need:
            L.append(f"    const double E{k} = exp_cw(g{k});")
        if f"Ei{k}" in need:
            L.append(f"    const double Ei{k} = rcp_nr(E{k});")
    C = m["pstd"] / R_CGS
    if "PRT" in need:
        L.append(f"    const double PRT = {lit(C)} * invT;")
    if "RTP" in need:
        L.append(f"    const double RTP = {lit(1.0 / C)} * T;")
    L += _rate_lines(m, orders)
    num = " + ".join(f"(h{k} - 1.0) * w{k}" for k in range(N))
    L.append(f"    const double num = {num};")
    L.append("    f[0] = -T * num * rcp_nr(den);")
    for k, s in enumerate(sp):
        L.append(f"    f[{k + 1}] = w{k} * ({lit(s['W'])} * inv_rho);")
    L.append("  }")
    return "\n".join(L)


ROS4_MAX_N1 = 16   # the Rosenbrock comparator holds the (N+1)^2 Jacobian in registers


def gen_jac(m: dict) -> str:
    """f(u) and the exact Jacobian J[i*(N+1) + k] = df_i/du_k of the same ODE,
    for the implicit (Rosenbrock) comparator: derivatives of every term of
    ``gen_rhs`` written out (chain rule through the Arrhenius and equilibrium
    exponentials, the NASA-7 polynomials, the mass-action products, the
    third-body sums and the quotient of the temperature equation).  Only
    nonzero species couplings get a register; the rest of J is zero.
    Mechanisms with N + 1 > ROS4_MAX_N1 get no Jacobian (the comparator is not
    built for them)."""
    sp, rxs = m["species"], m["reactions"]
    N = len(sp)
    N1 = N + 1
    if N1 > ROS4_MAX_N1:
        return "  static constexpr bool HAS_JAC = false;"
    L = ["  static constexpr bool HAS_JAC = true;",
         "  __device__ __forceinline__ static void jac(const double* __restrict__ u, double rho,",
         "                                             double inv_rho, double* __restrict__ f,",
         "                                             double* __restrict__ J) {",
         "    asm volatile(\"\" : \"+v\"(rho), \"+v\"(inv_rho));",
         "    const double T = u[0];",
         "    const double lnT = log(T);",
         "    const double invT = 1.0 / T;",
         "    const double omlnT = 1.0 - lnT;",
         f"    const double lnPRT = {lit(math.log(m['pstd'] / R_CGS))} - lnT;"]
    for k, s_ in enumerate(sp):
        L.append(f"    const double c{k} = u[{k + 1}] * (rho * {lit(1.0 / s_['W'])});")
    # thermo and its T-derivatives, per lane range selection
    for k, s_ in enumerate(sp):
        L.append(f"    double h{k}, g{k}, cm{k}, dcp{k};")
        for rng, head in (("lo", f"    if (T < {lit(s_['Tmid'])}) {{"), ("hi", "    } else {")):
            a = s_[rng]
            L.append(head)
            L.append(f"      h{k} = {_horner([a[0], a[1] / 2, a[2] / 3, a[3] / 4, a[4] / 5], 'T')} + {lit(a[5])} * invT;")
            L.append(f"      g{k} = {lit(a[0])} * omlnT - T * ({_horner([a[1] / 2, a[2] / 6, a[3] / 12, a[4] / 20], 'T')}) + {lit(a[5])} * invT - {lit(a[6])};")
            L.append(f"      cm{k} = {_horner([a[0] - 1.0] + list(a[1:5]), 'T')};")
            L.append(f"      dcp{k} = {_horner([a[1], 2 * a[2], 3 * a[3], 4 * a[4]], 'T')};")
        L.append("    }")
        # d(h/RT)/dT = (cp/R - h/RT)/T, d(g/RT)/dT = -(h/RT)/T
        L.append(f"    const double dh{k} = (cm{k} + 1.0 - h{k}) * invT;")
        L.append(f"    const double dg{k} = -h{k} * invT;")
    L.append("    const double den = " + " + ".join(f"c{k} * cm{k}" for k in range(N)) + ";")
    L.append("    const double dden_dT = " + " + ".join(f"c{k} * dcp{k}" for k in range(N)) + ";")
    # production rates and their derivatives (concentration space, and T)
    pairs = set()
    for rx in rxs:
        nu = {}
        for k, v in rx["reac"].items():
            nu[k] = nu.get(k, 0) - v
        for k, v in rx["prod"].items():
            nu[k] = nu.get(k, 0) + v
        dep = set(rx["reac"]) | set(rx["prod"])
        if rx["tb"]:
            dep |= {k for k in range(N) if rx["eff"][k] != 0.0}
        for k, v in nu.items():
            if v != 0:
                for l in dep:
                    pairs.add((k, l))
    pairs = sorted(pairs)
    L.append("    double " + ", ".join(f"w{k} = 0.0, wT{k} = 0.0" for k in range(N)) + ";")
    if pairs:
        L.append("    double " + ", ".join(f"wc{k}_{l} = 0.0" for k, l in pairs) + ";")

    def mono(side, coef, skip=None):
        """coef * prod c^nu, or its derivative in c_skip (nu c^(nu-1) ...)."""
        terms = [coef]
        for k, v in sorted(side.items()):
            p = v - 1 if k == skip else v
            if k == skip:
                terms.insert(0, lit(float(v)) if v != 1 else "1.0")
            terms += [f"c{k}"] * p
        return " * ".join(terms)

    for j, rx in enumerate(rxs):
        L.append(f"    {{  // reaction {j}")
        e = [lit(math.log(rx["A"]))]
        if rx["b"] != 0.0:
            e.append(f"{lit(rx['b'])} * lnT")
        if rx["Ea"] != 0.0:
            e.append(f"- {lit(rx['Ea'] / R_J)} * invT")
        L.append(f"      const double lkf = {' + '.join(e).replace('+ -', '-')};")
        L.append(f"      const double dlkf = ({lit(rx['b'])} + {lit(rx['Ea'] / R_J)} * invT) * invT;")
        L.append("      const double kf = exp_cw(lkf);")
        nu = {}
        for k, v in rx["reac"].items():
            nu[k] = nu.get(k, 0) - v
        for k, v in rx["prod"].items():
            nu[k] = nu.get(k, 0) + v
        dnu = sum(nu.values())
        gsum = "".join(f" + {lit(float(v))} * g{k}" for k, v in sorted(nu.items()) if v != 0)
        dgsum = "".join(f" + {lit(float(v))} * dg{k}" for k, v in sorted(nu.items()) if v != 0)
        L.append(f"      const double kr = exp_cw(lkf{gsum} - {lit(float(dnu))} * lnPRT);")
        L.append(f"      const double dlkr = dlkf{dgsum} + {lit(float(dnu))} * invT;")
        L.append(f"      const double fw = {mono(rx['reac'], 'kf')};")
        L.append(f"      const double rv = {mono(rx['prod'], 'kr')};")
        dep = sorted(set(rx["reac"]) | set(rx["prod"]) |
                     ({k for k in range(N) if rx["eff"][k] != 0.0} if rx["tb"] else set()))
        if rx["tb"]:
            mt = " + ".join(f"{lit(a)} * c{k}" for k, a in enumerate(rx["eff"]) if a != 0.0)
            L.append(f"      const double mt = {mt};")
            L.append("      const double q = mt * (fw - rv);")
            L.append("      const double qT = mt * (fw * dlkf - rv * dlkr);")
        else:
            L.append("      const double q = fw - rv;")
            L.append("      const double qT = fw * dlkf - rv * dlkr;")
        for l in dep:
            parts = []
            if l in rx["reac"]:
                parts.append(mono(rx["reac"], "kf", skip=l))
            if l in rx["prod"]:
                parts.append("-" + mono(rx["prod"], "kr", skip=l))
            d = " + ".join(parts).replace("+ -", "- ") if parts else "0.0"
            if rx["tb"]:
                expr = f"mt * ({d})" if parts else "0.0"
                if rx["eff"][l] != 0.0:
                    expr = f"{expr} + {lit(rx['eff'][l])} * (fw - rv)" if parts else \
                        f"{lit(rx['eff'][l])} * (fw - rv)"
            else:
                expr = d
            L.append(f"      const double qc{l} = {expr};")
        for k, v in sorted(nu.items()):
            if v == 0:
                continue
            cv = lit(float(v))
            L.append(f"      w{k} += {cv} * q;")
            L.append(f"      wT{k} += {cv} * qT;")
            for l in dep:
                L.append(f"      wc{k}_{l} += {cv} * qc{l};")
        L.append("    }")
    L.append("    const double num = " + " + ".join(f"(h{k} - 1.0) * w{k}" for k in range(N)) + ";")
    L.append("    const double inv_den = 1.0 / den;")
    L.append("    const double r = num * inv_den;")
    L.append("    f[0] = -T * r;")
    for k, s_ in enumerate(sp):
        L.append(f"    f[{k + 1}] = w{k} * ({lit(s_['W'])} * inv_rho);")
    # species rows
    nz = {(k, l) for k, l in pairs}
    for k, s_ in enumerate(sp):
        L.append(f"    J[{(k + 1) * N1}] = wT{k} * ({lit(s_['W'])} * inv_rho);")
        for l, s2 in enumerate(sp):
            idx = (k + 1) * N1 + l + 1
            if (k, l) in nz:
                L.append(f"    J[{idx}] = {lit(s_['W'] / s2['W'])} * wc{k}_{l};")
            else:
                L.append(f"    J[{idx}] = 0.0;")
    # temperature row: f0 = -T num / den
    dnT = " + ".join(f"(h{k} - 1.0) * wT{k} + dh{k} * w{k}" for k in range(N))
    L.append(f"    const double dnum_dT = {dnT};")
    L.append("    J[0] = -r - T * (dnum_dT - r * dden_dT) * inv_den;")
    for l, s2 in enumerate(sp):
        terms = [f"(h{k} - 1.0) * wc{k}_{l}" for k in range(N) if (k, l) in nz]
        dnl = " + ".join(terms) if terms else "0.0"
        L.append(f"    J[{l + 1}] = -T * (({dnl}) * (rho * {lit(1.0 / s2['W'])}) - r * "
                 f"(rho * {lit(1.0 / s2['W'])}) * cm{l}) * inv_den;")
    L.append("  }")
    return "\n".join(L)


def gen_aux(m: dict) -> str:
    """Constants and thermo helpers used by the surrogate's features and trust
    test: molecular weights, element mass coefficients a_ek m_e / W_k, and the
    mixture internal energy e = R T sum_k Y_k (h_k/RT - 1)/W_k [erg/g] with
    c_v = R sum_k Y_k (cp_k/R - 1)/W_k [erg/(g K)] from the same NASA-7 fits."""
    sp = m["species"]
    N = len(sp)
    E = len(m["elements"])
    L = []
    L.append(f"  static constexpr int NE = {E};")
    L.append("  static constexpr double W[NS] = {" + ", ".join(lit(s["W"]) for s in sp) + "};")
    coefs = []
    for e, el in enumerate(m["elements"]):
        aw = m["element_weights"][e]
        coefs.append("{" + ", ".join(lit(s["comp"][e] * aw / s["W"]) for s in sp) + "}")
    L.append("  static constexpr double ELEM[NE][NS] = {" + ", ".join(coefs) + "};")
    # e/(R T) = sum_k Y_k/W_k (h_k/RT - 1), c_v/R = sum_k Y_k/W_k (cp_k/R - 1)
    # from the shared powers of T (one coefficient per multiply-add, as in
    # the RHS's thermo), with the NASA-7 range chosen per wave like there
    L.append("  __device__ __forceinline__ static void energy_cv(double T, const double* Y, "
             "double& e, double& cv) {")
    L.append("    const double invT = rcp_nr(T);")
    L.append("    const double T2 = T * T, T3 = T2 * T, T4 = T3 * T;")
    L.append("    double se = 0.0, sc = 0.0;")

    def block(idx, rng, se="se", sc="sc"):
        out = []
        for k in idx:
            a = sp[k][rng]
            hm1 = _powsum([a[0] - 1.0, a[1] / 2, a[2] / 3, a[3] / 4, a[4] / 5])
            cpm1 = _powsum([a[0] - 1.0] + list(a[1:5]))
            out.append(f"      {{ const double yw = Y[{k}] * {lit(1.0 / sp[k]['W'])};")
            out.append(f"        {se} += yw * ({hm1} + {lit(a[5])} * invT);")
            out.append(f"        {sc} += yw * ({cpm1}); }}")
        return out
    groups: dict = {}
    for k, s in enumerate(sp):
        groups.setdefault(s["Tmid"], []).append(k)
    for gi, (tm, idx) in enumerate(groups.items()):
        L.append(f"    const bool lo{gi} = T < {lit(tm)};")
        L.append(f"    if (__all(lo{gi})) {{")
        L += block(idx, "lo")
        L.append(f"    }} else if (!__any(lo{gi})) {{")
        L += block(idx, "hi")
        L.append("    } else {")
        L.append("      double sel = 0.0, scl = 0.0, seh = 0.0, sch = 0.0;")
        L += block(idx, "lo", "sel", "scl")
        L += block(idx, "hi", "seh", "sch")
        L.append(f"      se += lo{gi} ? sel : seh;")
        L.append(f"      sc += lo{gi} ? scl : sch;")
        L.append("    }")
    L.append(f"    e = {lit(R_CGS)} * T * se;")
    L.append(f"    cv = {lit(R_CGS)} * sc;")
    L.append("  }")
    return "\n".join(L)


COOP_TH = 18   # thermo table entries per (range, species), padded to 16-byte rows


def coop_group(m: dict) -> int:
    """Lanes that advance one cell together in the cooperative kernel: one
    lane per species and per reaction, at most a wave (64; larger mechanisms
    give a lane several reactions).  Groups need not divide the wave: a
    wave holds floor(64 / G) groups, so the 21 reactions of the 9-species
    mechanism put three cells in a wave (one lane spare) instead of two
    with G rounded up to 32 -- the step's instruction stream is per lane,
    so a wave's cost per step hardly depends on G."""
    return min(64, max(len(m["species"]), len(m["reactions"])))


def gen_coop(m: dict, tag: str) -> tuple[str, str]:
    """Tables of the cooperative (reaction-parallel) RHS.

    The same rate law as ``gen_rhs`` written as data: per reaction ln A, b,
    Ea/R, the reactant and product species lists (a species of stoichiometric
    coefficient nu appears nu times; pad = N, whose concentration slot holds
    1), the net-stoichiometry terms of the K_c exponent (pad = N, g slot 0),
    its third-body row; per species the reactions it appears in with their
    net coefficients, and the NASA-7 Horner coefficients of both ranges.
    Returns (namespace-scope __constant__ arrays, struct member block)."""
    sp, rxs = m["species"], m["reactions"]
    N, J = len(sp), len(rxs)
    nets = []
    for r in rxs:
        nu = {}
        for k, v in r["reac"].items():
            nu[k] = nu.get(k, 0) - v
        for k, v in r["prod"].items():
            nu[k] = nu.get(k, 0) + v
        nets.append([(k, v) for k, v in sorted(nu.items()) if v != 0])
    MR = max(1, max(max(sum(r["reac"].values()), sum(r["prod"].values())) for r in rxs))
    MG = max(1, max(len(n) for n in nets))
    occ = [[] for _ in range(N)]
    for j, n in enumerate(nets):
        for k, v in n:
            occ[k].append((j, v))
    L = max(1, max(len(o) for o in occ))
    tb_rows = [r["eff"] for r in rxs if r["tb"]]
    NTB = len(tb_rows)

    D, I = [], []     # flat double and int tables
    off = {}

    def put_d(name, vals):
        off[name] = len(D)
        D.extend(float(x) for x in vals)

    def put_i(name, vals):
        off[name] = len(I)
        I.extend(int(x) for x in vals)

    put_d("LNA", [math.log(r["A"]) for r in rxs])
    put_d("BEXP", [r["b"] for r in rxs])
    put_d("EAR", [r["Ea"] / R_J for r in rxs])
    put_d("DNU", [sum(v for _, v in n) for n in nets])
    gnu = []
    for n in nets:
        gnu += [float(v) for _, v in n] + [0.0] * (MG - len(n))
    put_d("GNU", gnu)
    tbe = []
    for row in tb_rows:
        tbe += row
    put_d("TBEFF", tbe if tbe else [0.0] * N)    # row 0 is read (and discarded) by non-third-body lanes
    slnu = []
    for o in occ:
        slnu += [float(v) for _, v in o] + [0.0] * (L - len(o))
    put_d("SLNU", slnu)
    put_d("INVW", [1.0 / s["W"] for s in sp])
    put_d("WK", [s["W"] for s in sp])
    put_d("TMID", [s["Tmid"] for s in sp])
    while len(D) % 2:
        D.append(0.0)
    th = []
    for rng in ("lo", "hi"):
        for s in sp:
            a = s[rng]
            row = [a[0], a[1] / 2, a[2] / 3, a[3] / 4, a[4] / 5, a[5],
                   a[0], a[1] / 2, a[2] / 6, a[3] / 12, a[4] / 20, a[6],
                   a[0] - 1.0, a[1], a[2], a[3], a[4], 0.0]
            assert len(row) == COOP_TH
            th += row
    put_d("TH", th)
    ri, pi_, gk, tbi = [], [], [], []
    tb_row = 0
    for r, n in zip(rxs, nets):
        rs = [k for k, v in sorted(r["reac"].items()) for _ in range(v)]
        ps = [k for k, v in sorted(r["prod"].items()) for _ in range(v)]
        ri += rs + [N] * (MR - len(rs))
        pi_ += ps + [N] * (MR - len(ps))
        gk += [k for k, _ in n] + [N] * (MG - len(n))
        if r["tb"]:
            tbi.append(tb_row)
            tb_row += 1
        else:
            tbi.append(-1)
    put_i("RI", ri)
    put_i("PI", pi_)
    put_i("GK", gk)
    put_i("TB", tbi)
    put_i("SLJ", [j for o in occ for j in [jj for jj, _ in o] + [0] * (L - len(o))])
    while len(I) % 4:
        I.append(0)

    ns = f"coop_{tag}"
    glob = [f"namespace {ns} {{",
            f"static __constant__ double D[{len(D)}] = {{" + ", ".join(lit(x) for x in D) + "};",
            f"static __constant__ int I[{len(I)}] = {{" + ", ".join(str(x) for x in I) + "};",
            "}"]
    mem = ["  struct Coop {",
           f"    static constexpr int G = {coop_group(m)};",
           f"    static constexpr int J = {J}, MR = {MR}, MG = {MG}, L = {L}, NTB = {NTB};",
           f"    static constexpr int ND = {len(D)}, NI = {len(I)}, TH_ROW = {COOP_TH};",
           f"    static constexpr double LNPRT0 = {lit(math.log(m['pstd'] / R_CGS))};"]
    mem.append("    static constexpr int " + ", ".join(f"O_{k} = {v}" for k, v in off.items()) + ";")
    mem.append(f"    __device__ static const double* dtab() {{ return {ns}::D; }}")
    mem.append(f"    __device__ static const int* itab() {{ return {ns}::I; }}")
    mem.append("  };")
    return "\n".join(glob), "\n".join(mem)


def op_counts(m: dict) -> dict:
    """Algorithmic FP64 operation counts of one RHS evaluation: the method's
    arithmetic as the paper states it, with k_f and k_r = k_f / K_c each
    through an exponential per reaction (the generated code evaluates K_c
    from N shared per-species exponentials instead, which changes the
    instruction count, not this figure).

    Counted per expression (FMA-able pairs count as 2 flops):
    thermo 13 FMA + 4 mul/add per species (one range), concentrations 2 mul,
    per reaction: lkf (up to 2 FMA), kr exponent (1 add per nu term), products,
    third-body sum (1 FMA per species), accumulation (1 add per nu term),
    assembly 2 FMA per species + 2 mul per species.  Transcendentals counted
    separately."""
    sp, rx = m["species"], m["reactions"]
    N = len(sp)
    flops = 0
    flops += N * (2 * 13 + 4)            # cp (4 FMA), h (4 FMA + 1 FMA), g (3 FMA + 1 mul + 2 FMA + 2 add)
    flops += N * 2                       # c_k
    exps = 0
    for r in rx:
        flops += 2 * (1 if r["b"] != 0 else 0) + 2 * (1 if r["Ea"] != 0 else 0)
        nu = {}
        for k, v in r["reac"].items():
            nu[k] = nu.get(k, 0) - v
        for k, v in r["prod"].items():
            nu[k] = nu.get(k, 0) + v
        nz = sum(1 for v in nu.values() if v != 0)
        flops += nz + (1 if sum(nu.values()) != 0 else 0)      # kr exponent
        flops += sum(r["reac"].values()) + sum(r["prod"].values()) + 1  # products and difference
        if r["tb"]:
            flops += 2 * N + 1
        flops += nz                                             # accumulation
        exps += 2
    flops += 2 * N * 2 + 2 + N                                  # num, den, dT, dY
    return dict(flops=flops, exp=exps, log=1, div=2, n_species=N, n_reactions=len(rx))


# Algorithmic FP64 cost assigned to each non-polynomial operation, in flops
# (FMA = 2): exp = range reduction (1 mul, 2 FMA) + degree-11 polynomial
# (11 FMA) = 27 (the conventional cost; the device exponential spends a
# little more); log similar = 30; a correctly rounded divide or square root
# = reciprocal seed + 2 Newton refinements + correction = 10.  The step
# factor err^(-1/4) is two square roots and a divide.
FLOP_EXP, FLOP_LOG, FLOP_DIV, FLOP_SQRT = 27, 30, 10, 10


def rhs_flops(m: dict) -> int:
    c = op_counts(m)
    return c["flops"] + FLOP_EXP * c["exp"] + FLOP_LOG * c["log"] + FLOP_DIV * c["div"]


def jac_flops(m: dict) -> int:
    """Operation count of the generated Jacobian (``gen_jac``): every binary
    arithmetic operator and accumulation in its source (FMA-able pairs
    counted as 2), plus its exponentials, logarithm and the two divisions."""
    src = gen_jac(m)
    if "jac(" not in src:
        return 0
    body = src.split("double* __restrict__ J) {", 1)[1]
    ops = body.count(" * ") + body.count(" + ") + body.count(" - ") + body.count(" += ")
    c = op_counts(m)
    return ops + FLOP_EXP * c["exp"] + FLOP_LOG + 2 * FLOP_DIV


def step_flops(m: dict, scheme: str = "lsrk") -> int:
    """Flops of one LSRK step: 5 RHS + stage updates + WRMS norm + control.

    For the full-storage Fehlberg 4(5) scheme: 6 RHS; stage inputs
    u + h sum_j a_ij K_j (1, 2, 3, 4, 5 FMA per component for stages 2-6),
    X and E accumulated with one FMA each per stage, one multiply per
    coefficient by h; the factor err^(-1/5) through pow.

    Stage updates: E, U, X each one FMA per component for stages 1-4, E and X
    for stage 5: 14 FMA = 28 flops per component.  WRMS: weight (FMA), divide,
    square-accumulate (FMA) per component, then a scale, a sqrt and the
    factor err^(-1/4) (two square roots and a divide), plus 4 scalar flops
    of control."""
    n1 = len(m["species"]) + 1
    wrms = n1 * (2 + FLOP_DIV + 2) + 1 + FLOP_SQRT
    if scheme == "ros4":
        # Jacobian (which also returns f(u_n)), two more RHS, LU with
        # partial pivoting (2/3 n^3 + one division per column), four solves
        # (2 n^2 each, one division per row), stage combinations and the
        # diagonal shift (~33 n), WRMS and the factor as for the LSRK step
        lu = (2 * n1 ** 3) // 3 + n1 * FLOP_DIV
        solves = 4 * (2 * n1 * n1 + n1 * FLOP_DIV)
        return (jac_flops(m) + 2 * rhs_flops(m) + lu + solves + 33 * n1 + wrms
                + 2 * FLOP_SQRT + FLOP_DIV + 4)
    if scheme == "rkf45":
        upd = 2 * (1 + 2 + 3 + 4 + 5) * n1 + 2 * 2 * 6 * n1 + 6 * 7
        return 6 * rhs_flops(m) + upd + wrms + FLOP_LOG + FLOP_EXP + 4
    upd = 28 * n1
    return 5 * rhs_flops(m) + upd + wrms + 2 * FLOP_SQRT + FLOP_DIV + 4


def t_split(m: dict) -> float:
    """The T_mid shared by the most species (the first such on a tie)."""
    count: dict = {}
    for sp in m["species"]:
        count[sp["Tmid"]] = count.get(sp["Tmid"], 0) + 1
    return max(count, key=lambda t: count[t])


def gen_header(path: str) -> tuple[str, dict]:
    m = parse(path)
    N = len(m["species"])
    tag = f"{m['name']}_{m['hash']:016x}"
    coop_glob, coop_mem = gen_coop(m, tag)
    rhs = gen_rhs(m)
    body = [
        f"// Generated from {os.path.basename(path)} -- do not edit.",
        coop_glob,
        f"struct Mech_{tag} {{",
        f"  static constexpr int NS = {N};",
        f"  static constexpr int NR = {len(m['reactions'])};",
        f"  static constexpr unsigned long long HASH = 0x{m['hash']:016x}ULL;",
        f"  static constexpr const char* NAME = \"{m['name']}\";",
        "  // the NASA-7 range switch shared by the most species: the RHS branches",
        "  // on it per wave, so the pool order that groups cells by range uses it",
        f"  static constexpr double T_SPLIT = {lit(t_split(m))};",
        rhs,
        gen_jac(m),
        gen_aux(m),
        coop_mem,
        "};",
    ]
    return "\n".join(body) + "\n", dict(tag=tag, hash=m["hash"], ns=N, nr=len(m["reactions"]),
                                        name=m["name"], ops=op_counts(m))


def generate(mech_files, out_dir: str) -> list:
    os.makedirs(out_dir, exist_ok=True)
    infos = []
    for p in mech_files:
        text, info = gen_header(p)
        with open(os.path.join(out_dir, f"mech_{info['tag']}.inc"), "w") as f:
            f.write(text)
        infos.append(info)
    reg = ["// Generated list of built-in mechanisms -- do not edit."]
    for info in infos:
        reg.append(f"#include \"mech_{info['tag']}.inc\"")
    reg.append("#define CHEM_FOR_EACH_MECH(X) \\")
    reg.append(" \\\n".join(f"  X(Mech_{info['tag']})" for info in infos))
    with open(os.path.join(out_dir, "registry.inc"), "w") as f:
        f.write("\n".join(reg) + "\n")
    return infos
