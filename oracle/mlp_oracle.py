"""CPU oracle for the learned surrogate -- TEST INFRASTRUCTURE ONLY.

Plain numpy in FP64.  The paper proposes machine-learned acceleration of the
chemistry only as future work (Sec. 7) and gives no design, so this follows
the design the build states for it (12 -> 128 -> 128 -> 128 -> 10 MLP with
SiLU hidden layers, BF16 GEMM operands with wider accumulation, FP32 master
weights trained by Adam on an MSE loss over standardised increments, and a
per-cell trust test).  No passage of the paper fixes this arithmetic, so its
pins are mathematical ones: finite differences of the loss for the backward
pass, torch's bfloat16 conversion for the rounding points, and closed forms
of Adam's first step.

Parameter vector layout (FP32 master weights, flat):
    W1 [H, I], b1 [H], W2 [H, H], b2 [H], W3 [H, H], b3 [H], W4 [O, H], b4 [O]
with I = N + 3 inputs (T, ln p, ln dt, Y_1..Y_N), O = N + 1 outputs
(dT, dY_1..dY_N), H = 128.

BF16 points (round-to-nearest-even to 8 significant bits): the network input,
every weight matrix, and every hidden activation before it enters a GEMM; in
the backward pass the output gradient, every pre-activation gradient dZ and
the weights/activations it multiplies.  Bias adds, SiLU, its derivative,
reductions and Adam are exact (FP64 here).
"""
from __future__ import annotations

import numpy as np

R_CGS = 8.31446261815324e7


def bf16(x):
    """Round to the nearest bfloat16 value (ties to even), returned as float64."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                # x = m 2^e, 0.5 <= |m| < 1
    r = np.round(m * 256.0)           # 8 significant bits; np.round is half-to-even
    return np.ldexp(r / 256.0, e)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def param_shapes(n_in, n_out, hidden=128):
    return [("W1", (hidden, n_in)), ("b1", (hidden,)), ("W2", (hidden, hidden)), ("b2", (hidden,)),
            ("W3", (hidden, hidden)), ("b3", (hidden,)), ("W4", (n_out, hidden)), ("b4", (n_out,))]


def unpack(theta, n_in, n_out, hidden=128):
    out, o = {}, 0
    for name, shp in param_shapes(n_in, n_out, hidden):
        k = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def pack(p, n_in, n_out, hidden=128):
    return np.concatenate([p[name].reshape(-1) for name, _ in param_shapes(n_in, n_out, hidden)])


def forward(theta, X, n_in, n_out, hidden=128, emulate_bf16=True):
    """X: standardised inputs [B, n_in].  Returns (out [B, n_out], cache)."""
    q = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    p = unpack(theta, n_in, n_out, hidden)
    h = q(X)
    cache = {"x0": h, "Z": [], "H": [h]}
    for l in (1, 2, 3):
        z = h @ q(p[f"W{l}"]).T + p[f"b{l}"]
        h = q(silu(z))
        cache["Z"].append(z)
        cache["H"].append(h)
    out = h @ q(p["W4"]).T + p["b4"]
    return out, cache


def mse(out, Y):
    return float(np.mean((out - Y) ** 2))


def backward(theta, X, Y, n_in, n_out, hidden=128, emulate_bf16=True):
    """Gradient of mean((out - Y)^2) over all B * n_out entries."""
    q = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    p = unpack(theta, n_in, n_out, hidden)
    out, c = forward(theta, X, n_in, n_out, hidden, emulate_bf16)
    B = X.shape[0]
    g = {}
    d = q(2.0 * (out - Y) / (B * n_out))               # dL/dout
    g["W4"] = d.T @ c["H"][3]
    g["b4"] = d.sum(axis=0)
    dh = d @ q(p["W4"])
    for l in (3, 2, 1):
        dz = q(dh * silu_grad(c["Z"][l - 1]))
        g[f"W{l}"] = dz.T @ c["H"][l - 1]
        g[f"b{l}"] = dz.sum(axis=0)
        if l > 1:
            dh = dz @ q(p[f"W{l}"])
    return pack(g, n_in, n_out, hidden), mse(out, Y)


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1).  Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def cosine_lr(lr0, step, total):
    return lr0 * 0.5 * (1.0 + np.cos(np.pi * step / total))


def he_uniform_init(n_in, n_out, hidden, rng):
    """W ~ U[-sqrt(6/fan_in), +sqrt(6/fan_in)], biases zero."""
    p = {}
    for name, shp in param_shapes(n_in, n_out, hidden):
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shp[1])
            p[name] = rng.uniform(-lim, lim, size=shp)
        else:
            p[name] = np.zeros(shp)
    return pack(p, n_in, n_out, hidden)


# ------------------------------------------------------- features and trust
def features(state, dt, W):
    """Raw inputs (T, ln p, ln dt, Y_1..Y_N) of every cell of an SoA block
    state[(N+3), n]; p = rho R T sum_k Y_k / W_k (ideal gas)."""
    N = len(W)
    T = state[0]
    Y = state[1:N + 1]
    rho = state[N + 1]
    p = rho * R_CGS * T * (Y / W[:, None]).sum(axis=0)
    n = state.shape[1]
    return np.vstack([T, np.log(p), np.full(n, np.log(dt)), Y]).T


def energy_cv(omech, T, Y):
    """Mixture internal energy [erg/g] and c_v [erg/(g K)] from the oracle's
    NASA-7 thermo: e = sum_k Y_k R T (h_k/RT - 1)/W_k, c_v = sum_k Y_k R (cp_k/R - 1)/W_k."""
    cp, h, _ = omech.thermo(T)
    e = float(np.sum(Y * R_CGS * T * (h - 1.0) / omech.W))
    cv = float(np.sum(Y * R_CGS * (cp - 1.0) / omech.W))
    return e, cv


# trust-test failure bits
TRUST_HULL, TRUST_ELEM, TRUST_POS, TRUST_ENERGY, TRUST_NONFINITE = 1, 2, 4, 8, 16


def trusted_update(state, inc):
    """New (T, Y) rows of trusted cells: T + dT and Y + dY with what lies
    below zero written as zero (the positivity criterion already bounds it
    by pos_tol).  state: [(N+3), n]; inc: [n, N+1] de-standardised increments."""
    N = inc.shape[1] - 1
    out = np.array(state[:N + 1], dtype=np.float64)
    out[0] += inc[:, 0]
    out[1:] = np.maximum(out[1:] + inc[:, 1:].T, 0.0)
    return out


def trust_codes(omech, state, dt, z_in, out_std, norm, trust):
    """Per-cell bitmask of failed criteria (0 = trusted), all in FP64.

    z_in: standardised inputs [n, I]; out_std: network outputs [n, O]
    (standardised); norm: dict with mu_out, sd_out, zmin, zmax;
    trust = (hull_margin, elem_tol, pos_tol, energy_tol).
      hull:   every z_in within [zmin - margin, zmax + margin]
      elem:   |sum_k a_ek m_e / W_k (Y'_k - Y_k)| <= elem_tol for each element e
              (change of the element's mass fraction; m_e its atomic weight)
      pos:    min_k Y'_k >= -pos_tol
      energy: |e(T', Y') - e(T, Y)| / c_v(T, Y) <= energy_tol  [K]
    with Y' = Y + dY, T' = T + dT and (dT, dY) = out_std * sd_out + mu_out."""
    hull_margin, elem_tol, pos_tol, energy_tol = trust
    N = omech.ns
    n = state.shape[1]
    codes = np.zeros(n, dtype=np.int32)
    inc = out_std.astype(np.float64) * norm["sd_out"] + norm["mu_out"]
    A = omech.comp.astype(np.float64)                  # [N, E] atoms per molecule
    for i in range(n):
        c = 0
        z = z_in[i]
        if np.any(z < norm["zmin"] - hull_margin) or np.any(z > norm["zmax"] + hull_margin):
            c |= TRUST_HULL
        T, Y = state[0, i], state[1:N + 1, i]
        T1, Y1 = T + inc[i, 0], Y + inc[i, 1:]
        if not (np.all(np.isfinite(inc[i]))):
            c |= TRUST_NONFINITE
        else:
            dmol = (Y1 - Y) / omech.W                  # mol/g change per species
            if np.any(np.abs(omech.ew * (A.T @ dmol)) > elem_tol):
                c |= TRUST_ELEM
            if np.min(Y1) < -pos_tol:
                c |= TRUST_POS
            e0, cv = energy_cv(omech, T, Y)
            e1, _ = energy_cv(omech, T1, Y1)
            if not (abs(e1 - e0) / cv <= energy_tol):
                c |= TRUST_ENERGY
        codes[i] = c
    return codes
