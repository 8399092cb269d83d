// Cooperative integration: G lanes of one wave advance one cell together.
//
// Used for the tail of a flow step -- the few stiff cells still stepping
// after the rest have finished -- where one cell per lane leaves the chip
// nearly idle and the step latency of a single lane bounds the whole call.
// Splitting one cell's right-hand side over G lanes cuts that latency.
//
// Lane roles within a group (gl = lane index in the group, 0..G-1):
//   every lane      holds T and its stage registers (replicated: every lane
//                   computes the same dT/dt from the same sums);
//   species lane    k = gl < N: holds Y_k and its stage registers, evaluates
//                   species k's concentration and NASA-7 thermo (paper
//                   Eq. 10) and sums its production rate;
//   reaction lane   j = gl + r G < J: reaction j's forward and reverse rates
//                   and rate of progress (paper Eq. 15-16).
// Lanes without a species or reaction evaluate a clamped duplicate and
// discard it, so the rate law runs without divergent branches and the
// forward-rate exponentials overlap the thermo.  The rate law is the one of
// the unrolled per-lane RHS, read from the mechanism's generated tables.
// Values pass between lanes through the group's LDS area; every sum over
// species is taken by every lane in the same order, so all lanes of a group
// hold the same bits and the step-control decisions (paper Eq. 22) are
// uniform within the group.
#pragma once

#include <hip/hip_runtime.h>

#include "lsrk.hip.h"

namespace chemgpu {

__device__ __forceinline__ void coop_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS scratch of one group (doubles): concentrations c[N+1] (c[N] = 1, the
// pad of the species lists), g/RT g[N+1] (g[N] = 0), c_k (cp_k/R - 1) d[N],
// rates of progress q[J], per-species terms w[N] of the energy and error
// sums, and one discard slot per lane of the group: a lane without a
// species or reaction stores there instead of branching around the store.
template <class M>
struct CoopScratch {
  static constexpr int N = M::NS;
  static constexpr int SC = 0, SG = N + 1, SD = 2 * (N + 1), SQ = SD + N, SW = SQ + M::Coop::J;
  static constexpr int SX = (SW + N + 1) & ~1;  // one slot per lane for discarded stores
  static constexpr int SIZE = (SX + M::Coop::G + 1) & ~1;
};

// Groups of G lanes never straddle a wave: a wave holds floor(64 / G) of
// them and its remaining lanes (64 mod G) stay idle.
template <int G>
struct CoopWave {
  static_assert(G >= 1 && G <= 64, "a group fits in one wave");
  static constexpr int GPW = 64 / G;  // groups per wave
};

template <class M>
struct CoopCtx {
  const double* D;  // the mechanism's double table, in LDS
  const double* E;  // 2^(j/64), j = 0..63 (kExp2Frac), in LDS
  const int* I;     // its int table, in LDS
  double* s;        // this group's scratch
  int gl;
};

// A lane's own table entries (its reaction, its species' production list,
// its reaction's third-body row), read once into registers when they fit
// (one reaction per lane and short lists); otherwise read from LDS at each
// evaluation.
template <class M, int G>
struct CoopLane {
  using C = typename M::Coop;
  static constexpr int R = (C::J + G - 1) / G;
  static constexpr bool PRE = R == 1 && C::L <= 16 && M::NS <= 16;
  double lna, bexp, ear, dnu;
  double gnu[PRE ? C::MG : 1];
  int gk[PRE ? C::MG : 1], ri[PRE ? C::MR : 1], pi[PRE ? C::MR : 1];
  int tb;
  double eff[PRE ? M::NS : 1];
  double slnu[PRE ? C::L : 1];
  int slj[PRE ? C::L : 1];

  __device__ __forceinline__ void load(const double* D, const int* I, int gl) {
    if constexpr (PRE) {
      constexpr int N = M::NS;
      const int j = min(gl, C::J - 1);
      const int k = min(gl, N - 1);
      lna = D[C::O_LNA + j];
      bexp = D[C::O_BEXP + j];
      ear = D[C::O_EAR + j];
      dnu = D[C::O_DNU + j];
#pragma unroll
      for (int q = 0; q < C::MG; ++q) {
        gnu[q] = D[C::O_GNU + j * C::MG + q];
        gk[q] = I[C::O_GK + j * C::MG + q];
      }
#pragma unroll
      for (int q = 0; q < C::MR; ++q) {
        ri[q] = I[C::O_RI + j * C::MR + q];
        pi[q] = I[C::O_PI + j * C::MR + q];
      }
      tb = I[C::O_TB + j];
      const int row = tb >= 0 ? tb : 0;
#pragma unroll
      for (int kk = 0; kk < N; ++kk) eff[kk] = D[C::O_TBEFF + row * N + kk];
#pragma unroll
      for (int l = 0; l < C::L; ++l) {
        slnu[l] = D[C::O_SLNU + k * C::L + l];
        slj[l] = I[C::O_SLJ + k * C::L + l];
      }
    }
  }
};

// f(T, Y): returns this lane's dY_k/dt (0 for lanes past N) and, on every
// lane, dT/dt in fT.
template <class M, int G>
__device__ __forceinline__ double coop_rhs(double Yk, double T, double rho, double inv_rho,
                                           const CoopCtx<M>& x, const CoopLane<M, G>& ln,
                                           double& fT) {
  using C = typename M::Coop;
  using S = CoopScratch<M>;
  using L = CoopLane<M, G>;
  constexpr int N = M::NS;
  constexpr int R = L::R;
  constexpr bool PRE = L::PRE;
  static_assert(N <= G, "one lane per species");
  double* const s = x.s;
  const double* D = x.D;
  const int* I = x.I;
  const int gl = x.gl;
  const bool sl = gl < N;
  const int k = sl ? gl : N - 1;
  const double lnT = log_atanh(T);
  const double invT = rcp_nr(T);
  const double omlnT = 1.0 - lnT;
  const double lnPRT = C::LNPRT0 - lnT;
  // forward rates: depend on T only
  double lkf[R], kf[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = min(gl + r * G, C::J - 1);
    if constexpr (PRE)
      lkf[r] = ln.lna + ln.bexp * lnT - ln.ear * invT;
    else
      lkf[r] = D[C::O_LNA + j] + D[C::O_BEXP + j] * lnT - D[C::O_EAR + j] * invT;
    kf[r] = exp_tab(lkf[r], x.E);
  }
  // species k: concentration and thermo
  const double c = Yk * (rho * D[C::O_INVW + k]);
  const double* th = D + C::O_TH + (T < D[C::O_TMID + k] ? 0 : N * C::TH_ROW) + k * C::TH_ROW;
  const double hm1 = th[0] + T * (th[1] + T * (th[2] + T * (th[3] + T * th[4]))) + th[5] * invT - 1.0;
  const double gp = th[7] + T * (th[8] + T * (th[9] + T * th[10]));
  const double gk = th[6] * omlnT - T * gp + th[5] * invT - th[11];
  const double dk = c * (th[12] + T * (th[13] + T * (th[14] + T * (th[15] + T * th[16]))));
  {
    // lanes past N store into their own discard slot: no branch
    const int o = sl ? k : S::SX - S::SC + gl;
    s[S::SC + o] = c;
    s[(sl ? S::SG + k : S::SX + gl)] = gk;
    s[(sl ? S::SD + k : S::SX + gl)] = dk;
  }
  coop_sync();
  // reactions: reverse rates, rates of progress
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j0 = gl + r * G;
    const int j = min(j0, C::J - 1);
    double dg = 0.0;
#pragma unroll
    for (int q = 0; q < C::MG; ++q) {
      if constexpr (PRE)
        dg += ln.gnu[q] * s[S::SG + ln.gk[q]];
      else
        dg += D[C::O_GNU + j * C::MG + q] * s[S::SG + I[C::O_GK + j * C::MG + q]];
    }
    const double dn = PRE ? ln.dnu : D[C::O_DNU + j];
    const double kr = exp_tab(lkf[r] + dg - dn * lnPRT, x.E);
    double fw = kf[r], rv = kr;
#pragma unroll
    for (int q = 0; q < C::MR; ++q) {
      if constexpr (PRE) {
        fw *= s[S::SC + ln.ri[q]];
        rv *= s[S::SC + ln.pi[q]];
      } else {
        fw *= s[S::SC + I[C::O_RI + j * C::MR + q]];
        rv *= s[S::SC + I[C::O_PI + j * C::MR + q]];
      }
    }
    const double qraw = fw - rv;
    const int tb = PRE ? ln.tb : I[C::O_TB + j];
    const int row = tb >= 0 ? tb : 0;
    double mt = 0.0;
#pragma unroll
    for (int kk = 0; kk < N; ++kk) {
      if constexpr (PRE)
        mt += ln.eff[kk] * s[S::SC + kk];
      else
        mt += D[C::O_TBEFF + row * N + kk] * s[S::SC + kk];
    }
    const double qj = tb >= 0 ? mt * qraw : qraw;
    s[j0 < C::J ? S::SQ + j : S::SX + gl] = qj;
  }
  // sum_k c_k (cp_k/R - 1), the same order on every lane (two interleaved
  // partial sums: half the dependent chain)
  double den0 = 0.0, den1 = 0.0;
#pragma unroll
  for (int kk = 0; kk < N; ++kk) {
    if (kk & 1) den1 += s[S::SD + kk];
    else den0 += s[S::SD + kk];
  }
  const double den = den0 + den1;
  coop_sync();
  // species k: production rate (two partial sums)
  double wk0 = 0.0, wk1 = 0.0;
#pragma unroll
  for (int l = 0; l < C::L; ++l) {
    double& acc = (l & 1) ? wk1 : wk0;
    if constexpr (PRE)
      acc = fma(ln.slnu[l], s[S::SQ + ln.slj[l]], acc);
    else
      acc = fma(D[C::O_SLNU + k * C::L + l], s[S::SQ + I[C::O_SLJ + k * C::L + l]], acc);
  }
  const double wk = wk0 + wk1;
  s[sl ? S::SW + k : S::SX + gl] = hm1 * wk;
  coop_sync();
  double num0 = 0.0, num1 = 0.0;
#pragma unroll
  for (int kk = 0; kk < N; ++kk) {
    if (kk & 1) num1 += s[S::SW + kk];
    else num0 += s[S::SW + kk];
  }
  const double num = num0 + num1;
  fT = -T * num * rcp_nr(den);
  return sl ? wk * (D[C::O_WK + k] * inv_rho) : 0.0;
}

// One step of size h (paper Eq. 21).  (uT, uk): the state at the start of
// the step (T on every lane, Y_k on species lanes); (XT, Xk) receive the new
// state.  Returns the group's WRMS error (the same on every lane).
template <class M, int G>
__device__ __forceinline__ double coop_step(double uT, double uk, double rho, double inv_rho,
                                            double h, double& XT, double& Xk, const Control& c,
                                            const CoopCtx<M>& x, const CoopLane<M, G>& ln) {
  using S = CoopScratch<M>;
  constexpr int N = M::NS, N1 = N + 1;
  double UT = uT, Uk = uk, ET = 0.0, Ek = 0.0;
  XT = uT;
  Xk = uk;
  auto stage = [&](int s) {
    double FT;
    const double Fk = coop_rhs<M, G>(Uk, UT, rho, inv_rho, x, ln, FT);
    const double bs = s == 0 ? LS_B[0] : s == 1 ? LS_B[1] : s == 2 ? LS_B[2] : s == 3 ? LS_B[3] : LS_B[4];
    const double bhs = s == 0 ? LS_BH[0] : s == 1 ? LS_BH[1] : s == 2 ? LS_BH[2] : s == 3 ? LS_BH[3] : LS_BH[4];
    const double as = s == 0 ? LS_A[0] : s == 1 ? LS_A[1] : s == 2 ? LS_A[2] : s == 3 ? LS_A[3] : 0.0;
    const double eh = (bs - bhs) * h;
    ET += eh * FT;
    Ek += eh * Fk;
    if (s < 4) {
      const double ah = as * h, bah = (bs - as) * h;
      UT = XT + ah * FT;
      XT = UT + bah * FT;
      Uk = Xk + ah * Fk;
      Xk = Uk + bah * Fk;
    } else {
      const double bh = bs * h;
      XT = XT + bh * FT;
      Xk = Xk + bh * Fk;
    }
  };
  if constexpr (CoopLane<M, G>::PRE) {
    // small mechanisms: the five stages unrolled (coefficients become
    // immediates, the loop's selects and branches go away: ~15 % fewer
    // instructions, still two waves per SIMD)
#pragma unroll
    for (int s = 0; s < 5; ++s) stage(s);
  } else {
    // large ones stay rolled: unrolled they would drop to one wave per SIMD
#pragma unroll 1
    for (int s = 0; s < 5; ++s) stage(s);
  }
  const double wT = ET / (c.rtol * fabs(uT) + c.atol);
  const double wk = Ek / (c.rtol * fabs(uk) + c.atol);
  coop_sync();
  x.s[x.gl < N ? S::SW + x.gl : S::SX + x.gl] = wk * wk;
  coop_sync();
  double sum = wT * wT;
#pragma unroll
  for (int kk = 0; kk < N; ++kk) sum += x.s[S::SW + kk];
  return sqrt(sum * (1.0 / N1));
}

// One attempted step towards dt (same control as `advance`): returns
// CELL_RUNNING or the cell's final code.
template <class M, int G>
__device__ __forceinline__ int coop_try_step(double& uT, double& uk, double rho, double inv_rho,
                                             double dt, double& t, double& h, int& nacc,
                                             int& nrej, const Control& c, const CoopCtx<M>& x,
                                             const CoopLane<M, G>& ln) {
  bool last = false;
  double hh = h;
  if (hh >= dt - t) { hh = dt - t; last = true; }
  double XT, Xk;
  const double err = coop_step<M, G>(uT, uk, rho, inv_rho, hh, XT, Xk, c, x, ln);
  const double fac = step_factor(err);
  if (err <= 1.0) {
    uT = XT;
    uk = Xk;
    ++nacc;
    if (last) { h = hh * fac; return CELL_OK; }
    t = t + hh;
  } else {
    ++nrej;
  }
  h = hh * fac;
  if (nacc + nrej >= c.max_steps) return CELL_MAXSTEPS;
  if (h < 1e-14 * dt) return CELL_H_UNDERFLOW;
  return CELL_RUNNING;
}

}  // namespace chemgpu
