// Cooperative integration: G lanes of one wave advance one cell together.
//
// Used for the tail of a flow step -- the few stiff cells still stepping
// after the rest have finished -- where one cell per lane leaves the chip
// nearly idle and the step latency of a single lane bounds the whole call.
// Splitting one cell's right-hand side over G lanes cuts that latency.
//
// Lane roles within a group (gl = lane index in the group, 0..G-1):
//   component lane  gl <= N: holds component gl of the state and of the
//                   stage registers X, U, E (0 = T, k+1 = Y_k); lanes
//                   1..N also evaluate species k's concentration and NASA-7
//                   thermo (paper Eq. 10) and sum its production rate;
//   reaction lane   j = gl + r G < J: reaction j's forward and reverse rates
//                   and rate of progress (paper Eq. 15-16).
// The rate law is the one of the unrolled per-lane RHS, read from the
// mechanism's generated tables.  Concentrations, g_k/RT and rates of
// progress pass between lanes through the group's LDS area; the energy
// closure and the WRMS norm are summed with xor butterflies, which leave
// every lane of the group with the same bits, so the step-control decisions
// (paper Eq. 22) are uniform within the group.
#pragma once

#include <hip/hip_runtime.h>

#include "lsrk.hip.h"

namespace chemgpu {

__device__ __forceinline__ void coop_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int G>
__device__ __forceinline__ double group_sum(double x) {
#pragma unroll
  for (int m = 1; m < G; m <<= 1) x += __shfl_xor(x, m, G);
  return x;
}

// LDS scratch of one group: concentrations c[N+1] (c[N] = 1, the pad of the
// species lists), g/RT g[N+1] (g[N] = 0), rates of progress q[J].
template <class M>
struct CoopScratch {
  static constexpr int N1 = M::NS + 1;
  static constexpr int SIZE = (2 * N1 + M::Coop::J + 1) & ~1;  // doubles
};

template <class M>
struct CoopCtx {
  const double* D;  // the mechanism's double table, in LDS
  const int* I;     // its int table, in LDS
  double* s;        // this group's scratch
  int gl;
};

// This lane's component of f(U) (0 for lanes past N).
template <class M, int G>
__device__ __forceinline__ double coop_rhs(double Uv, double rho, double inv_rho,
                                           const CoopCtx<M>& x) {
  using C = typename M::Coop;
  constexpr int N = M::NS;
  constexpr int R = (C::J + G - 1) / G;
  double* sc = x.s;
  double* sg = x.s + (N + 1);
  double* sq = x.s + 2 * (N + 1);
  const double* D = x.D;
  const int* I = x.I;
  const int gl = x.gl;
  const double T = __shfl(Uv, 0, G);
  const double lnT = log(T);
  const double invT = 1.0 / T;
  const double omlnT = 1.0 - lnT;
  const double lnPRT = C::LNPRT0 - lnT;
  const bool sl = gl >= 1 && gl <= N;
  const int k = sl ? gl - 1 : 0;
  double hk = 0.0, dpart = 0.0;
  coop_sync();  // the previous evaluation's readers of the scratch are done
  if (sl) {
    const double c = Uv * (rho * D[C::O_INVW + k]);
    const double* th = D + C::O_TH + (T < D[C::O_TMID + k] ? 0 : N * C::TH_ROW) + k * C::TH_ROW;
    hk = th[0] + T * (th[1] + T * (th[2] + T * (th[3] + T * th[4]))) + th[5] * invT;
    const double gp = th[7] + T * (th[8] + T * (th[9] + T * th[10]));
    sg[k] = th[6] * omlnT - T * gp + th[5] * invT - th[11];
    dpart = c * (th[12] + T * (th[13] + T * (th[14] + T * (th[15] + T * th[16]))));
    sc[k] = c;
  }
  coop_sync();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = gl + r * G;
    if (j < C::J) {
      const double lkf = D[C::O_LNA + j] + D[C::O_BEXP + j] * lnT - D[C::O_EAR + j] * invT;
      const double kf = exp(lkf);
      double dg = 0.0;
#pragma unroll
      for (int q = 0; q < C::MG; ++q)
        dg += D[C::O_GNU + j * C::MG + q] * sg[I[C::O_GK + j * C::MG + q]];
      const double kr = exp(lkf + dg - D[C::O_DNU + j] * lnPRT);
      double fw = kf, rv = kr;
#pragma unroll
      for (int q = 0; q < C::MR; ++q) {
        fw *= sc[I[C::O_RI + j * C::MR + q]];
        rv *= sc[I[C::O_PI + j * C::MR + q]];
      }
      double qj = fw - rv;
      const int tb = I[C::O_TB + j];
      if (tb >= 0) {
        double mt = 0.0;
#pragma unroll
        for (int kk = 0; kk < N; ++kk) mt += D[C::O_TBEFF + tb * N + kk] * sc[kk];
        qj = mt * qj;
      }
      sq[j] = qj;
    }
  }
  coop_sync();
  double wk = 0.0;
  if (sl) {
#pragma unroll
    for (int l = 0; l < C::L; ++l)
      wk += D[C::O_SLNU + k * C::L + l] * sq[I[C::O_SLJ + k * C::L + l]];
  }
  const double num = group_sum<G>(sl ? (hk - 1.0) * wk : 0.0);
  const double den = group_sum<G>(dpart);
  if (gl == 0) return -T * num / den;
  return sl ? wk * (D[C::O_WK + k] * inv_rho) : 0.0;
}

// One step of size h (paper Eq. 21), this lane's component; returns the
// group's WRMS error.
template <class M, int G>
__device__ __forceinline__ double coop_step(double uv, double rho, double inv_rho, double h,
                                            double& Xv, const Control& c, const CoopCtx<M>& x) {
  constexpr int N1 = M::NS + 1;
  double U = uv, E = 0.0;
  Xv = uv;
#pragma unroll 1
  for (int s = 0; s < 5; ++s) {
    const double F = coop_rhs<M, G>(U, rho, inv_rho, x);
    const double bs = s == 0 ? LS_B[0] : s == 1 ? LS_B[1] : s == 2 ? LS_B[2] : s == 3 ? LS_B[3] : LS_B[4];
    const double bhs = s == 0 ? LS_BH[0] : s == 1 ? LS_BH[1] : s == 2 ? LS_BH[2] : s == 3 ? LS_BH[3] : LS_BH[4];
    const double as = s == 0 ? LS_A[0] : s == 1 ? LS_A[1] : s == 2 ? LS_A[2] : s == 3 ? LS_A[3] : 0.0;
    const double eh = (bs - bhs) * h;
    E += eh * F;
    if (s < 4) {
      U = Xv + (as * h) * F;
      Xv = U + ((bs - as) * h) * F;
    } else {
      Xv = Xv + (bs * h) * F;
    }
  }
  const double w = x.gl < N1 ? E / (c.rtol * fabs(uv) + c.atol) : 0.0;
  return sqrt(group_sum<G>(w * w) * (1.0 / N1));
}

// One attempted step towards dt (same control as `advance`): returns
// CELL_RUNNING or the cell's final code.
template <class M, int G>
__device__ __forceinline__ int coop_try_step(double& uv, double rho, double inv_rho, double dt,
                                             double& t, double& h, int& nacc, int& nrej,
                                             const Control& c, const CoopCtx<M>& x) {
  bool last = false;
  double hh = h;
  if (hh >= dt - t) { hh = dt - t; last = true; }
  double Xv;
  const double err = coop_step<M, G>(uv, rho, inv_rho, hh, Xv, c, x);
  const double fac = step_factor(err);
  if (err <= 1.0) {
    uv = Xv;
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
