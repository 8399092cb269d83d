// Per-lane step driver shared by the kernels: the adaptive advance towards
// dt with the Eq. 22 controller and the fixed-step test mode, for each
// scheme (the paper's low-storage LSRK4(3)5, the full-storage Fehlberg 4(5)
// comparison scheme, or the implicit Rosenbrock comparator).
#pragma once

#include "lsrk.hip.h"
#include "rkf45.hip.h"
#include "ros4.hip.h"

namespace chemgpu {

enum : int { SCHEME_LSRK = 0, SCHEME_RKF45 = 1, SCHEME_ROS4 = 2 };

template <class M, int S>
__device__ __forceinline__ double take_step(const double (&u)[M::NS + 1], double rho,
                                            double inv_rho, double h, double (&X)[M::NS + 1],
                                            const Control& c) {
  if constexpr (S == SCHEME_RKF45)
    return rkf45_step<M>(u, rho, inv_rho, h, X, c);
  else if constexpr (S == SCHEME_ROS4)
    return ros4_step<M>(u, rho, inv_rho, h, X, c);
  else
    return lsrk_step<M>(u, rho, inv_rho, h, X, c);
}

// Advance one cell by at most `budget` steps towards dt.  (t, h, nacc, nrej)
// carry the cell's progress.  Returns CELL_RUNNING or a final CELL_* code.
template <class M, int S = SCHEME_LSRK>
__device__ __forceinline__ int advance(double (&u)[M::NS + 1], double rho, double inv_rho,
                                       double dt, double& t, double& h, int& nacc, int& nrej,
                                       const Control& c, int budget) {
  constexpr int N1 = M::NS + 1;
#pragma unroll 1
  for (int s = 0; s < budget; ++s) {
    bool last = false;
    double hh = h;
    if (hh >= dt - t) { hh = dt - t; last = true; }
    double X[N1];
    const double err = take_step<M, S>(u, rho, inv_rho, hh, X, c);
    const double fac = S == SCHEME_RKF45 ? step_factor_rkf(err) : step_factor(err);
    if (err <= 1.0) {
#pragma unroll
      for (int i = 0; i < N1; ++i) u[i] = X[i];
      ++nacc;
      if (last) { h = hh * fac; return CELL_OK; }
      t = t + hh;
    } else {
      ++nrej;
    }
    h = hh * fac;
    if (nacc + nrej >= c.max_steps) return CELL_MAXSTEPS;
    if (h < 1e-14 * dt) return CELL_H_UNDERFLOW;
  }
  return CELL_RUNNING;
}

// Test mode: exactly n steps of dt/n, every step accepted.
template <class M, int S = SCHEME_LSRK>
__device__ __forceinline__ void advance_fixed(double (&u)[M::NS + 1], double rho, double inv_rho,
                                              double dt, int n, double& h, int& nacc,
                                              const Control& c) {
  constexpr int N1 = M::NS + 1;
  const double hh = dt / n;
#pragma unroll 1
  for (int s = 0; s < n; ++s) {
    double X[N1];
    (void)take_step<M, S>(u, rho, inv_rho, hh, X, c);
#pragma unroll
    for (int i = 0; i < N1; ++i) u[i] = X[i];
  }
  nacc = n;
  h = hh;
}

}  // namespace chemgpu
