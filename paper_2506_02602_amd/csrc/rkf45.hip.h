// Full-storage comparison scheme: Fehlberg's six-stage 4(5) pair (the paper
// compares its low-storage integrator with a Runge-Kutta-Fehlberg method,
// Sec. 4.2.2).  Stage i evaluates F at u + h sum_{j<i} a_ij K_j, so the
// stage vectors K_1..K_5 stay live in registers until the last stage -- the
// storage the two-register scheme of Eq. 21 avoids.  The step advances with
// the fourth-order weights; the error estimate is the difference to the
// fifth-order ones, and the controller exponent is 1/5.
#pragma once

#include <hip/hip_runtime.h>

#include "lsrk.hip.h"

namespace chemgpu {

constexpr double RKF_A[6][5] = {
    {0.0, 0.0, 0.0, 0.0, 0.0},
    {1.0 / 4.0, 0.0, 0.0, 0.0, 0.0},
    {3.0 / 32.0, 9.0 / 32.0, 0.0, 0.0, 0.0},
    {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0.0, 0.0},
    {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0.0},
    {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0}};
constexpr double RKF_B4[6] = {25.0 / 216.0, 0.0, 1408.0 / 2565.0, 2197.0 / 4104.0, -1.0 / 5.0, 0.0};
constexpr double RKF_B5[6] = {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0, -9.0 / 50.0,
                              2.0 / 55.0};

// Coefficient (s, j) of the tableau for a run-time stage s (a chain of
// selects on wave-uniform s).
__device__ __forceinline__ double rkf_a(int s, int j) {
  double v = 0.0;
#pragma unroll
  for (int r = 1; r < 6; ++r) v = (s == r) ? RKF_A[r][j] : v;
  return v;
}

__device__ __forceinline__ double rkf_pick(const double (&t)[6], int s) {
  double v = t[0];
#pragma unroll
  for (int r = 1; r < 6; ++r) v = (s == r) ? t[r] : v;
  return v;
}

// One Fehlberg step of size h from u: X receives the fourth-order solution,
// returns the WRMS norm of the embedded error.  The stage loop stays rolled
// (one inlined RHS); K_s is written through selects on the stage index so
// that the stage vectors keep static register indices.
template <class M>
__device__ __forceinline__ double rkf45_step(const double (&u)[M::NS + 1], double rho,
                                             double inv_rho, double h, double (&X)[M::NS + 1],
                                             const Control& c) {
  constexpr int N1 = M::NS + 1;
  double K[5][N1], U[N1], E[N1], F[N1];
#pragma unroll
  for (int i = 0; i < N1; ++i) { X[i] = u[i]; E[i] = 0.0; }
#pragma unroll
  for (int j = 0; j < 5; ++j)
#pragma unroll
    for (int i = 0; i < N1; ++i) K[j][i] = 0.0;
#pragma unroll 1
  for (int s = 0; s < 6; ++s) {
    double ah[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) ah[j] = rkf_a(s, j) * h;
#pragma unroll
    for (int i = 0; i < N1; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < 5; ++j) acc += ah[j] * K[j][i];
      U[i] = u[i] + acc;
    }
    M::rhs(U, rho, inv_rho, F);
    const double b4h = rkf_pick(RKF_B4, s) * h;
    const double eh = (rkf_pick(RKF_B5, s) - rkf_pick(RKF_B4, s)) * h;
#pragma unroll
    for (int i = 0; i < N1; ++i) {
      X[i] += b4h * F[i];
      E[i] += eh * F[i];
    }
#pragma unroll
    for (int j = 0; j < 5; ++j)
#pragma unroll
      for (int i = 0; i < N1; ++i) K[j][i] = (s == j) ? F[i] : K[j][i];
  }
  double sum = 0.0;
#pragma unroll
  for (int i = 0; i < N1; ++i) {
    const double w = E[i] / (c.rtol * fabs(u[i]) + c.atol);
    sum += w * w;
  }
  return sqrt(sum * (1.0 / N1));
}

// Eq. 22's factor for the fourth-order estimate: 0.9 err^(-1/5) in [0.2, 5].
__device__ __forceinline__ double step_factor_rkf(double err) {
  if (err != err) return 0.2;
  if (err == 0.0) return 5.0;
  double fac = 0.9 * pow(err, -0.2);
  fac = fac < 0.2 ? 0.2 : fac;
  fac = fac > 5.0 ? 5.0 : fac;
  return fac;
}

}  // namespace chemgpu
