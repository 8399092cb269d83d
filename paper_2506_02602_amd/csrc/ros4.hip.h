// Implicit comparator: a linearly implicit (Rosenbrock) step, fourth order
// with an embedded third-order solution -- Shampine's parameter set in the
// Kaps-Rentrop form -- standing in for the implicit integrator the paper
// measures its explicit scheme against (Sec. 4.2.2).  Per cell and step:
// the exact Jacobian (generated `M::jac`, which also returns f(u_n)),
// W = I/(gamma h) - J factorised by LU with partial pivoting, three RHS
// evaluations and four solves:
//   W g1 = f(u_n)
//   W g2 = f(u_n + a21 g1) + c21 g1 / h
//   W g3 = f(u_n + a31 g1 + a32 g2) + (c31 g1 + c32 g2) / h
//   W g4 = f(u_n + a31 g1 + a32 g2) + (c41 g1 + c42 g2 + c43 g3) / h
//   u_{n+1} = u_n + sum b_i g_i,  error = sum e_i g_i,
// under the same WRMS controller (exponent 1/4, the embedded order being 3).
// One cell per lane: the (N+1)^2 matrix lives in registers with static
// indices, so the factorisation is fully unrolled and row swaps are selects.
#pragma once

#include <hip/hip_runtime.h>

#include "lsrk.hip.h"

namespace chemgpu {

constexpr double RO_GAMMA = 0.5;
constexpr double RO_A21 = 2.0, RO_A31 = 48.0 / 25.0, RO_A32 = 6.0 / 25.0;
constexpr double RO_C21 = -8.0, RO_C31 = 372.0 / 25.0, RO_C32 = 12.0 / 5.0;
constexpr double RO_C41 = -112.0 / 125.0, RO_C42 = -54.0 / 125.0, RO_C43 = -2.0 / 5.0;
constexpr double RO_B1 = 19.0 / 9.0, RO_B2 = 1.0 / 2.0, RO_B3 = 25.0 / 108.0, RO_B4 = 125.0 / 108.0;
constexpr double RO_E1 = 17.0 / 54.0, RO_E2 = 7.0 / 36.0, RO_E4 = 125.0 / 108.0;

// P A = L U in place (unit L below the diagonal, whole rows swapped);
// piv[k] = the row exchanged with row k at column k.
template <int n>
__device__ __forceinline__ void lu_factor_regs(double (&a)[n * n], int (&piv)[n]) {
#pragma unroll
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = fabs(a[k * n + k]);
#pragma unroll
    for (int r = k + 1; r < n; ++r) {
      const double v = fabs(a[r * n + k]);
      const bool bigger = v > best;
      best = bigger ? v : best;
      p = bigger ? r : p;
    }
    piv[k] = p;
#pragma unroll
    for (int r = k + 1; r < n; ++r) {
      const bool sw = p == r;
#pragma unroll
      for (int j = 0; j < n; ++j) {
        const double x = a[k * n + j], y = a[r * n + j];
        a[k * n + j] = sw ? y : x;
        a[r * n + j] = sw ? x : y;
      }
    }
    const double inv = 1.0 / a[k * n + k];
#pragma unroll
    for (int r = k + 1; r < n; ++r) {
      const double l = a[r * n + k] * inv;
      a[r * n + k] = l;
#pragma unroll
      for (int j = k + 1; j < n; ++j) a[r * n + j] -= l * a[k * n + j];
    }
  }
}

// Solve A x = b in place from the factors: b <- P b (every swap, in
// factorisation order), then L y = P b and U x = y.
template <int n>
__device__ __forceinline__ void lu_solve_regs(const double (&a)[n * n], const int (&piv)[n],
                                              double (&b)[n]) {
#pragma unroll
  for (int k = 0; k < n; ++k) {
#pragma unroll
    for (int r = k + 1; r < n; ++r) {
      const bool sw = piv[k] == r;
      const double x = b[k], y = b[r];
      b[k] = sw ? y : x;
      b[r] = sw ? x : y;
    }
  }
#pragma unroll
  for (int k = 0; k < n; ++k)
#pragma unroll
    for (int r = k + 1; r < n; ++r) b[r] -= a[r * n + k] * b[k];
#pragma unroll
  for (int k = n - 1; k >= 0; --k) {
    double s = b[k];
#pragma unroll
    for (int j = k + 1; j < n; ++j) s -= a[k * n + j] * b[j];
    b[k] = s / a[k * n + k];
  }
}

// One Rosenbrock step of size h from u: X receives the fourth-order
// solution; returns the WRMS norm of the embedded error estimate.
template <class M>
__device__ __forceinline__ double ros4_step(const double (&u)[M::NS + 1], double rho,
                                            double inv_rho, double h, double (&X)[M::NS + 1],
                                            const Control& c) {
  constexpr int N1 = M::NS + 1;
  double A[N1 * N1], F[N1], g1[N1], g2[N1], g3[N1], g4[N1], y[N1];
  int piv[N1];
  M::jac(u, rho, inv_rho, F, A);
  const double d = 1.0 / (RO_GAMMA * h);
  const double inv_h = 1.0 / h;
#pragma unroll
  for (int i = 0; i < N1 * N1; ++i) A[i] = -A[i];
#pragma unroll
  for (int i = 0; i < N1; ++i) A[i * N1 + i] += d;
  lu_factor_regs<N1>(A, piv);
#pragma unroll
  for (int i = 0; i < N1; ++i) { g1[i] = F[i]; g2[i] = 0.0; }
  lu_solve_regs<N1>(A, piv, g1);
  // the second and third RHS evaluations share one inlined RHS
#pragma unroll 1
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int i = 0; i < N1; ++i)
      y[i] = s == 0 ? u[i] + RO_A21 * g1[i] : u[i] + RO_A31 * g1[i] + RO_A32 * g2[i];
    M::rhs(y, rho, inv_rho, F);
    if (s == 0) {
#pragma unroll
      for (int i = 0; i < N1; ++i) g2[i] = F[i] + (RO_C21 * inv_h) * g1[i];
      lu_solve_regs<N1>(A, piv, g2);
    }
  }
#pragma unroll
  for (int i = 0; i < N1; ++i) g3[i] = F[i] + (RO_C31 * g1[i] + RO_C32 * g2[i]) * inv_h;
  lu_solve_regs<N1>(A, piv, g3);
#pragma unroll
  for (int i = 0; i < N1; ++i)
    g4[i] = F[i] + (RO_C41 * g1[i] + RO_C42 * g2[i] + RO_C43 * g3[i]) * inv_h;
  lu_solve_regs<N1>(A, piv, g4);
  double sum = 0.0;
#pragma unroll
  for (int i = 0; i < N1; ++i) {
    X[i] = u[i] + RO_B1 * g1[i] + RO_B2 * g2[i] + RO_B3 * g3[i] + RO_B4 * g4[i];
    const double e = RO_E1 * g1[i] + RO_E2 * g2[i] + RO_E4 * g4[i];
    const double w = e / (c.rtol * fabs(u[i]) + c.atol);
    sum += w * w;
  }
  return sqrt(sum * (1.0 / N1));
}

}  // namespace chemgpu
