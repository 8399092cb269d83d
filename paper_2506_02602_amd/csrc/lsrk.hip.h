// Device side of the per-cell LSRK chemistry integrator (gfx950, FP64 VALU).
//
// One cell per lane.  The cell's state vector u = (T, Y_1..Y_N) lives in
// registers as a fully unrolled array; the right-hand side is the
// mechanism's generated straight-line function M::rhs.
//
// Step (paper Eq. 21, two registers plus the error register): with
// F_i = f(U), for stages i = 1..5
//     E <- E + (b_i - bhat_i) h F_i
//     U <- X + a_{i+1,i} h F_i ;  X <- U + (b_i - a_{i+1,i}) h F_i      (i < 5)
//     X <- X + b_5 h F_5                                               (i = 5)
// Control (Eq. 22): err = WRMS(E) with weights rtol |u_n| + atol over all
// N+1 components; accept iff err <= 1; factor 0.9 err^(-1/4) clamped to
// [0.2, 5] (NaN error: 0.2; zero error: 5); the last step is clipped to end
// on dt.  Coefficients: Kennedy-Carpenter-Lewis RK4(3)5[2R+]C, the scheme
// the paper cites as its ref. [37].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chemgpu {

// Exact rationals of the published tableau; each quotient is a compile-time
// IEEE division of two exactly representable integers (correctly rounded).
constexpr double LS_A[4] = {970286171893.0 / 4311952581923.0,
                            6584761158862.0 / 12103376702013.0,
                            2251764453980.0 / 15575788980749.0,
                            26877169314380.0 / 34165994151039.0};
constexpr double LS_B[5] = {1153189308089.0 / 22510343858157.0,
                            1772645290293.0 / 4653164025191.0,
                            -1672844663538.0 / 4480602732383.0,
                            2114624349019.0 / 3568978502595.0,
                            5198255086312.0 / 14908931495163.0};
constexpr double LS_BH[5] = {1016888040809.0 / 7410784769900.0,
                             11231460423587.0 / 58533540763752.0,
                             -1563879915014.0 / 6823010717585.0,
                             606302364029.0 / 971179775848.0,
                             1097981568119.0 / 3980877426909.0};

enum : int { CELL_RUNNING = -1, CELL_OK = 0, CELL_MAXSTEPS = 1, CELL_NONFINITE = 2,
             CELL_H_UNDERFLOW = 3 };

struct Control {
  double rtol, atol;
  int max_steps;
};

// One LSRK step of size h from u; X receives the new state, returns the WRMS
// error.  The stage loop stays rolled so that the generated RHS is inlined
// once; the stage coefficients are wave-uniform scalars.
template <class M>
__device__ __forceinline__ double lsrk_step(const double (&u)[M::NS + 1], double rho,
                                            double inv_rho, double h, double (&X)[M::NS + 1],
                                            const Control& c) {
  constexpr int N1 = M::NS + 1;
  double U[N1], E[N1], F[N1];
#pragma unroll
  for (int i = 0; i < N1; ++i) { X[i] = u[i]; U[i] = u[i]; E[i] = 0.0; }
#pragma unroll 1
  for (int s = 0; s < 5; ++s) {
    M::rhs(U, rho, inv_rho, F);
    const double bs = s == 0 ? LS_B[0] : s == 1 ? LS_B[1] : s == 2 ? LS_B[2] : s == 3 ? LS_B[3] : LS_B[4];
    const double bhs = s == 0 ? LS_BH[0] : s == 1 ? LS_BH[1] : s == 2 ? LS_BH[2] : s == 3 ? LS_BH[3] : LS_BH[4];
    const double as = s == 0 ? LS_A[0] : s == 1 ? LS_A[1] : s == 2 ? LS_A[2] : s == 3 ? LS_A[3] : 0.0;
    const double eh = (bs - bhs) * h;
    if (s < 4) {
      const double ah = as * h;
      const double bah = (bs - as) * h;
#pragma unroll
      for (int i = 0; i < N1; ++i) {
        E[i] += eh * F[i];
        U[i] = X[i] + ah * F[i];
        X[i] = U[i] + bah * F[i];
      }
    } else {
      const double bh = bs * h;
#pragma unroll
      for (int i = 0; i < N1; ++i) {
        E[i] += eh * F[i];
        X[i] = X[i] + bh * F[i];
      }
    }
  }
  double sum = 0.0;
#pragma unroll
  for (int i = 0; i < N1; ++i) {
    const double w = E[i] / (c.rtol * fabs(u[i]) + c.atol);
    sum += w * w;
  }
  return sqrt(sum * (1.0 / N1));
}

// e^x for the rate constants: Cody-Waite reduction x = n ln2 + r, |r| <=
// ln2/2, with ln 2 split into its correctly rounded double and the
// remainder (both products applied with FMAs), then p(r) ~ e^r of degree 11
// in Horner form, scaled by 2^n with ldexp.  p is the Chebyshev
// approximation of e^r on [-ln2/2, ln2/2] (interpolation at the Chebyshev
// nodes, within a few per cent of the minimax polynomial), coefficients
// rounded to doubles: relative error below 1.7e-17 in exact arithmetic,
// 0.77 ulp with the Horner roundings (a CPU test re-evaluates these
// coefficients in extended precision).  n is clamped so that its conversion
// to int is defined; past the double range ldexp gives inf or 0 (or a
// subnormal); NaN propagates through r.  Within 1 ulp of a correctly
// rounded exponential on [-708, 709]; fewer instructions than the library
// exponential, which also tests for the out-of-range cases.  (Converting
// with an inline v_cvt_i32_f64, which saturates by itself, would save the
// clamp's two instructions, but the opaque statement costs the per-lane
// kernels their register allocation: mech9 went from 235 VGPRs to spills.)
__device__ __forceinline__ double exp_cw(double x) {
  constexpr double LOG2E = 1.4426950408889634;
  constexpr double LN2_HI = 0.6931471805599453;
  constexpr double LN2_LO = 2.3190468138462996e-17;
  double n = rint(x * LOG2E);
  n = fmax(fmin(n, 2100.0), -2100.0);
  const int ni = (int)n;
  double r = fma(-n, LN2_HI, x);
  r = fma(-n, LN2_LO, r);
  double p = 0x1.af631d0059becp-26;
  p = fma(p, r, 0x1.28b4057f44145p-22);
  p = fma(p, r, 0x1.71ddf5749d126p-19);
  p = fma(p, r, 0x1.a01991ac8730ap-16);
  p = fma(p, r, 0x1.a01a01b14378fp-13);
  p = fma(p, r, 0x1.6c16c187fbe02p-10);
  p = fma(p, r, 0x1.111111110f225p-7);
  p = fma(p, r, 0x1.555555554f0cfp-5);
  p = fma(p, r, 0x1.555555555555ap-3);
  p = fma(p, r, 0x1.0000000000011p-1);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, ni);
}

// 2^(j/64), j = 0..63: each the double nearest the exact value (hexadecimal
// literals, so the table is bit-exact).  The kernels that use exp_tab stage it
// in LDS.
static __constant__ double kExp2Frac[64] = {
    0x1.0000000000000p+0, 0x1.02c9a3e778061p+0, 0x1.059b0d3158574p+0, 0x1.0874518759bc8p+0,
    0x1.0b5586cf9890fp+0, 0x1.0e3ec32d3d1a2p+0, 0x1.11301d0125b51p+0, 0x1.1429aaea92de0p+0,
    0x1.172b83c7d517bp+0, 0x1.1a35beb6fcb75p+0, 0x1.1d4873168b9aap+0, 0x1.2063b88628cd6p+0,
    0x1.2387a6e756238p+0, 0x1.26b4565e27cddp+0, 0x1.29e9df51fdee1p+0, 0x1.2d285a6e4030bp+0,
    0x1.306fe0a31b715p+0, 0x1.33c08b26416ffp+0, 0x1.371a7373aa9cbp+0, 0x1.3a7db34e59ff7p+0,
    0x1.3dea64c123422p+0, 0x1.4160a21f72e2ap+0, 0x1.44e086061892dp+0, 0x1.486a2b5c13cd0p+0,
    0x1.4bfdad5362a27p+0, 0x1.4f9b2769d2ca7p+0, 0x1.5342b569d4f82p+0, 0x1.56f4736b527dap+0,
    0x1.5ab07dd485429p+0, 0x1.5e76f15ad2148p+0, 0x1.6247eb03a5585p+0, 0x1.6623882552225p+0,
    0x1.6a09e667f3bcdp+0, 0x1.6dfb23c651a2fp+0, 0x1.71f75e8ec5f74p+0, 0x1.75feb564267c9p+0,
    0x1.7a11473eb0187p+0, 0x1.7e2f336cf4e62p+0, 0x1.82589994cce13p+0, 0x1.868d99b4492edp+0,
    0x1.8ace5422aa0dbp+0, 0x1.8f1ae99157736p+0, 0x1.93737b0cdc5e5p+0, 0x1.97d829fde4e50p+0,
    0x1.9c49182a3f090p+0, 0x1.a0c667b5de565p+0, 0x1.a5503b23e255dp+0, 0x1.a9e6b5579fdbfp+0,
    0x1.ae89f995ad3adp+0, 0x1.b33a2b84f15fbp+0, 0x1.b7f76f2fb5e47p+0, 0x1.bcc1e904bc1d2p+0,
    0x1.c199bdd85529cp+0, 0x1.c67f12e57d14bp+0, 0x1.cb720dcef9069p+0, 0x1.d072d4a07897cp+0,
    0x1.d5818dcfba487p+0, 0x1.da9e603db3285p+0, 0x1.dfc97337b9b5fp+0, 0x1.e502ee78b3ff6p+0,
    0x1.ea4afa2a490dap+0, 0x1.efa1bee615a27p+0, 0x1.f50765b6e4540p+0, 0x1.fa7c1819e90d8p+0,
};

// e^x from the 2^(j/64) table and a short polynomial, for the cooperative
// kernel: m = 64 k + j is the integer nearest 64 x / ln 2 (clamped so the
// conversion is defined), r = x - m ln2/64 by two FMAs with ln2/64 split in
// two parts (|r| <= ln2/128), and e^x = 2^k 2^(j/64) (1 + p(r)) with p the
// degree-6 Taylor polynomial of e^r - 1 (truncation below 3e-20 relative) by
// Estrin's scheme; t + t p is rounded once.  E points at kExp2Frac's values
// (in LDS).  Error: the table entry's rounding (at most 2^-53 relative) plus
// the final rounding, about 1 ulp at most on [-745, 709]; inf above, 0 or a
// subnormal below, NaN through, like exp_cw.  18 VALU instructions and one
// LDS read.
__device__ __forceinline__ double exp_tab(double x, const double* E) {
  constexpr double K = 92.33248261689366;            // 64 / ln 2
  constexpr double L_HI = 0.010830424696249145;        // ln2 / 64, nearest double
  constexpr double L_LO = 3.623510646634843e-19;   // ln2 / 64 - L_HI
  double m = rint(x * K);
  m = fmax(fmin(m, 134400.0), -134400.0);
  double r = fma(-m, L_HI, x);
  r = fma(-m, L_LO, r);
  const int mi = (int)m;
  const double t = E[mi & 63];
  const double r2 = r * r;
  const double a = fma(r, 1.0 / 6.0, 0.5);
  const double b = fma(r, 1.0 / 120.0, 1.0 / 24.0);
  const double q = fma(r2, fma(r2, 1.0 / 720.0, b), a);
  const double p = fma(r2, q, r);
  return ldexp(fma(t, p, t), mi >> 6);
}

// 1/x from the hardware reciprocal refined by two Newton steps: within an
// ulp of the quotient for normal x (T and the heat-capacity sum of the
// temperature equation, both positive), half the instructions of the IEEE
// division sequence.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}

// ln x for finite x > 0 (NaN otherwise) with a short dependency chain: x =
// 2^e m with m in [sqrt(1/2), sqrt(2)), f = m - 1 (exact), s = f / (2 + f)
// (hardware reciprocal refined by two Newton steps), and
// ln m = 2 atanh s = f - (f^2/2 - s (f^2/2 + R(s^2))) with R the series
// sum_k>=1 2 z^k / (2k + 1) in z = s^2 (|z| < 0.0295, ten terms, Estrin's
// scheme); e ln 2 is added with ln 2 split so that e times its leading part is
// exact, in the order that keeps the cancellation for x near 1/sqrt(2)
// harmless.  Within 1 ulp of the correctly rounded logarithm; about a third of
// the library logarithm's instructions and dependency depth, which carries
// double-double intermediates for correct rounding.
__device__ __forceinline__ double log_atanh(double x) {
  constexpr double LN2_HI = 0.6931471803691238;     // ln 2, low 21 mantissa bits cleared
  constexpr double LN2_LO = 1.9082149292705877e-10;  // ln 2 - LN2_HI
  constexpr double SQRT_HALF = 0.70710678118654752;
  double m = __builtin_amdgcn_frexp_mant(x);         // [0.5, 1)
  int e = __builtin_amdgcn_frexp_exp(x);
  const bool lo_half = m < SQRT_HALF;
  m = lo_half ? m + m : m;
  e = lo_half ? e - 1 : e;
  const double f = m - 1.0;
  const double d = 2.0 + f;
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  r = fma(fma(-d, r, 1.0), r, r);
  const double s = f * r;
  const double z = s * s;
  const double z2 = z * z, z4 = z2 * z2, z8 = z4 * z4;
  const double a0 = fma(2.0 / 5.0, z, 2.0 / 3.0), a1 = fma(2.0 / 9.0, z, 2.0 / 7.0);
  const double a2 = fma(2.0 / 13.0, z, 2.0 / 11.0), a3 = fma(2.0 / 17.0, z, 2.0 / 15.0);
  const double a4 = fma(2.0 / 21.0, z, 2.0 / 19.0);
  const double q = fma(a4, z8, fma(fma(a3, z2, a2), z4, fma(a1, z2, a0)));
  const double hfsq = 0.5 * f * f;
  const double de = (double)e;
  const double y = de * LN2_HI - ((hfsq - fma(s, fma(z, q, hfsq), de * LN2_LO)) - f);
  return x > 0.0 ? y : __builtin_nan("");
}

__device__ __forceinline__ double step_factor(double err) {
  if (err != err) return 0.2;
  if (err == 0.0) return 5.0;
  // err^(-1/4) as 1/sqrt(sqrt(err)): correctly rounded square roots and a
  // division, a few ulp from pow() at a tenth of its cost
  double fac = 0.9 / sqrt(sqrt(err));
  fac = fac < 0.2 ? 0.2 : fac;
  fac = fac > 5.0 ? 5.0 : fac;
  return fac;
}

template <int N1>
__device__ __forceinline__ bool all_finite(const double (&u)[N1], double rho) {
  bool ok = isfinite(rho);
#pragma unroll
  for (int i = 0; i < N1; ++i) ok = ok && isfinite(u[i]);
  return ok;
}

}  // namespace chemgpu
