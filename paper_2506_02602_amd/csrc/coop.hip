// coop.hip -- the cooperative integrator kernel (several lanes per cell; the
// LSRK4(3)5 step of paper Eq. 21 under the controller of Eq. 22), compiled on its own
// so that loop-invariant constants of its step loop may stay in registers
// (the per-lane kernels are built with that hoisting off: there it costs
// registers and spills).
#include <hip/hip_runtime.h>

#include "pool.hip.h"
#include "lsrk_coop.hip.h"

using namespace chemgpu;

#include "generated/registry.inc"

namespace chemgpu {
namespace {

// ------------------------------------------------------- cooperative kernel
// Finishes the cells the persistent kernel handed over: each group of
// Coop::G lanes (floor(64 / G) groups per wave) claims tail records one at
// a time and integrates that cell to the end of its flow step (all
// remaining sub-calls).  Grid-size independent: a group exits once the
// records are used up.
template <class M>
size_t coop_lds_bytes(int block) {
  using C = typename M::Coop;
  const int groups = (block / 64) * CoopWave<C::G>::GPW;
  return (size_t)(C::ND + 64) * sizeof(double) + (size_t)C::NI * sizeof(int) +
         (size_t)groups * CoopScratch<M>::SIZE * sizeof(double);
}

template <class M>
__global__ __launch_bounds__(256) void lsrk_coop(PoolArgs a) {
  using C = typename M::Coop;
  constexpr int G = C::G, N = M::NS;
  static_assert(C::NI % 4 == 0 && C::ND % 2 == 0, "table padding");
  // LDS: the double table, the 2^(j/64) table, the int table, group scratch
  extern __shared__ double smem[];
  double* D = smem;
  double* E = smem + C::ND;
  int* I = reinterpret_cast<int*>(smem + C::ND + 64);
  double* scr = smem + C::ND + 64 + C::NI / 2;
  const unsigned int count = *a.tail.split;  // the records this kernel takes (tail_scatter)
  if (count == 0u) return;
  const int tid = threadIdx.x;
  for (int i = tid; i < C::ND; i += blockDim.x) D[i] = C::dtab()[i];
  for (int i = tid; i < C::NI; i += blockDim.x) I[i] = C::itab()[i];
  for (int i = tid; i < 64; i += blockDim.x) E[i] = kExp2Frac[i];
  // group gw of this wave, lane gl within it; lanes past the wave's last
  // group (gw == GPW) take no cells
  constexpr int GPW = CoopWave<G>::GPW;
  const int lane = tid & 63;
  const int gw = min(lane / G, GPW);
  const int gl = lane - gw * G;
  const bool idle = gw == GPW;
  using S = CoopScratch<M>;
  double* sgrp = scr + ((tid >> 6) * GPW + (idle ? 0 : gw)) * S::SIZE;
  if (gl == 0 && !idle) {
    sgrp[S::SC + N] = 1.0;
    sgrp[S::SG + N] = 0.0;
  }
  __syncthreads();
  const CoopCtx<M> x{D, E, I, sgrp, gl};
  CoopLane<M, G> ln;
  ln.load(D, I, gl);
  // One step per iteration; a group whose cell finishes claims the next
  // record at once instead of waiting for the other groups of its wave.
  bool have = false;
  double* st = nullptr;
  int32_t* status = nullptr;
  int32_t* counts = nullptr;
  int64_t ld = 0, nbox = 0, i = 0;
  double dt = 0.0;
  int n_sub = 1;
  double uT = 0.0, uk = 0.0, rho = 1.0, inv_rho = 1.0, h = 0.0, t = 0.0;
  int nacc = 0, nrej = 0, sub = 0, base = 0, n0 = 0;
#pragma unroll 1
  for (;;) {
    if (idle) break;
    if (!have) {
      unsigned int r = 0;
      if (gl == 0) r = (unsigned int)atomicAdd(a.tail.next, 1ull);
      r = __shfl(r, gw * G);  // the group's first lane, within the wave
      if (r >= count) break;
      r = (unsigned int)a.tail.order[r];
      using TR = TailRec<M>;
      const double* rc = a.tail.rec ? a.tail.rec + (int64_t)r * TR::RD : nullptr;
      const int* ri = rc ? reinterpret_cast<const int*>(rc + TR::INTS) : nullptr;
      const int64_t item = rc ? ri[0] : a.tail.item[r];
      {
        const BoxDesc& bd = box_ref(a, find_box(a, item));
        i = cell_index(bd, item);
        st = bd.state; ld = bd.ld; nbox = bd.n; dt = bd.dt; n_sub = bd.n_sub;
        status = bd.status; counts = bd.counts;
      }
      if (rc) {
        // the state travels with the record; the cell's rows get the result
        uT = rc[0];
        uk = gl < N ? rc[gl + 1] : 0.0;
        rho = rc[TR::RHO];
        h = rc[TR::H];
        t = rc[TR::T];
        nacc = ri[1]; nrej = ri[2]; sub = ri[3]; base = ri[4];
      } else {
        uT = st[i];
        uk = gl < N ? st[(gl + 1) * ld + i] : 0.0;
        rho = st[(N + 1) * ld + i];
        h = st[(N + 2) * ld + i];
        t = a.tail.t[r];
        nacc = a.tail.nacc[r]; nrej = a.tail.nrej[r];
        sub = a.tail.sub[r]; base = a.tail.base[r];
      }
      inv_rho = 1.0 / rho;
      n0 = nacc + nrej;
      have = true;
    }
    Control c = a.c;
    c.max_steps = base + a.c.max_steps;
    int code = coop_try_step<M, G>(uT, uk, rho, inv_rho, dt, t, h, nacc, nrej, c, x, ln);
    if (code == CELL_OK && sub + 1 < n_sub) {
      ++sub; t = 0.0; base = nacc + nrej;
      h = initial_h(h, dt);
      code = CELL_RUNNING;
    }
    if (code != CELL_RUNNING) {
      if (gl < N) st[(gl + 1) * ld + i] = uk;
      if (gl == 0) {
        st[i] = uT;
        st[(N + 2) * ld + i] = h;
        if (status) status[i] = code;
        if (counts) { counts[i] = nacc; counts[nbox + i] = nrej; }
        atomicAdd(a.tail.coop_steps, (unsigned long long)(nacc + nrej - n0));
      }
      have = false;
    }
  }
}

}  // namespace

// The cooperative kernel after the persistent one: enough 256-lane blocks to
// put one group on every SIMD several times over; surplus groups exit at once.
template <class M>
hipError_t launch_coop(const PoolArgs& a, int n_cu, hipStream_t s) {
  constexpr int kBlock = 256;
  const size_t lds = coop_lds_bytes<M>(kBlock);
  if (lds > 65536) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(lsrk_coop<M>, dim3(4 * n_cu), dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

#define CHEM_COOP_INSTANCE(M) template hipError_t launch_coop<M>(const PoolArgs&, int, hipStream_t);
CHEM_FOR_EACH_MECH(CHEM_COOP_INSTANCE)
#undef CHEM_COOP_INSTANCE

}  // namespace chemgpu
