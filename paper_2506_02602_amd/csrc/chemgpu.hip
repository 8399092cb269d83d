// chemgpu.hip -- kernels and C ABI of the per-cell FP64 chemistry integrator.
//
// Kernels
//   lsrk_direct     one cell per lane for the whole flow step (no compaction).
//   lsrk_persistent persistent workgroups over a pool of work items (cells of
//                   one or more state blocks); every `chunk` steps the
//                   still-active cells of a workgroup are packed through LDS
//                   into its lowest lanes and the freed lanes take fresh
//                   items from a global atomic counter.  A work item is
//                   (block, cell); a block may ask for n_sub successive
//                   sub-calls of its own dt (AMR subcycling: a level-l box
//                   runs 2^l calls of dt0 / 2^l, paper Algorithm 1).
//
// Memory: the caller's SoA state is read when a lane claims an item and
// written when the item finishes; no cell's data is touched by two
// workgroups, so no cross-workgroup coherence is needed beyond the pool
// counter's atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "chemgpu.h"
#include "advance.hip.h"
#include "pool.hip.h"

using namespace chemgpu;

#include "generated/registry.inc"

namespace {

// ------------------------------------------------------------ direct kernel
template <class M, int LB, int S>
__global__ __launch_bounds__(LB) void lsrk_direct(PoolArgs a) {
  constexpr int N1 = M::NS + 1;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const BoxDesc& bd = a.one;
  if (i >= bd.n) return;
  double u[N1], rho, h;
  load_cell<M>(bd, i, u, rho, h);
  int nacc = 0, nrej = 0, st;
  if (!all_finite(u, rho)) {
    st = CELL_NONFINITE;
  } else {
    const double inv_rho = 1.0 / rho;
    if (a.fixed_steps > 0) {
      advance_fixed<M, S>(u, rho, inv_rho, bd.dt, a.fixed_steps, h, nacc, a.c);
      st = CELL_OK;
    } else {
      double t = 0.0;
      h = initial_h(h, bd.dt);
      st = advance<M, S>(u, rho, inv_rho, bd.dt, t, h, nacc, nrej, a.c, a.c.max_steps);
    }
  }
  store_cell<M>(bd, i, u, h, st, nacc, nrej);
}

// -------------------------------------------------------- persistent kernel
// Per-lane slot in LDS used to pack active cells: u[N1], t, h, rho (doubles)
// then item, nacc, nrej, sub, base, box (ints).
template <class M>
struct Slots {
  static constexpr int N1 = M::NS + 1;
  static constexpr int ND = N1 + 3;
  static constexpr int NI = 6;  // item, nacc, nrej, sub, base, box
  static size_t bytes(int block) { return (size_t)block * (ND * sizeof(double) + NI * sizeof(int)); }
};

__global__ void eval_math_kernel(int fn, const double* x, double* y, int64_t n) {
  __shared__ double E[64];  // exp_tab's table, staged in LDS as in the cooperative kernel
  for (int k = threadIdx.x; k < 64; k += blockDim.x) E[k] = kExp2Frac[k];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = x[i];
  y[i] = fn == CHEM_MATH_LOG_ATANH ? log_atanh(v)
         : fn == CHEM_MATH_EXP_TAB   ? exp_tab(v, E)
                                     : exp_cw(v);
}

__global__ void pool_reset(unsigned long long* next, unsigned int* tail_count,
                           unsigned long long* tail_next, unsigned long long* tail_next2,
                           unsigned long long* coop_steps, unsigned int* buckets) {
  if (threadIdx.x == 0) {
    *next = 0ull;
    if (tail_count) *tail_count = 0u;
    if (tail_next) *tail_next = 0ull;
    if (tail_next2) *tail_next2 = 0ull;
    if (coop_steps) *coop_steps = 0ull;
  }
  if (buckets) buckets[threadIdx.x] = 0u;
}

// Order of the tail list.  Handed-over cells are claimed one after another
// (by the cooperative kernel's groups, or one per lane by the per-lane
// resumption), so the flow step ends when whoever claimed the longest
// remaining integration finishes it; claiming the longest first (the
// longest-processing-time rule of list scheduling) keeps a long cell from
// starting late, and when the list is resumed one per lane it keeps the
// launch from draining on long cells claimed last.  A cell's remaining work
// is estimated from its state at the hand-off, in its current step size:
// rem/h steps for the time rem left in its flow step (all remaining
// sub-calls); the key buckets that estimate four to an octave, 0 for fewer
// than two steps, up to kTailBuckets - 1.
constexpr int kTailBuckets = 64;

__device__ __forceinline__ int32_t tail_key(double rem, double h) {
  const double est = rem / h;
  if (!(est > 1.0)) return 0;
  const double k = 4.0 * log2(est);
  return k >= (double)(kTailBuckets - 1) ? kTailBuckets - 1 : (int32_t)k;
}

// Wave priorities for the resumption launch.  When the longest handed-over
// cell's estimate (the top bucket of the key histogram btot) exceeds the
// per-lane share of all the estimated steps, the launch ends with its
// longest cells stepping while most lanes are idle; a wave whose cells have
// more steps left then issues first on its SIMD (s_setprio) and the others
// fill its stalls.  Returns the top level's threshold, half the longest
// estimate, or 0 (off) when the work per lane exceeds the longest cell and
// the launch is bound by throughput, where priorities only cost issue slots.
// Scheduling only: no result depends on it.
__device__ __forceinline__ float resume_priority(const unsigned int* btot, float lanes) {
  int k = kTailBuckets - 1;
  while (k > 0 && btot[k] == 0u) --k;
  float sum = 0.f;
  for (int j = 0; j <= k; ++j) sum += (float)btot[j] * exp2f(((float)j + 0.5f) * 0.25f);
  const float top = exp2f((float)(k + 1) * 0.25f);
  return top >= sum / lanes ? 0.5f * top : 0.f;
}

// Counting sort of the tail records by key, largest first, over the whole
// grid: tail_count adds every block's histogram of its chunk of records to
// the bucket totals; tail_scatter gives each block a range per bucket (one
// atomic per bucket and block) and writes the record indices into tb.order.
// Both read the record count on the device, so a captured launch sequence
// serves any list length.  tail_scatter also decides which kernel finishes
// the list: at most tb.cap records go to the cooperative kernel (split =
// count), more are resumed one per lane (split = 0); several lanes per cell
// only pay while the list is short next to the chip, and the choice depends
// only on the list's length, so on the input.  Records with equal keys keep
// no particular order: a cell's integration does not depend on when or by
// which lanes it runs.
constexpr int kSortBlock = 1024;
constexpr int kSortGridMax = 512;

__device__ __forceinline__ void sort_chunk(unsigned int count, unsigned int& lo, unsigned int& hi) {
  const unsigned int per = (count + gridDim.x - 1u) / gridDim.x;
  lo = min(count, blockIdx.x * per);
  hi = min(count, lo + per);
}

__global__ __launch_bounds__(kSortBlock) void tail_count(TailBuf tb) {
  __shared__ unsigned int h[kTailBuckets];
  const unsigned int count = *tb.count;
  if (count == 0u) return;
  for (int k = threadIdx.x; k < kTailBuckets; k += blockDim.x) h[k] = 0u;
  __syncthreads();
  unsigned int lo, hi;
  sort_chunk(count, lo, hi);
  for (unsigned int r = lo + threadIdx.x; r < hi; r += blockDim.x) atomicAdd(&h[tb.key[r]], 1u);
  __syncthreads();
  for (int k = threadIdx.x; k < kTailBuckets; k += blockDim.x)
    if (h[k]) atomicAdd(&tb.btot[k], h[k]);
}

__global__ __launch_bounds__(kSortBlock) void tail_scatter(TailBuf tb) {
  __shared__ unsigned int h[kTailBuckets], base[kTailBuckets];
  const unsigned int count = *tb.count;
  if (blockIdx.x == 0 && threadIdx.x == 0)
    *tb.split = count > 0u && count <= (unsigned int)tb.cap ? count : 0u;
  if (count == 0u) return;
  for (int k = threadIdx.x; k < kTailBuckets; k += blockDim.x) h[k] = 0u;
  __syncthreads();
  unsigned int lo, hi;
  sort_chunk(count, lo, hi);
  for (unsigned int r = lo + threadIdx.x; r < hi; r += blockDim.x) atomicAdd(&h[tb.key[r]], 1u);
  __syncthreads();
  for (int k = threadIdx.x; k < kTailBuckets; k += blockDim.x) {
    // records in larger buckets come first
    unsigned int pre = 0u;
    for (int q = kTailBuckets - 1; q > k; --q) pre += tb.btot[q];
    base[k] = pre + (h[k] ? atomicAdd(&tb.bcur[k], h[k]) : 0u);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kTailBuckets; k += blockDim.x) h[k] = 0u;
  __syncthreads();
  for (unsigned int r = lo + threadIdx.x; r < hi; r += blockDim.x) {
    const int k = tb.key[r];
    tb.order[base[k] + atomicAdd(&h[k], 1u)] = (int32_t)r;
  }
}

// Pool order.  Blocks claim work items in pool order, so cells that need
// many steps but sit late in the pool (a hot band in the middle of a field)
// start late, and cells that sit together land in a few blocks.  With
// ordering on, "heavy" cells are dealt round-robin over the first claim of
// every resident block (R claims of B items): claim c gets heavy items
// c, c + R, c + 2R, ... at its start and light items fill the rest, in pool
// order (runs of up to 64 consecutive cells stay together, so loads stay
// coalesced); everything after the first R*B positions keeps pool order.
// A cell is heavy when its step hint promises at least kHeavySteps steps
// over its flow step, or, without a usable hint (h <= 0 or h >= dt), when
// it is at least kHeavyT hot (below that the chemistry is slow).  The
// second order, by range, puts the cells below the mechanism's NASA-7 range
// switch first and the rest after them, each in pool order: the RHS
// evaluates one range's polynomials for a wave whose cells all sit in it
// and both for a wave that straddles the switch, so on a field with
// temperatures scattered around it (the stress fields) grouping by range
// spares most waves the second set.  Neither order changes a result: each
// cell's integration is independent of when and where it runs.  The dealt
// order is skipped (identity) when nothing is heavy, when heavy cells are
// more than half of the first round, or when the pool is smaller than one
// round.
constexpr double kHeavySteps = 8.0;
constexpr double kHeavyT = 1000.0;

constexpr int ORDER_DEAL = 1;    // heavy cells dealt over the first claims
constexpr int ORDER_RANGE = 2;   // cells below the NASA-7 range switch first
constexpr int ORDER_RANGE_DEFER = 3;  // as ORDER_RANGE; cells below the switch wait for the resumption

struct OrderBuf {
  int32_t* rank;          // per item: rank among class 0 (>= 0) or -(rank among class 1) - 1
  int32_t* order;         // pool position -> item
  unsigned int* counts;   // [0] class 0, [1] class 1 (zeroed before order_rank)
  int mode;               // ORDER_DEAL (class 0 = heavy) or ORDER_RANGE (class 0 = T < t_split)
  int defer;              // with ORDER_RANGE: class 0 is claimed after the resumption's records
  double t_split;
};

__global__ void order_reset(unsigned int* counts) {
  counts[0] = 0u;
  counts[1] = 0u;
}

// Classify every item and rank it within its class.  One 1024-lane block
// takes kOrderRounds * 1024 consecutive items: wave ballots count each
// class, one lane turns the per-wave counts into offsets in pool order and
// takes the block's two ranges with one atomic each, so the ranks keep pool
// order within the block and the counters see a few hundred atomics (one
// per wave would serialise tens of thousands on two addresses).
constexpr int kOrderRounds = 4;
constexpr int kOrderBlock = 1024;

__global__ __launch_bounds__(kOrderBlock) void order_rank(PoolArgs a, int ns, OrderBuf ob) {
  constexpr int W = kOrderBlock / 64;
  __shared__ unsigned int off_h[kOrderRounds][W], off_l[kOrderRounds][W];
  __shared__ unsigned int base_h, base_l;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t first = (int64_t)blockIdx.x * kOrderBlock * kOrderRounds;
  bool heavy[kOrderRounds];
  unsigned long long bh[kOrderRounds], bl[kOrderRounds];
  // the pool's size: fixed, or (a list built on the device) read here
  const int64_t total = a.total_dev ? (int64_t)*a.total_dev : a.total;
#pragma unroll
  for (int r = 0; r < kOrderRounds; ++r) {
    const int64_t g = first + (int64_t)r * kOrderBlock + threadIdx.x;
    const bool valid = g < total;
    heavy[r] = false;
    if (valid) {
      const BoxDesc& bd = box_ref(a, find_box(a, g));
      const int64_t i = cell_index(bd, g);
      const double T = bd.state[i];
      const double h = bd.state[(int64_t)(ns + 2) * bd.ld + i];
      if (ob.mode == ORDER_RANGE)
        heavy[r] = T < ob.t_split;
      else
        heavy[r] = (h > 0.0 && h < bd.dt) ? (double)bd.n_sub * bd.dt >= kHeavySteps * h
                                          : T >= kHeavyT;
    }
    bh[r] = __ballot(valid && heavy[r]);
    bl[r] = __ballot(valid && !heavy[r]);
    if (lane == 0) {
      off_h[r][wave] = (unsigned int)__popcll(bh[r]);
      off_l[r][wave] = (unsigned int)__popcll(bl[r]);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int th = 0u, tl = 0u;
    for (int r = 0; r < kOrderRounds; ++r)
      for (int w = 0; w < W; ++w) {
        const unsigned int xh = off_h[r][w], xl = off_l[r][w];
        off_h[r][w] = th;
        off_l[r][w] = tl;
        th += xh;
        tl += xl;
      }
    base_h = th ? atomicAdd(&ob.counts[0], th) : 0u;
    base_l = tl ? atomicAdd(&ob.counts[1], tl) : 0u;
  }
  __syncthreads();
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int r = 0; r < kOrderRounds; ++r) {
    const int64_t g = first + (int64_t)r * kOrderBlock + threadIdx.x;
    if (g >= total) continue;
    ob.rank[g] = heavy[r]
                     ? (int32_t)(base_h + off_h[r][wave] + (unsigned int)__popcll(bh[r] & below))
                     : -(int32_t)(base_l + off_l[r][wave] + (unsigned int)__popcll(bl[r] & below)) - 1;
  }
}

// Position of every item in the order (a bijection of [0, total)): by range,
// class 0 then class 1, each in pool order; dealt, as described above.
__global__ __launch_bounds__(256) void order_place(int64_t total, const unsigned int* total_dev,
                                                   int R, int B, OrderBuf ob) {
  if (total_dev) total = (int64_t)*total_dev;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int64_t H = ob.counts[0];
  if (ob.mode == ORDER_RANGE) {
    const int64_t r = ob.rank[g];
    const int64_t q = r >= 0 ? r : H + (-r - 1);
    if (q >= 0 && q < total) ob.order[q] = (int32_t)g;
    return;
  }
  const int64_t RB = (int64_t)R * B;
  int64_t q = g;
  if (H > 0 && 2 * H <= RB && total >= RB) {
    const int64_t r = ob.rank[g];
    const int64_t hq = H / R, hr = H % R;
    if (r >= 0) {
      q = (r % R) * B + r / R;
    } else {
      const int64_t p = -r - 1;
      const int64_t w1 = B - hq - 1, w0 = B - hq;  // light slots of claims c < hr, c >= hr
      if (p < hr * w1) {
        q = (p / w1) * B + hq + 1 + p % w1;
      } else if (p < RB - H) {
        const int64_t pp = p - hr * w1;
        q = (hr + pp / w0) * B + hq + pp % w0;
      } else {
        q = p + H;
      }
    }
  }
  if (q >= 0 && q < total) ob.order[q] = (int32_t)g;
}

template <class M, int LB, int S>
__global__ __launch_bounds__(LB) void lsrk_persistent(PoolArgs a) {
  constexpr int N1 = M::NS + 1;
  constexpr int ND = Slots<M>::ND;
  extern __shared__ double smem[];
  const int B = blockDim.x;
  const int tid = threadIdx.x;
  double* sd = smem;                                       // [ND][B]
  int* si = reinterpret_cast<int*>(smem + (size_t)ND * B);  // [6][B]
  __shared__ int s_active;
  __shared__ long long s_base;
  __shared__ int s_take;
  __shared__ int s_wave_cnt[16];

  // lane state
  int64_t item = -1;
  double u[N1], t = 0.0, h = 0.0, rho = 1.0;
  int nacc = 0, nrej = 0, sub = 0, base = 0;
  int bx = 0;
  int64_t total = a.total_dev ? (int64_t)*a.total_dev : a.total;
  // with deferred cells: dH of them, at positions [0, dH) of defer_order
  const int64_t pool_n = a.pool_dev ? (int64_t)*a.pool_dev : total;
  const int64_t dH = a.defer ? min((int64_t)*a.defer_h, pool_n) : 0;
  int64_t nrec = 0, off = 0;
  if (a.resume) {
    // resume the tail records when the cooperative kernel does not take
    // them, then step the deferred cells
    const unsigned int cnt = *a.tail.count;
    nrec = *a.tail.split < cnt ? (int64_t)cnt : 0;
    total = nrec + dH;
  } else if (a.defer) {
    off = dH;
    total = pool_n - dH;
  }
  const float prio = a.resume ? resume_priority(a.tail.btot, (float)gridDim.x * (float)B) : 0.f;

  // claim the first B items
  if (tid == 0) {
    const unsigned long long got = atomicAdd(a.next, (unsigned long long)B);
    s_base = (long long)got;
  }
  __syncthreads();
  int free_from = 0;  // lanes [free_from, B) need a fresh item
  for (;;) {
    // ---- refill lanes [free_from, B) from the pool base s_base
    if (tid >= free_from) {
      const int64_t g = s_base + (tid - free_from);
      item = -1;
      bool fresh = false;
      if (a.resume) {
        // a cell handed over at tail_steps, longest first: its state and
        // hint are in its rows, its progress in record r
        if (g < nrec) {
          const int r = a.tail.order[g];
          if (a.tail.rec) {
            using TR = TailRec<M>;
            const double* rc = a.tail.rec + (int64_t)r * TR::RD;
#pragma unroll
            for (int v = 0; v < N1; ++v) u[v] = rc[v];
            rho = rc[TR::RHO];
            h = rc[TR::H];
            t = rc[TR::T];
            const int* ri = reinterpret_cast<const int*>(rc + TR::INTS);
            item = ri[0]; nacc = ri[1]; nrej = ri[2]; sub = ri[3]; base = ri[4];
            bx = find_box(a, item);
          } else {
            item = a.tail.item[r];
            bx = find_box(a, item);
            const BoxDesc& bd = box_ref(a, bx);
            load_cell<M>(bd, cell_index(bd, item), u, rho, h);
            t = a.tail.t[r];
            nacc = a.tail.nacc[r]; nrej = a.tail.nrej[r];
            sub = a.tail.sub[r]; base = a.tail.base[r];
          }
        } else if (g < total) {
          // a deferred cell, not stepped yet
          item = a.defer_order[g - nrec];
          fresh = true;
          if (item < 0 || item >= pool_n) item = -1;
        }
      } else if (g < total) {
        item = a.order ? (int64_t)a.order[off + g] : off + g;
        if (item < 0 || item >= pool_n) item = -1;
      }
      if (item >= 0 && (!a.resume || fresh)) {
        bx = find_box(a, item);
        const BoxDesc& bd = box_ref(a, bx);
        const int64_t i = cell_index(bd, item);
        load_cell<M>(bd, i, u, rho, h);
        nacc = nrej = 0; sub = 0; base = 0; t = 0.0;
        if (!all_finite(u, rho)) {
          store_cell<M>(bd, i, u, h, CELL_NONFINITE, 0, 0);
          item = -1;
        } else if (a.fixed_steps > 0) {
          const double inv_rho = 1.0 / rho;
          for (int s = 0; s < bd.n_sub; ++s)
            advance_fixed<M, S>(u, rho, inv_rho, bd.dt, a.fixed_steps, h, nacc, a.c);
          nacc = a.fixed_steps * bd.n_sub;
          store_cell<M>(bd, i, u, h, CELL_OK, nacc, 0);
          item = -1;
        } else {
          h = initial_h(h, bd.dt);
        }
      }
    }
    // ---- priority levels at 1/1, 1/2, 1/4 of the threshold, from the
    // wave's largest estimate of remaining steps
    if (prio > 0.f) {
      float est = 0.f;
      if (item >= 0) {
        const BoxDesc& bd = box_ref(a, bx);
        est = (float)((bd.n_sub - sub) * bd.dt - t) * __builtin_amdgcn_rcpf((float)h);
      }
      if (__any(est >= prio)) __builtin_amdgcn_s_setprio(3);
      else if (__any(est >= 0.5f * prio)) __builtin_amdgcn_s_setprio(2);
      else if (__any(est >= 0.25f * prio)) __builtin_amdgcn_s_setprio(1);
      else __builtin_amdgcn_s_setprio(0);
    }
    // ---- run one chunk
    if (item >= 0) {
      const BoxDesc& bd = box_ref(a, bx);
      const double inv_rho = 1.0 / rho;
      int budget = a.chunk;
      // a cell stops exactly at tail_steps, whatever the chunk length, so
      // the hand-off point (and so the result) does not depend on tuning
      if (a.tail_steps > 0) budget = min(budget, a.tail_steps - (nacc + nrej));
      Control c = a.c;
      for (;;) {
        c.max_steps = base + a.c.max_steps;  // per sub-call step budget
        const int before = nacc + nrej;
        int st = advance<M, S>(u, rho, inv_rho, bd.dt, t, h, nacc, nrej, c, budget);
        budget -= (nacc + nrej) - before;
        if (st == CELL_RUNNING) break;
        if (st == CELL_OK && sub + 1 < bd.n_sub) {
          ++sub; t = 0.0; base = nacc + nrej;
          h = initial_h(h, bd.dt);
          if (budget > 0) continue;
          break;
        }
        store_cell<M>(bd, cell_index(bd, item), u, h, st, nacc, nrej);
        item = -1;
        break;
      }
      if (item >= 0 && a.tail_steps > 0 && nacc + nrej >= a.tail_steps) {
        // hand the cell over: state, hint and progress to a tail record (or
        // state and hint to its own rows, progress to the record's fields)
        const unsigned int r = atomicAdd(a.tail.count, 1u);
        if (a.tail.rec) {
          using TR = TailRec<M>;
          double* rc = a.tail.rec + (int64_t)r * TR::RD;
#pragma unroll
          for (int v = 0; v < N1; ++v) rc[v] = u[v];
          rc[TR::RHO] = rho;
          rc[TR::H] = h;
          rc[TR::T] = t;
          int* ri = reinterpret_cast<int*>(rc + TR::INTS);
          ri[0] = (int)item; ri[1] = nacc; ri[2] = nrej; ri[3] = sub; ri[4] = base;
        } else {
          const int64_t i = cell_index(bd, item);
          double* s = bd.state;
#pragma unroll
          for (int v = 0; v < N1; ++v) s[v * bd.ld + i] = u[v];
          s[(N1 + 1) * bd.ld + i] = h;
          a.tail.item[r] = (int32_t)item;
          a.tail.t[r] = t;
          a.tail.nacc[r] = nacc;
          a.tail.nrej[r] = nrej;
          a.tail.sub[r] = sub;
          a.tail.base[r] = base;
        }
        a.tail.key[r] = tail_key((bd.n_sub - sub) * bd.dt - t, h);
        item = -1;
      }
    }
    // ---- pack active lanes to the front through LDS
    const bool act = item >= 0;
    const unsigned long long ball = __ballot(act);
    const int lane = tid & 63, wave = tid >> 6, nw = (B + 63) >> 6;
    if (lane == 0) s_wave_cnt[wave] = __popcll(ball);
    __syncthreads();
    int off = 0, n_active = 0;
    for (int w = 0; w < nw; ++w) {
      const int cnt = s_wave_cnt[w];
      if (w < wave) off += cnt;
      n_active += cnt;
    }
    const int rank = off + __popcll(ball & ((1ull << lane) - 1ull));
    if (act) {
#pragma unroll
      for (int v = 0; v < N1; ++v) sd[(size_t)v * B + rank] = u[v];
      sd[(size_t)N1 * B + rank] = t;
      sd[(size_t)(N1 + 1) * B + rank] = h;
      sd[(size_t)(N1 + 2) * B + rank] = rho;
      si[0 * B + rank] = (int)item;
      si[1 * B + rank] = nacc;
      si[2 * B + rank] = nrej;
      si[3 * B + rank] = sub;
      si[4 * B + rank] = base;
      si[5 * B + rank] = bx;
    }
    if (tid == 0) {
      int take = 0;
      long long gbase = 0;
      const int want = B - n_active;
      if (want > 0) {
        const unsigned long long cur = __hip_atomic_load(a.next, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
        if ((int64_t)cur < total) {
          gbase = (long long)atomicAdd(a.next, (unsigned long long)want);
          take = want;
        }
      }
      s_base = gbase;
      s_take = take;
      s_active = n_active;
    }
    __syncthreads();
    const int A = s_active;
    if (tid < A) {
#pragma unroll
      for (int v = 0; v < N1; ++v) u[v] = sd[(size_t)v * B + tid];
      t = sd[(size_t)N1 * B + tid];
      h = sd[(size_t)(N1 + 1) * B + tid];
      rho = sd[(size_t)(N1 + 2) * B + tid];
      item = si[0 * B + tid];
      nacc = si[1 * B + tid];
      nrej = si[2 * B + tid];
      sub = si[3 * B + tid];
      base = si[4 * B + tid];
      bx = si[5 * B + tid];  // the box travels with the cell: no search
    } else {
      item = -1;
    }
    const int take = s_take;
    __syncthreads();  // LDS slots and s_* reused next round
    if (A == 0 && (take == 0 || s_base >= total)) break;
    free_from = take > 0 ? A : B;
  }
}

// ------------------------------------------- split-scheme coupling kernels
// Conserved rows (paper Sec. 2.2.1, the reaction part of the Strang split):
// rho, rho u, rho v, rho w, rho E, rho Y_1..rho Y_N, T, h.
constexpr int CELL_T_NEWTON = 4;

// Primitive state for the integrator: Y = rho Y / rho and T from
// e = E - |u|^2/2 by Newton on e(T, Y) (the T row is the initial guess,
// <= 0: 1000 K; |dT| <= 1e-12 T within 50 iterations).  A cell whose
// iteration fails gets T = NaN (the integrator leaves it alone) and flag 1.
template <class M>
__global__ void cons_to_prim(const double* __restrict__ cons, int64_t ld, int64_t n,
                             double* __restrict__ work, int8_t* __restrict__ flag) {
  constexpr int N = M::NS;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double rho = cons[i];
  const double mu = cons[ld + i], mv = cons[2 * ld + i], mw = cons[3 * ld + i];
  const double e_t = cons[4 * ld + i] / rho - 0.5 * (mu * mu + mv * mv + mw * mw) / (rho * rho);
  double Y[N];
#pragma unroll
  for (int k = 0; k < N; ++k) Y[k] = cons[(5 + k) * ld + i] / rho;
  double T = cons[(5 + N) * ld + i];
  T = T > 0.0 ? T : 1000.0;
  bool ok = false;
  for (int it = 0; it < 50; ++it) {
    double e, cv;
    M::energy_cv(T, Y, e, cv);
    const double dT = (e - e_t) / cv;
    T -= dT;
    if (!(T > 0.0) || !isfinite(T)) break;
    if (fabs(dT) <= 1e-12 * T) { ok = true; break; }
  }
  work[i] = ok ? T : __builtin_nan("");
#pragma unroll
  for (int k = 0; k < N; ++k) work[(1 + k) * n + i] = Y[k];
  work[(N + 1) * n + i] = rho;
  work[(N + 2) * n + i] = cons[(6 + N) * ld + i];
  flag[i] = ok ? 0 : 1;
}

// Write back rho Y_k, T and h; rho, momentum and rho E are unchanged.
template <class M>
__global__ void prim_to_cons(const double* __restrict__ work, const int8_t* __restrict__ flag,
                             int64_t n, double* __restrict__ cons, int64_t ld,
                             int32_t* __restrict__ status) {
  constexpr int N = M::NS;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (flag[i]) {
    if (status) status[i] = CELL_T_NEWTON;
    return;
  }
  const double rho = cons[i];
#pragma unroll
  for (int k = 0; k < N; ++k) cons[(5 + k) * ld + i] = rho * work[(1 + k) * n + i];
  cons[(5 + N) * ld + i] = work[i];
  cons[(6 + N) * ld + i] = work[(N + 2) * n + i];
}

}  // namespace

#include "surrogate_kernels.hip.h"
#include "surrogate_train.hip.h"

namespace {

// ------------------------------------------------------------- registry
struct MechEntry {
  unsigned long long hash;
  int ns, nr;
  const char* name;
  bool has_jac;  // a generated Jacobian: the Rosenbrock comparator is built
  double t_split;  // the NASA-7 range switch the RHS branches on (ORDER_RANGE)
  hipError_t (*launch_direct)(const PoolArgs&, int block, hipStream_t);
  hipError_t (*launch_persistent)(const PoolArgs&, int block, int grid, hipStream_t);
  hipError_t (*launch_coop)(const PoolArgs&, int n_cu, hipStream_t);
  hipError_t (*launch_cons_to_prim)(const double*, int64_t, int64_t, double*, int8_t*, hipStream_t);
  hipError_t (*launch_prim_to_cons)(const double*, const int8_t*, int64_t, double*, int64_t,
                                    int32_t*, hipStream_t);
  int (*max_blocks_per_cu)(int block, int scheme);
  size_t (*lds_per_lane)();
  hipError_t (*launch_surr_infer)(const surr::InferArgs&, int grid, hipStream_t);
  hipError_t (*launch_make_pairs)(const double*, const double*, long, long, double, const double*,
                                  float*, float*, hipStream_t);
  hipError_t (*launch_train)(const surr::TrainArgs&, int phase, hipStream_t);
  long train_wtpack_elems;  // the transposed packed weights of the training step
  int train_w4t_ld;
  long train_wt4, train_wt2;
  int tail_rd;  // doubles per tail record carrying the state (TailRec)
};

// Kernels are instantiated for launch bounds 256 (blocks of 64..256 threads)
// and 512; the bound caps the registers the compiler may give a lane.
template <class M, int S>
hipError_t launch_direct_s(const PoolArgs& a, int block, hipStream_t s) {
  const int64_t grid = (a.one.n + block - 1) / block;
  if (grid == 0) return hipSuccess;
  if constexpr (S == SCHEME_ROS4) {
    hipLaunchKernelGGL((lsrk_direct<M, 256, S>), dim3((unsigned)grid), dim3(block), 0, s, a);
  } else {
    if (block <= 256)
      hipLaunchKernelGGL((lsrk_direct<M, 256, S>), dim3((unsigned)grid), dim3(block), 0, s, a);
    else
      hipLaunchKernelGGL((lsrk_direct<M, 512, S>), dim3((unsigned)grid), dim3(block), 0, s, a);
  }
  return hipGetLastError();
}

// The Rosenbrock comparator holds its (N+1)^2 matrix in registers: it is
// built only for mechanisms with a generated Jacobian and only with the
// 256-lane launch bound (one wave per SIMD may use every register).
template <class M>
hipError_t launch_direct(const PoolArgs& a, int block, hipStream_t s) {
  if (a.scheme == SCHEME_ROS4) {
    if constexpr (M::HAS_JAC) {
      if (block > 256) return hipErrorInvalidConfiguration;
      return launch_direct_s<M, SCHEME_ROS4>(a, block, s);
    } else {
      return hipErrorInvalidValue;
    }
  }
  return a.scheme == SCHEME_RKF45 ? launch_direct_s<M, SCHEME_RKF45>(a, block, s)
                                  : launch_direct_s<M, SCHEME_LSRK>(a, block, s);
}

template <class M, int S>
hipError_t launch_persistent_s(const PoolArgs& a, int block, int grid, hipStream_t s) {
  if constexpr (S == SCHEME_ROS4) {
    hipLaunchKernelGGL((lsrk_persistent<M, 256, S>), dim3(grid), dim3(block),
                       Slots<M>::bytes(block), s, a);
  } else {
    if (block <= 256)
      hipLaunchKernelGGL((lsrk_persistent<M, 256, S>), dim3(grid), dim3(block),
                         Slots<M>::bytes(block), s, a);
    else
      hipLaunchKernelGGL((lsrk_persistent<M, 512, S>), dim3(grid), dim3(block),
                         Slots<M>::bytes(block), s, a);
  }
  return hipGetLastError();
}

template <class M>
hipError_t launch_persistent(const PoolArgs& a, int block, int grid, hipStream_t s) {
  // one lane per key-bucket counter (btot and bcur are adjacent)
  hipLaunchKernelGGL(pool_reset, dim3(1), dim3(2 * kTailBuckets), 0, s, a.next,
                     a.tail_steps > 0 ? a.tail.count : nullptr,
                     a.tail_steps > 0 ? a.tail.next : nullptr,
                     a.tail_steps > 0 ? a.tail.next2 : nullptr,
                     a.tail_steps > 0 ? a.tail.coop_steps : nullptr,
                     a.tail_steps > 0 ? a.tail.btot : nullptr);
  if (a.scheme == SCHEME_ROS4) {
    if constexpr (M::HAS_JAC) {
      if (block > 256) return hipErrorInvalidConfiguration;
      return launch_persistent_s<M, SCHEME_ROS4>(a, block, grid, s);
    } else {
      return hipErrorInvalidValue;
    }
  }
  return a.scheme == SCHEME_RKF45 ? launch_persistent_s<M, SCHEME_RKF45>(a, block, grid, s)
                                  : launch_persistent_s<M, SCHEME_LSRK>(a, block, grid, s);
}

template <class M>
hipError_t launch_cons_to_prim(const double* cons, int64_t ld, int64_t n, double* work,
                               int8_t* flag, hipStream_t s) {
  const int64_t grid = (n + 255) / 256;
  hipLaunchKernelGGL(cons_to_prim<M>, dim3((unsigned)grid), dim3(256), 0, s, cons, ld, n, work, flag);
  return hipGetLastError();
}

template <class M>
hipError_t launch_prim_to_cons(const double* work, const int8_t* flag, int64_t n, double* cons,
                               int64_t ld, int32_t* status, hipStream_t s) {
  const int64_t grid = (n + 255) / 256;
  hipLaunchKernelGGL(prim_to_cons<M>, dim3((unsigned)grid), dim3(256), 0, s, work, flag, n, cons,
                     ld, status);
  return hipGetLastError();
}

template <class M, int S>
int max_blocks_per_cu_s(int block) {
  int nb = 0;
  hipError_t e;
  if constexpr (S == SCHEME_ROS4) {
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lsrk_persistent<M, 256, S>, block,
                                                     Slots<M>::bytes(block));
  } else {
    if (block <= 256)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lsrk_persistent<M, 256, S>, block,
                                                       Slots<M>::bytes(block));
    else
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lsrk_persistent<M, 512, S>, block,
                                                       Slots<M>::bytes(block));
  }
  if (e != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

template <class M>
int max_blocks_per_cu(int block, int scheme) {
  if (scheme == SCHEME_ROS4) {
    if constexpr (M::HAS_JAC) return max_blocks_per_cu_s<M, SCHEME_ROS4>(block);
    else return 1;
  }
  return scheme == SCHEME_RKF45 ? max_blocks_per_cu_s<M, SCHEME_RKF45>(block)
                                : max_blocks_per_cu_s<M, SCHEME_LSRK>(block);
}

template <class M>
size_t lds_per_lane() {
  return Slots<M>::bytes(1);
}

#define CHEM_ENTRY(M) {M::HASH, M::NS, M::NR, M::NAME, M::HAS_JAC, M::T_SPLIT, \
                       &launch_direct<M>, &launch_persistent<M>, \
                       &launch_coop<M>, &launch_cons_to_prim<M>, &launch_prim_to_cons<M>, \
                       &max_blocks_per_cu<M>, &lds_per_lane<M>, \
                       &launch_surr_infer<M>, &launch_make_pairs<M>, &launch_train<M>, \
                       TrainSizes<M>::wtpack_elems, TrainSizes<M>::w4t_ld, TrainSizes<M>::wt4, \
                       TrainSizes<M>::wt2, TailRec<M>::RD},
const MechEntry g_registry[] = {CHEM_FOR_EACH_MECH(CHEM_ENTRY)};
#undef CHEM_ENTRY

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(CHEM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

uint64_t fnv1a64(const std::vector<char>& d) {
  uint64_t h = 0xCBF29CE484222325ull;
  for (char c : d) { h ^= (unsigned char)c; h *= 0x100000001B3ull; }
  return h;
}

}  // namespace

// Device storage of the tail records (see TailBuf): one allocation holding
// cap records and the two counters.
struct TailStore {
  void* mem = nullptr;
  int64_t cap = 0;
  int rd = 0;  // doubles per record carrying the state (TailRec<M>::RD), or 0
  // [next u64][count u32][split u32][next2 u64][coop_steps u64]
  // [btot, bcur: kTailBuckets u32 each][pad to 768 bytes], then
  // rd > 0: [rec: cap records of rd doubles][key, order: cap int32 each]
  // rd = 0: [t: cap doubles][item, nacc, nrej, sub, base, key, order: cap int32 each]
  static constexpr size_t kHead = 768;
  static_assert(32 + 2 * kTailBuckets * sizeof(unsigned int) <= kHead, "tail head");
  TailBuf view() const {
    TailBuf b{};
    char* p = static_cast<char*>(mem);
    b.next = reinterpret_cast<unsigned long long*>(p);
    b.count = reinterpret_cast<unsigned int*>(p + 8);
    b.split = reinterpret_cast<unsigned int*>(p + 12);
    b.next2 = reinterpret_cast<unsigned long long*>(p + 16);
    b.coop_steps = reinterpret_cast<unsigned long long*>(p + 24);
    b.btot = reinterpret_cast<unsigned int*>(p + 32);
    b.bcur = b.btot + kTailBuckets;
    if (rd > 0) {
      b.rec = reinterpret_cast<double*>(p + kHead);
      int32_t* q = reinterpret_cast<int32_t*>(p + kHead + sizeof(double) * rd * cap);
      b.key = q; b.order = q + cap;
      return b;
    }
    b.t = reinterpret_cast<double*>(p + kHead);
    int32_t* q = reinterpret_cast<int32_t*>(p + kHead + sizeof(double) * cap);
    b.item = q; b.nacc = q + cap; b.nrej = q + 2 * cap; b.sub = q + 3 * cap; b.base = q + 4 * cap;
    b.key = q + 5 * cap; b.order = q + 6 * cap;
    return b;
  }
  static constexpr size_t bytes(int64_t cap, int rd = 0) {
    return rd > 0 ? kHead + (size_t)cap * (sizeof(double) * rd + 2 * sizeof(int32_t))
                  : kHead + (size_t)cap * (sizeof(double) + 7 * sizeof(int32_t));
  }
};

// Device storage of the pool order (see OrderBuf): rank and order arrays of
// cap entries and the two class counters, one allocation.
struct OrderStore {
  void* mem = nullptr;
  int64_t cap = 0;
  OrderBuf view() const {
    OrderBuf b{};
    char* p = static_cast<char*>(mem);
    b.counts = reinterpret_cast<unsigned int*>(p);
    b.rank = reinterpret_cast<int32_t*>(p + 16);
    b.order = b.rank + cap;
    return b;
  }
  static constexpr size_t bytes(int64_t cap) { return 16 + (size_t)cap * 2 * sizeof(int32_t); }
};

// Batched calls stage their box table through a ring of slots (pinned host
// copy + device copy, kMaxBoxes entries each); a slot is reused once the call
// that last used it has finished on the device, so a host wait happens only
// when kBoxRing batched calls are still queued.
constexpr int kMaxBoxes = 4096;
constexpr int kBoxRing = 4;

namespace {

// Scratch memory of chem_integrate_noalloc: the pool counter, the tail
// records and the pool order of one call on up to kNoAllocMaxCells cells, in
// a fixed device array (one copy per GPU, held until the process ends).
// Host code never passes `scratch` itself to a kernel or a copy: the array's
// device address comes from hipGetSymbolAddress, once per device, at the
// first chem_mech_load on that device (g_scratch_ptr).
constexpr int64_t kNoAllocMaxCells = int64_t(1) << 20;
constexpr size_t round256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t kScratchTailOff = 256;
constexpr size_t kScratchOrderOff = kScratchTailOff + round256(TailStore::bytes(kNoAllocMaxCells));
constexpr size_t kScratchBytes = kScratchOrderOff + round256(OrderStore::bytes(kNoAllocMaxCells));

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

struct chem_mech_s {
  const MechEntry* entry;
  TailStore tail;
  OrderStore order;
  struct Tuned { int block, chunk, tail, cap, order; };
  std::map<int, Tuned> tuned;  // (size bucket, scheme) -> tuned launch
  // workspace, all of it allocated by chem_workspace_reserve
  unsigned long long* d_next = nullptr;
  BoxDesc* d_boxes = nullptr;      // kBoxRing slots of kMaxBoxes entries
  BoxDesc* h_boxes = nullptr;      // pinned staging, same shape
  hipEvent_t box_done[kBoxRing] = {};
  int box_slot = 0;
  int64_t reserved = 0;
  bool fixed_ready = false;        // pool counter, box ring and events allocated
  double* d_prim = nullptr;        // primitive work state of chem_react_conserved
  int8_t* d_flag = nullptr;
  int device = 0;
  int n_cu = 0;
  void* scratch = nullptr;         // this device's copy of `scratch` (chem_integrate_noalloc)
  // optional per-kernel timing of plain (not captured) calls: events around
  // the persistent launch, the tail sort, the cooperative launch and the
  // resumption launch of the last call
  bool timing = false;
  bool timed_last = false;
  hipEvent_t tev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  const TailStore* timed_tail = nullptr;  // the tail records of the last timed call
};

struct chem_graph_s {
  TailStore tail;
  OrderStore order;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  BoxDesc* d_boxes = nullptr;
  unsigned long long* d_next = nullptr;
  int32_t* fb_list = nullptr;    // a captured surrogate step's fallback list
  unsigned* fb_count = nullptr;  // and its length
};

namespace {

// Tail records of a workspace or a captured graph: the state travels with
// each record (rd doubles, the mechanism's TailRec size).
int alloc_tail(TailStore& ts, int64_t cap, int rd) {
  ts.mem = nullptr;
  ts.cap = 0;
  ts.rd = 0;
  hipError_t e = hipMalloc(&ts.mem, TailStore::bytes(cap, rd));
  if (e != hipSuccess) { ts.mem = nullptr; return hip_fail(e, "hipMalloc(tail records)"); }
  ts.cap = cap;
  ts.rd = rd;
  return CHEM_OK;
}

int alloc_order(OrderStore& os, int64_t cap) {
  os.mem = nullptr;
  os.cap = 0;
  hipError_t e = hipMalloc(&os.mem, OrderStore::bytes(cap));
  if (e != hipSuccess) { os.mem = nullptr; return hip_fail(e, "hipMalloc(pool order)"); }
  os.cap = cap;
  return CHEM_OK;
}

// The per-cell part of a mechanism's workspace (tail records, pool order,
// primitive work state); teardown and reservation only.
void free_cell_workspace(chem_mech m) {
  if (m->tail.mem) (void)hipFree(m->tail.mem);
  if (m->order.mem) (void)hipFree(m->order.mem);
  if (m->d_prim) (void)hipFree(m->d_prim);
  if (m->d_flag) (void)hipFree(m->d_flag);
  m->tail = TailStore{};
  m->order = OrderStore{};
  m->d_prim = nullptr;
  m->d_flag = nullptr;
  m->reserved = 0;
}

// Pool counter, box-table ring and its events: sized independently of the
// cell count.
int alloc_fixed_workspace(chem_mech m) {
  if (m->fixed_ready) return CHEM_OK;
  hipError_t e = hipMalloc(&m->d_next, sizeof(unsigned long long));
  if (e != hipSuccess) { m->d_next = nullptr; return hip_fail(e, "hipMalloc(pool counter)"); }
  e = hipMalloc(&m->d_boxes, sizeof(BoxDesc) * kMaxBoxes * kBoxRing);
  if (e != hipSuccess) { m->d_boxes = nullptr; return hip_fail(e, "hipMalloc(box table)"); }
  e = hipHostMalloc(&m->h_boxes, sizeof(BoxDesc) * kMaxBoxes * kBoxRing, hipHostMallocDefault);
  if (e != hipSuccess) { m->h_boxes = nullptr; return hip_fail(e, "hipHostMalloc(box table)"); }
  for (hipEvent_t& ev : m->box_done) {
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) { ev = nullptr; return hip_fail(e, "hipEventCreate(box table)"); }
  }
  m->fixed_ready = true;
  return CHEM_OK;
}

// Calls that use the mechanism's own workspace need a reservation covering
// their cells (and, for batched calls, at most kMaxBoxes boxes).
int check_capacity(chem_mech m, int64_t cells, const char* where) {
  if (m->fixed_ready && cells <= m->reserved) return CHEM_OK;
  char msg[200];
  snprintf(msg, sizeof msg, "%s: %lld cells but the workspace is reserved for %lld "
           "(call chem_workspace_reserve first)", where, (long long)cells,
           (long long)(m->fixed_ready ? m->reserved : 0));
  return fail(CHEM_ECAPACITY, msg);
}

Control make_control(const chem_opts* o) {
  Control c;
  c.rtol = (o && o->rtol > 0) ? o->rtol : 1e-8;
  c.atol = (o && o->atol > 0) ? o->atol : 1e-10;
  c.max_steps = (o && o->max_steps > 0) ? o->max_steps : 100000;
  return c;
}

int check_opts(const chem_opts* o) {
  if (!o) return CHEM_OK;
  if (!(o->rtol >= 0) || !(o->atol >= 0) || o->max_steps < 0 || o->fixed_steps < 0)
    return fail(CHEM_EINVAL, "chem_opts: negative or NaN field");
  if (o->scheme != SCHEME_LSRK && o->scheme != SCHEME_RKF45 && o->scheme != SCHEME_ROS4)
    return fail(CHEM_EINVAL,
                "chem_opts.scheme must be 0 (LSRK4(3)5), 1 (RKF45) or 2 (Rosenbrock)");
  if (o->pool_order > 3)
    return fail(CHEM_EINVAL, "chem_opts.pool_order must be <= 0 (off or tuned), 1, 2 or 3");
  if (o->block_size != 0 && (o->block_size % 64 != 0 || o->block_size > 512 || o->block_size < 64))
    return fail(CHEM_EINVAL, "chem_opts.block_size must be a multiple of 64 in [64, 512]");
  return CHEM_OK;
}

// The Rosenbrock comparator needs a generated Jacobian and the 256-lane
// launch bound.
int check_scheme_launch(chem_mech m, const chem_opts* o, int block) {
  if (!o || o->scheme != SCHEME_ROS4) return CHEM_OK;
  if (!m->entry->has_jac)
    return fail(CHEM_EUNSUPPORTED, "no Rosenbrock kernel for this mechanism (more than 15 species)");
  if (block > 256) return fail(CHEM_EINVAL, "the Rosenbrock scheme runs with block_size <= 256");
  return CHEM_OK;
}

constexpr int kDefaultBlock = 128;
constexpr int kDefaultChunk = 8;
constexpr int kDefaultTail = 32;

int size_bucket(int64_t total) {
  int b = 0;
  while (b < 62 && (int64_t(1) << b) < total) ++b;
  return b;
}

// Tuned launches are kept per (size bucket, scheme).
int tuned_key(int64_t total, const chem_opts* o) {
  return size_bucket(total) * 4 + (o ? o->scheme : SCHEME_LSRK);
}

int pick_tail(chem_mech m, int64_t total, const chem_opts* o) {
  if (o && o->fixed_steps > 0) return 0;
  if (o && o->scheme != SCHEME_LSRK) return 0;  // the cooperative kernel runs the LSRK scheme
  int t = o ? o->tail_steps : 0;
  if (t == 0) {
    auto it = m->tuned.find(tuned_key(total, o));
    t = (it != m->tuned.end() && it->second.tail != 0) ? it->second.tail : kDefaultTail;
  }
  return t > 0 ? t : 0;
}

constexpr int kDefaultTailCap = 64;

// Most handed-over cells the cooperative kernel takes, over the whole chip.
// Pool order: ORDER_DEAL or ORDER_RANGE (chem_opts.pool_order 1 or 2), off
// (< 0), else the tuned choice, else off.  Returns 0 for off.
int pick_order(chem_mech m, int64_t total, const chem_opts* o) {
  int v = o ? o->pool_order : 0;
  if (v == 0) {
    auto it = m->tuned.find(tuned_key(total, o));
    v = it != m->tuned.end() ? it->second.order : 0;
  }
  return v == ORDER_DEAL || v == ORDER_RANGE || v == ORDER_RANGE_DEFER ? v : 0;
}

int pick_cap(chem_mech m, int64_t total, const chem_opts* o) {
  int c = o ? o->tail_cap : 0;
  if (c == 0) {
    auto it = m->tuned.find(tuned_key(total, o));
    c = (it != m->tuned.end() && it->second.cap != 0) ? it->second.cap : kDefaultTailCap;
  }
  if (c < 0) return INT32_MAX;
  return (int)std::min<int64_t>((int64_t)c * m->n_cu, INT32_MAX);
}

void pick_launch(chem_mech m, int64_t total, const chem_opts* o, int* block, int* chunk) {
  *block = (o && o->block_size) ? o->block_size : 0;
  *chunk = (o && o->chunk_steps) ? o->chunk_steps : 0;
  auto it = m->tuned.find(tuned_key(total, o));
  if (it != m->tuned.end()) {
    if (!*block) *block = it->second.block;
    if (!*chunk) *chunk = it->second.chunk;
  }
  if (!*block) *block = kDefaultBlock;
  if (!*chunk) *chunk = kDefaultChunk;
}

int grid_for(chem_mech m, int block, int64_t total, int scheme);

// The flow step's launches: pool reset + persistent kernel, then, with a
// hand-off point, the tail sort, the cooperative kernel and the per-lane
// resumption of the list (exactly one of the last two does work, chosen by
// the list's length against a.tail.cap).  Timed calls record m->tev: [0]
// before the persistent kernel, [1] after it, [2] after the tail sort, [3]
// after the cooperative kernel, [4] after the resumption.
hipError_t launch_step(chem_mech m, PoolArgs& a, int block, int grid, hipStream_t s,
                       const OrderBuf* ob, bool timed = false) {
  hipError_t e;
  a.order = nullptr;
  a.defer = 0;
  hipEvent_t* tv = timed ? m->tev : nullptr;
  if (ob && a.total > 0 && !a.resume) {
    // the pool order (for a pool whose size is counted on the device, the
    // kernels are sized by a.total, its upper bound, and read the count):
    // R = the resident blocks (the grid), B = block
    const int64_t per = (int64_t)kOrderBlock * kOrderRounds;
    const unsigned rg = (unsigned)((a.total + per - 1) / per);
    const unsigned og = (unsigned)((a.total + 255) / 256);
    hipLaunchKernelGGL(order_reset, dim3(1), dim3(1), 0, s, ob->counts);
    hipLaunchKernelGGL(order_rank, dim3(rg), dim3(kOrderBlock), 0, s, a, m->entry->ns, *ob);
    hipLaunchKernelGGL(order_place, dim3(og), dim3(256), 0, s, a.total, a.total_dev, grid, block,
                       *ob);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    a.order = ob->order;
    if (ob->defer && a.tail_steps > 0) {
      a.defer = 1;
      a.defer_h = ob->counts;
      a.defer_order = ob->order;
    }
  }
  if (tv && (e = hipEventRecord(tv[0], s)) != hipSuccess) return e;
  e = m->entry->launch_persistent(a, block, grid, s);
  if (e != hipSuccess) return e;
  if (tv && (e = hipEventRecord(tv[1], s)) != hipSuccess) return e;
  if (a.tail_steps <= 0) {
    // no tail: the remaining intervals are empty
    for (int k = 2; tv && k < 5; ++k)
      if ((e = hipEventRecord(tv[k], s)) != hipSuccess) return e;
    return hipSuccess;
  }
  {
    // the records number at most a.total (a cell is handed over once)
    const int64_t sg = (a.total + 4 * kSortBlock - 1) / (4 * kSortBlock);
    const unsigned sgrid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(sg, kSortGridMax));
    hipLaunchKernelGGL(tail_count, dim3(sgrid), dim3(kSortBlock), 0, s, a.tail);
    hipLaunchKernelGGL(tail_scatter, dim3(sgrid), dim3(kSortBlock), 0, s, a.tail);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (tv && (e = hipEventRecord(tv[2], s)) != hipSuccess) return e;
  e = m->entry->launch_coop(a, m->n_cu, s);
  if (e != hipSuccess) return e;
  if (tv && (e = hipEventRecord(tv[3], s)) != hipSuccess) return e;
  PoolArgs r = a;
  r.pool_dev = a.total_dev;
  r.resume = 1;
  r.tail_steps = 0;
  r.next = a.tail.next2;
  r.total_dev = nullptr;
  r.order = nullptr;
  e = m->entry->launch_persistent(r, block, grid, s);
  if (e != hipSuccess) return e;
  if (tv && (e = hipEventRecord(tv[4], s)) != hipSuccess) return e;
  return hipSuccess;
}

// The integrator over a work pool with a given pool counter and tail store
// (calls that may run concurrently on one mechanism each bring their own).
int run_pool_with(chem_mech m, PoolArgs& a, const chem_opts* o, hipStream_t s,
                  unsigned long long* next, TailStore& tail, OrderStore* order, bool timed) {
  int block, chunk;
  pick_launch(m, a.total, o, &block, &chunk);
  if (m->entry->lds_per_lane() * block > 65536)
    return fail(CHEM_EINVAL, "block_size too large for this mechanism's LDS compaction slots");
  if (a.total > 0x7fffffff) return fail(CHEM_EINVAL, "more than 2^31-1 work items in one call");
  int rc0 = check_scheme_launch(m, o, block);
  if (rc0) return rc0;
  a.next = next;
  a.chunk = chunk > 0 ? chunk : kDefaultChunk;
  a.tail_steps = pick_tail(m, a.total, o);
  if (a.tail_steps > 0) {
    if (!tail.mem || a.total > tail.cap)
      return fail(CHEM_ECAPACITY, "more cells than the reserved tail records");
    a.tail = tail.view();
    a.tail.cap = pick_cap(m, a.total, o);
  }
  OrderBuf ob{};
  const int omode = order ? pick_order(m, a.total, o) : 0;
  const bool ordered = omode != 0;
  if (ordered) {
    if (!order->mem || a.total > order->cap)
      return fail(CHEM_ECAPACITY, "more cells than the reserved pool order");
    ob = order->view();
    ob.mode = omode == ORDER_RANGE_DEFER ? ORDER_RANGE : omode;
    ob.defer = omode == ORDER_RANGE_DEFER;
    ob.t_split = m->entry->t_split;
  }
  timed = timed && m->timing;
  hipError_t e = launch_step(m, a, block, grid_for(m, block, a.total, a.scheme), s,
                             ordered ? &ob : nullptr, timed);
  if (e != hipSuccess) return hip_fail(e, "launch integrator kernels");
  if (timed) {
    m->timed_last = true;
    m->timed_tail = a.tail_steps > 0 ? &tail : nullptr;
  }
  return CHEM_OK;
}

int run_pool(chem_mech m, PoolArgs& a, const chem_opts* o, hipStream_t s) {
  int rc = check_capacity(m, a.total, "integrator");
  if (rc) return rc;
  return run_pool_with(m, a, o, s, m->d_next, m->tail, &m->order, true);
}

int grid_for(chem_mech m, int block, int64_t total, int scheme) {
  const int per_cu = m->entry->max_blocks_per_cu(block, scheme);
  const int64_t need = (total + block - 1) / block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)per_cu * m->n_cu));
}

// Validate boxes and lay them out as one pool: boxes with more sub-calls
// first (they carry the most work per cell), empty boxes dropped.
int build_table(const chem_box* boxes, int32_t n, std::vector<BoxDesc>& out, int64_t* total) {
  if (n < 0 || (n > 0 && !boxes)) return fail(CHEM_EINVAL, "bad box list");
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return boxes[x].n_sub > boxes[y].n_sub; });
  out.clear();
  int64_t start = 0;
  for (int k = 0; k < n; ++k) {
    const chem_box& b = boxes[order[k]];
    if (b.n_cells < 0 || b.ld < b.n_cells) return fail(CHEM_EINVAL, "box: need 0 <= n_cells <= ld");
    if (!(b.dt > 0) || !std::isfinite(b.dt)) return fail(CHEM_EINVAL, "box: dt must be finite and > 0");
    if (b.n_sub < 1) return fail(CHEM_EINVAL, "box: n_sub must be >= 1");
    if (b.n_cells == 0) continue;
    if (!b.state) return fail(CHEM_EINVAL, "box: null state");
    out.push_back(BoxDesc{b.state, b.ld, b.n_cells, start, b.dt, b.n_sub, 0, b.status, b.counts,
                          nullptr});
    start += b.n_cells;
  }
  *total = start;
  return CHEM_OK;
}

std::string arch_name(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

struct TuneEntry { std::string key; int block, chunk, tail, cap, order; double ms; };

std::vector<TuneEntry> read_cache(const char* path) {
  std::vector<TuneEntry> v;
  FILE* f = fopen(path, "rb");
  if (!f) return v;
  std::string txt;
  char buf[4096];
  size_t k;
  while ((k = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, k);
  fclose(f);
  size_t pos = 0;
  const std::string tag = "\"key\": \"";
  while ((pos = txt.find(tag, pos)) != std::string::npos) {
    pos += tag.size();
    const size_t end = txt.find('"', pos);
    if (end == std::string::npos) break;
    TuneEntry e{txt.substr(pos, end - pos), 0, 0, 0, 0, 0, 0.0};
    const size_t close = txt.find('}', end);
    const std::string rec = txt.substr(end, close == std::string::npos ? std::string::npos : close - end);
    const size_t pb = rec.find("\"block\":"), pc = rec.find("\"chunk\":"), pm = rec.find("\"ms\":");
    const size_t pt = rec.find("\"tail\":"), pk = rec.find("\"cap\":");
    const size_t po = rec.find("\"order\":");
    if (pb != std::string::npos) e.block = atoi(rec.c_str() + pb + 8);
    if (pc != std::string::npos) e.chunk = atoi(rec.c_str() + pc + 8);
    if (pt != std::string::npos) e.tail = atoi(rec.c_str() + pt + 7);
    if (pk != std::string::npos) e.cap = atoi(rec.c_str() + pk + 6);
    if (po != std::string::npos) e.order = atoi(rec.c_str() + po + 8);
    if (pm != std::string::npos) e.ms = atof(rec.c_str() + pm + 5);
    if (e.block > 0 && e.chunk != 0) v.push_back(e);
    pos = end;
  }
  return v;
}

int write_cache(const char* path, const std::vector<TuneEntry>& v) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "wb");
  if (!f) return fail(CHEM_EINVAL, std::string("cannot write ") + path);
  fprintf(f, "{\"version\": 1, \"entries\": [\n");
  for (size_t i = 0; i < v.size(); ++i)
    fprintf(f,
            "  {\"key\": \"%s\", \"block\": %d, \"chunk\": %d, \"tail\": %d, \"cap\": %d, "
            "\"order\": %d, \"ms\": %.6f}%s\n",
            v[i].key.c_str(), v[i].block, v[i].chunk, v[i].tail, v[i].cap, v[i].order, v[i].ms,
            i + 1 < v.size() ? "," : "");
  fprintf(f, "]}\n");
  fclose(f);
  if (rename(tmp.c_str(), path) != 0) return fail(CHEM_EINVAL, std::string("cannot replace ") + path);
  return CHEM_OK;
}

// The launch search shared by chem_autotune and surrogate_autotune.
// time_one(t, &ms) runs one call with launch t (from the caller's pristine
// data) and times it.  Fills the best launch of the search into `best`
// (launch fields only) and its median time into *best_ms.
using TimeOne = std::function<int(const chem_opts&, float*)>;

int tune_search(chem_mech m, const chem_opts& o, int reps, const TimeOne& time_one,
                chem_opts* best, double* best_ms_out) {
  int rc;
  // median time of `reps` calls of one configuration (after one untimed call)
  auto trial = [&](const chem_opts& t, double* med) -> int {
    std::vector<float> ms;
    for (int r = 0; r <= reps; ++r) {
      float el = 0;
      const int trc = time_one(t, &el);
      if (trc != CHEM_OK) return trc;
      if (r > 0) ms.push_back(el);
    }
    std::sort(ms.begin(), ms.end());
    *med = ms[ms.size() / 2];
    return CHEM_OK;
  };
  // Coordinate descent: chunk at the default block, block at the best
  // chunk, chunk again at the best block, then the hand-off point for the
  // best pair, then hand-off point and cooperative cap together (an early
  // hand-off only pays when the cap lets the cooperative kernel take the
  // longer list), then the two pool orders, then block and chunk once more
  // at the final hand-off, cap and order.  Each sweep keeps the incumbent
  // unless a candidate is faster.  Then the fastest few launches seen are
  // timed again, round-robin and with more calls each, so that one noisy
  // trial (a clock ramp, other work on the device) does not decide, and the
  // winner is refined against its one-step neighbours the same way.
  const int blocks[] = {64, 128, 192, 256, 384, 512};
  const int chunks[] = {1, 2, 4, 8, 16, 32, 64};
  const int tails[] = {4, 8, 16, 32, 64, 128, 256, 512, -1};
  const int pair_tails[] = {4, 8, 16, 32, 64};
  // below this many ms per call the (block, chunk) plane is swept whole
  constexpr double kTuneGridMs = 50.0;
  struct Seen { int b, c, tl, cap, ord; double ms; };
  std::vector<Seen> seen;
  const int caps[] = {kDefaultTailCap, 128, 256, -1};
  double best_ms = 1e300;
  int best_block = kDefaultBlock, best_chunk = kDefaultChunk;
  int best_tail = o.tail_steps != 0 ? o.tail_steps : kDefaultTail;
  int best_cap = o.tail_cap != 0 ? o.tail_cap : kDefaultTailCap;
  int best_order = o.pool_order != 0 ? o.pool_order : -1;
  const bool tune_tail = o.tail_steps == 0 && o.fixed_steps == 0 && o.scheme == SCHEME_LSRK;
  const bool tune_cap = tune_tail && o.tail_cap == 0;
  auto consider = [&](int b, int c, int tl, int cap, int ord) -> int {
    if (m->entry->lds_per_lane() * b > 65536) return CHEM_OK;
    if (o.scheme == SCHEME_ROS4 && b > 256) return CHEM_OK;
    chem_opts t = o;
    t.block_size = b;
    t.chunk_steps = c;
    t.tail_steps = tl;
    t.tail_cap = cap;
    t.pool_order = ord;
    double med = 0;
    const int trc = trial(t, &med);
    if (trc != CHEM_OK) return trc;
    seen.push_back({b, c, tl, cap, ord, med});
    if (med < best_ms) {
      best_ms = med; best_block = b; best_chunk = c; best_tail = tl; best_cap = cap;
      best_order = ord;
    }
    return CHEM_OK;
  };
  rc = CHEM_OK;
  const int o0 = best_order;
  {
    // untimed calls first: the first launches after start-up run slow
    // (clocks ramping), which would penalise whichever candidate comes first
    chem_opts t = o;
    t.block_size = best_block; t.chunk_steps = chunks[0]; t.tail_steps = best_tail;
    t.tail_cap = best_cap; t.pool_order = o0;
    for (int w = 0; w < 2 * reps + 2 && rc == CHEM_OK; ++w) {
      float el = 0;
      rc = time_one(t, &el);
    }
  }
  for (int c : chunks)
    if (rc == CHEM_OK) rc = consider(best_block, c, best_tail, best_cap, o0);
  if (rc == CHEM_OK && best_ms < kTuneGridMs) {
    // cheap calls: every (block, chunk) pair (coordinate descent can stop
    // in a local optimum: a block that loses at one chunk may win at another)
    const int b0 = best_block;  // its chunks were just timed
    for (int b : blocks)
      for (int c : chunks)
        if (rc == CHEM_OK && b != b0) rc = consider(b, c, best_tail, best_cap, o0);
  } else {
    for (int b : blocks)
      if (rc == CHEM_OK && b != best_block) rc = consider(b, best_chunk, best_tail, best_cap, o0);
    const int b0 = best_block;
    for (int c : chunks)
      if (rc == CHEM_OK && c != best_chunk) rc = consider(b0, c, best_tail, best_cap, o0);
  }
  if (tune_tail) {
    const int b0 = best_block, c0 = best_chunk, t0 = best_tail;
    for (int tl : tails)
      if (rc == CHEM_OK && tl != t0) rc = consider(b0, c0, tl, best_cap, o0);
  }
  if (tune_cap) {
    const int b0 = best_block, c0 = best_chunk, t0 = best_tail, k0 = best_cap;
    for (int tl : pair_tails)
      for (int cap : caps)
        if (rc == CHEM_OK && !(tl == t0 && cap == k0)) rc = consider(b0, c0, tl, cap, o0);
  }
  if (o.pool_order == 0 && o.fixed_steps == 0) {
    // the three pool orders at the best launch so far
    if (rc == CHEM_OK) rc = consider(best_block, best_chunk, best_tail, best_cap, ORDER_DEAL);
    if (rc == CHEM_OK) rc = consider(best_block, best_chunk, best_tail, best_cap, ORDER_RANGE);
    if (rc == CHEM_OK && best_tail > 0)
      rc = consider(best_block, best_chunk, best_tail, best_cap, ORDER_RANGE_DEFER);
  }
  {
    // the hand-off, the cap and the order move the balance between
    // compaction and the tail (the first sweeps ran at the default hand-off,
    // where a long tail list may go to the per-lane resumption), so block
    // and chunk are swept once more at the final choice: the whole plane
    // for cheap calls, else chunk, block, chunk
    const int t0 = best_tail, k0 = best_cap, ob0 = best_order;
    if (best_ms < kTuneGridMs) {
      const int b1 = best_block, c1 = best_chunk;
      for (int b : blocks)
        for (int c : chunks)
          if (rc == CHEM_OK && !(b == b1 && c == c1)) rc = consider(b, c, t0, k0, ob0);
    } else {
      const int b1 = best_block, c1 = best_chunk;
      for (int c : chunks)
        if (rc == CHEM_OK && c != c1) rc = consider(b1, c, t0, k0, ob0);
      const int c2 = best_chunk, b2 = best_block;
      for (int b : blocks)
        if (rc == CHEM_OK && b != b2) rc = consider(b, c2, t0, k0, ob0);
      const int b3 = best_block, c3 = best_chunk;
      for (int c : chunks)
        if (rc == CHEM_OK && c != c3) rc = consider(b3, c, t0, k0, ob0);
    }
  }
  if (rc == CHEM_OK && seen.size() > 1) {
    // confirmation round over the (up to) eight fastest distinct launches
    std::stable_sort(seen.begin(), seen.end(),
                     [](const Seen& x, const Seen& y) { return x.ms < y.ms; });
    std::vector<Seen> top;
    for (const Seen& v : seen) {
      bool dup = false;
      for (const Seen& w : top)
        dup = dup || (w.b == v.b && w.c == v.c && w.tl == v.tl && w.cap == v.cap && w.ord == v.ord);
      if (!dup) top.push_back(v);
      if (top.size() == 8) break;
    }
    std::vector<std::vector<float>> ms(top.size());
    for (int r = 0; r < 3 * reps + 1 && rc == CHEM_OK; ++r)
      for (size_t k = 0; k < top.size() && rc == CHEM_OK; ++k) {
        chem_opts t = o;
        t.block_size = top[k].b; t.chunk_steps = top[k].c; t.tail_steps = top[k].tl;
        t.tail_cap = top[k].cap; t.pool_order = top[k].ord;
        float el = 0;
        rc = time_one(t, &el);
        ms[k].push_back(el);
      }
    if (rc == CHEM_OK) {
      best_ms = 1e300;
      for (size_t k = 0; k < top.size(); ++k) {
        std::sort(ms[k].begin(), ms[k].end());
        const double med = ms[k][ms[k].size() / 2];
        if (med < best_ms) {
          best_ms = med; best_block = top[k].b; best_chunk = top[k].c; best_tail = top[k].tl;
          best_cap = top[k].cap; best_order = top[k].ord;
        }
      }
    }
  }
  if (rc == CHEM_OK && seen.size() > 1) {
    // neighbour refinement: the sweeps change one setting at a time, so a
    // launch that wins only with two settings changed together can be
    // missed; the confirmed launch is timed round-robin (as above) against
    // its neighbours -- the adjacent block, chunk and hand-off values, the
    // other caps and pool orders -- and replaced by a faster one, at most
    // kRefineMoves times
    constexpr int kRefineMoves = 3;
    auto at = [](const int* arr, int n, int v) {
      for (int i = 0; i < n; ++i)
        if (arr[i] == v) return i;
      return -1;
    };
    constexpr int NB = sizeof(blocks) / sizeof(int), NC = sizeof(chunks) / sizeof(int),
                  NT = sizeof(tails) / sizeof(int), NK = sizeof(caps) / sizeof(int);
    const int orders[] = {-1, ORDER_DEAL, ORDER_RANGE, ORDER_RANGE_DEFER};
    for (int move = 0; move < kRefineMoves && rc == CHEM_OK; ++move) {
      const Seen cur{best_block, best_chunk, best_tail, best_cap, best_order, best_ms};
      std::vector<Seen> cand{cur};
      auto add = [&](int b, int c, int tl, int cap, int ord) {
        if (m->entry->lds_per_lane() * b > 65536) return;
        if (o.scheme == SCHEME_ROS4 && b > 256) return;
        for (const Seen& w : cand)
          if (w.b == b && w.c == c && w.tl == tl && w.cap == cap && w.ord == ord) return;
        cand.push_back({b, c, tl, cap, ord, 0.0});
      };
      const int ib = at(blocks, NB, cur.b), ic = at(chunks, NC, cur.c), it = at(tails, NT, cur.tl);
      for (int d : {-1, 1}) {
        if (ib >= 0 && ib + d >= 0 && ib + d < NB) add(blocks[ib + d], cur.c, cur.tl, cur.cap, cur.ord);
        if (ic >= 0 && ic + d >= 0 && ic + d < NC) add(cur.b, chunks[ic + d], cur.tl, cur.cap, cur.ord);
        if (tune_tail && it >= 0 && it + d >= 0 && it + d < NT)
          add(cur.b, cur.c, tails[it + d], cur.cap, cur.ord);
      }
      if (tune_cap)
        for (int k = 0; k < NK; ++k) add(cur.b, cur.c, cur.tl, caps[k], cur.ord);
      if (o.pool_order == 0 && o.fixed_steps == 0)
        for (int ord : orders) add(cur.b, cur.c, cur.tl, cur.cap, ord);
      if (cand.size() < 2) break;
      std::vector<std::vector<float>> ms(cand.size());
      for (int r = 0; r < 3 * reps + 1 && rc == CHEM_OK; ++r)
        for (size_t k = 0; k < cand.size() && rc == CHEM_OK; ++k) {
          chem_opts t = o;
          t.block_size = cand[k].b; t.chunk_steps = cand[k].c; t.tail_steps = cand[k].tl;
          t.tail_cap = cand[k].cap; t.pool_order = cand[k].ord;
          float el = 0;
          rc = time_one(t, &el);
          ms[k].push_back(el);
        }
      if (rc != CHEM_OK) break;
      size_t win = 0;
      double win_ms = 1e300;
      for (size_t k = 0; k < cand.size(); ++k) {
        std::sort(ms[k].begin(), ms[k].end());
        const double med = ms[k][ms[k].size() / 2];
        if (med < win_ms) { win_ms = med; win = k; }
      }
      best_ms = win_ms;
      if (win == 0) break;
      best_block = cand[win].b; best_chunk = cand[win].c; best_tail = cand[win].tl;
      best_cap = cand[win].cap; best_order = cand[win].ord;
    }
  }
  if (rc != CHEM_OK) return rc;
  *best = o;
  best->block_size = best_block; best->chunk_steps = best_chunk; best->tail_steps = best_tail;
  best->tail_cap = best_cap; best->pool_order = best_order;
  *best_ms_out = best_ms;
  return CHEM_OK;
}

}  // namespace

extern "C" {

const char* chem_strerror(int code) {
  switch (code) {
    case CHEM_OK: return "ok";
    case CHEM_EINVAL: return "invalid argument";
    case CHEM_ENOMEM: return "out of memory";
    case CHEM_EHIP: return "HIP runtime error";
    case CHEM_EPARSE: return "mechanism file unreadable or malformed";
    case CHEM_EUNSUPPORTED: return "no kernel built for this mechanism";
    case CHEM_ECAPACITY: return "more cells than the reserved workspace";
    default: return "unknown error";
  }
}

const char* chem_last_error(void) { return g_err.c_str(); }

int chem_eval_math(int32_t fn, const double* x, double* y, int64_t n, void* stream) {
  if (fn != CHEM_MATH_EXP_CW && fn != CHEM_MATH_LOG_ATANH &&
      fn != CHEM_MATH_EXP_TAB)
    return fail(CHEM_EINVAL, "chem_eval_math: unknown function");
  if (n < 0 || (n > 0 && (!x || !y))) return fail(CHEM_EINVAL, "chem_eval_math: bad argument");
  if (n == 0) return CHEM_OK;
  const int64_t grid = (n + 255) / 256;
  if (grid > 0x7fffffff) return fail(CHEM_EINVAL, "chem_eval_math: n too large");
  hipLaunchKernelGGL(eval_math_kernel, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream,
                     (int)fn, x, y, n);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CHEM_OK : hip_fail(e, "launch eval_math");
}

int chem_eval_exp(const double* x, double* y, int64_t n, void* stream) {
  return chem_eval_math(CHEM_MATH_EXP_CW, x, y, n, stream);
}

int chem_mech_load(const char* path, chem_mech* out) {
  if (!path || !out) return fail(CHEM_EINVAL, "chem_mech_load: null argument");
  *out = nullptr;
  FILE* f = fopen(path, "rb");
  if (!f) return fail(CHEM_EPARSE, std::string("cannot open ") + path);
  std::vector<char> data;
  char buf[65536];
  size_t k;
  while ((k = fread(buf, 1, sizeof buf, f)) > 0) data.insert(data.end(), buf, buf + k);
  fclose(f);
  if (data.size() < 6 || memcmp(data.data(), "MECH 1", 6) != 0)
    return fail(CHEM_EPARSE, std::string(path) + ":1: missing 'MECH 1' header");
  const uint64_t hsh = fnv1a64(data);
  const MechEntry* hit = nullptr;
  for (const auto& e : g_registry)
    if (e.hash == hsh) hit = &e;
  if (!hit) {
    char msg[128];
    snprintf(msg, sizeof msg, "no built-in kernel for mechanism hash %016llx",
             (unsigned long long)hsh);
    return fail(CHEM_EUNSUPPORTED, msg);
  }
  chem_mech m = new (std::nothrow) chem_mech_s();
  if (!m) return fail(CHEM_ENOMEM, "chem_mech_load: host allocation");
  m->entry = hit;
  hipError_t e = hipGetDevice(&m->device);
  if (e != hipSuccess) { delete m; return hip_fail(e, "hipGetDevice"); }
  e = hipDeviceGetAttribute(&m->n_cu, hipDeviceAttributeMultiprocessorCount, m->device);
  if (e != hipSuccess) { delete m; return hip_fail(e, "hipDeviceGetAttribute"); }
  if (m->device < 0 || m->device >= kMaxDevices) {
    delete m;
    return fail(CHEM_EUNSUPPORTED, "chem_mech_load: device ordinal beyond 63");
  }
  {
    // this device's address of the no-allocation scratch array, looked up
    // once per device with that device current
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[m->device]) {
      void* ptr = nullptr;
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr) {
        delete m;
        return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
      }
      g_scratch_ptr[m->device] = ptr;
    }
    m->scratch = g_scratch_ptr[m->device];
  }
  *out = m;
  return CHEM_OK;
}

int chem_mech_query(chem_mech m, int32_t* n_species, int32_t* n_reactions, uint64_t* hash) {
  if (!m) return fail(CHEM_EINVAL, "chem_mech_query: null handle");
  if (n_species) *n_species = m->entry->ns;
  if (n_reactions) *n_reactions = m->entry->nr;
  if (hash) *hash = m->entry->hash;
  return CHEM_OK;
}

void chem_mech_free(chem_mech m) {
  if (!m) return;
  // teardown: errors have nowhere to go
  for (hipEvent_t& ev : m->tev)
    if (ev) (void)hipEventDestroy(ev);
  for (hipEvent_t& ev : m->box_done)
    if (ev) {
      (void)hipEventSynchronize(ev);
      (void)hipEventDestroy(ev);
    }
  free_cell_workspace(m);
  if (m->d_next) (void)hipFree(m->d_next);
  if (m->d_boxes) (void)hipFree(m->d_boxes);
  if (m->h_boxes) (void)hipHostFree(m->h_boxes);
  delete m;
}

int chem_workspace_reserve(chem_mech m, int64_t max_cells) {
  if (!m || max_cells < 0) return fail(CHEM_EINVAL, "chem_workspace_reserve: bad argument");
  int rc = alloc_fixed_workspace(m);
  if (rc) return rc;
  if (max_cells <= m->reserved && m->tail.mem) return CHEM_OK;
  // growing: calls still queued may use the old buffers
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize(workspace)");
  free_cell_workspace(m);
  const int64_t cap = std::max<int64_t>(max_cells, 1);
  if ((rc = alloc_tail(m->tail, cap, m->entry->tail_rd)) != CHEM_OK ||
      (rc = alloc_order(m->order, cap)) != CHEM_OK) {
    free_cell_workspace(m);
    return rc;
  }
  e = hipMalloc(&m->d_prim, sizeof(double) * (size_t)cap * (m->entry->ns + 3));
  if (e == hipSuccess) e = hipMalloc(&m->d_flag, (size_t)cap);
  if (e != hipSuccess) {
    free_cell_workspace(m);
    return hip_fail(e, "hipMalloc(primitive work state)");
  }
  m->reserved = max_cells;
  return CHEM_OK;
}

int chem_set_kernel_timing(chem_mech m, int32_t on) {
  if (!m) return fail(CHEM_EINVAL, "chem_set_kernel_timing: null mechanism");
  if (on) {
    for (hipEvent_t& ev : m->tev) {
      if (ev) continue;
      hipError_t e = hipEventCreate(&ev);
      if (e != hipSuccess) { ev = nullptr; return hip_fail(e, "hipEventCreate(kernel timing)"); }
    }
  }
  m->timing = on != 0;
  m->timed_last = false;
  return CHEM_OK;
}

int chem_kernel_times(chem_mech m, float* ms, int32_t n) {
  if (!m || !ms || n < 4) return fail(CHEM_EINVAL, "chem_kernel_times: bad argument");
  if (!m->timed_last) return fail(CHEM_EINVAL, "chem_kernel_times: no timed call since timing was set");
  hipError_t e = hipEventSynchronize(m->tev[4]);
  if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize(kernel timing)");
  // persistent, tail sort, cooperative, resumption
  for (int k = 0; k < 4; ++k) {
    ms[k] = 0.0f;
    e = hipEventElapsedTime(&ms[k], m->tev[k], m->tev[k + 1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime(kernel timing)");
  }
  if (n >= 5) {
    ms[4] = 0.0f;
    e = hipEventElapsedTime(&ms[4], m->tev[0], m->tev[4]);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime(kernel timing)");
  }
  return CHEM_OK;
}

int chem_tail_stats(chem_mech m, int64_t* out, int32_t n) {
  if (!m || !out || n < 3) return fail(CHEM_EINVAL, "chem_tail_stats: bad argument");
  if (!m->timed_last) return fail(CHEM_EINVAL, "chem_tail_stats: no timed call since timing was set");
  hipError_t e = hipEventSynchronize(m->tev[4]);
  if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize(tail stats)");
  out[0] = out[1] = out[2] = 0;
  if (!m->timed_tail) return CHEM_OK;
  unsigned char head[TailStore::kHead];
  e = hipMemcpy(head, m->timed_tail->mem, sizeof head, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(tail stats)");
  unsigned int count, split;
  unsigned long long steps;
  memcpy(&count, head + 8, 4);
  memcpy(&split, head + 12, 4);
  memcpy(&steps, head + 24, 8);
  out[0] = count;
  out[1] = split;
  out[2] = (int64_t)steps;
  return CHEM_OK;
}

int chem_integrate(chem_mech m, double* state, int64_t ld, int64_t n_cells, double dt,
                   const chem_opts* opts, void* stream, int32_t* status, int32_t* counts) {
  if (!m) return fail(CHEM_EINVAL, "chem_integrate: null mechanism");
  if (n_cells < 0 || ld < n_cells) return fail(CHEM_EINVAL, "chem_integrate: need 0 <= n_cells <= ld");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(CHEM_EINVAL, "chem_integrate: dt must be finite and > 0");
  if (n_cells > 0 && !state) return fail(CHEM_EINVAL, "chem_integrate: null state");
  int rc = check_opts(opts);
  if (rc) return rc;
  if (n_cells == 0) return CHEM_OK;
  hipStream_t s = (hipStream_t)stream;
  PoolArgs a{};
  a.one = BoxDesc{state, ld, n_cells, 0, dt, 1, 0, status, counts, nullptr};
  a.boxes = nullptr;
  a.n_boxes = 1;
  a.total = n_cells;
  a.c = make_control(opts);
  a.fixed_steps = opts ? opts->fixed_steps : 0;
  a.scheme = opts ? opts->scheme : SCHEME_LSRK;
  int block, chunk;
  pick_launch(m, n_cells, opts, &block, &chunk);
  if (chunk < 0) {
    rc = check_scheme_launch(m, opts, block);
    if (rc) return rc;
    hipError_t e = m->entry->launch_direct(a, block, s);
    if (e != hipSuccess) return hip_fail(e, "launch lsrk_direct");
    return CHEM_OK;
  }
  return run_pool(m, a, opts, s);
}

int chem_integrate_noalloc(chem_mech m, double* state, int64_t ld, int64_t n_cells, double dt,
                           const chem_opts* opts, void* stream, int32_t* status, int32_t* counts) {
  if (!m) return fail(CHEM_EINVAL, "chem_integrate_noalloc: null mechanism");
  if (n_cells < 0 || ld < n_cells)
    return fail(CHEM_EINVAL, "chem_integrate_noalloc: need 0 <= n_cells <= ld");
  if (!(dt > 0) || !std::isfinite(dt))
    return fail(CHEM_EINVAL, "chem_integrate_noalloc: dt must be finite and > 0");
  if (n_cells > 0 && !state) return fail(CHEM_EINVAL, "chem_integrate_noalloc: null state");
  int rc = check_opts(opts);
  if (rc) return rc;
  if (n_cells > kNoAllocMaxCells)
    return fail(CHEM_ECAPACITY, "chem_integrate_noalloc: more than 1048576 cells");
  if (n_cells == 0) return CHEM_OK;
  if (!m->scratch) return fail(CHEM_EHIP, "chem_integrate_noalloc: no scratch address for this device");
  hipStream_t s = (hipStream_t)stream;
  PoolArgs a{};
  a.one = BoxDesc{state, ld, n_cells, 0, dt, 1, 0, status, counts, nullptr};
  a.boxes = nullptr;
  a.n_boxes = 1;
  a.total = n_cells;
  a.c = make_control(opts);
  a.fixed_steps = opts ? opts->fixed_steps : 0;
  a.scheme = opts ? opts->scheme : SCHEME_LSRK;
  int block, chunk;
  pick_launch(m, n_cells, opts, &block, &chunk);
  if (chunk < 0) {
    rc = check_scheme_launch(m, opts, block);
    if (rc) return rc;
    hipError_t e = m->entry->launch_direct(a, block, s);
    if (e != hipSuccess) return hip_fail(e, "launch lsrk_direct");
    return CHEM_OK;
  }
  // the same kernels as chem_integrate, on this device's scratch array: the
  // pool counter at its start, then the tail records and the pool order
  // (every counter is cleared by a kernel at the start of the call)
  unsigned char* base = static_cast<unsigned char*>(m->scratch);
  TailStore ts;
  ts.mem = base + kScratchTailOff;
  ts.cap = kNoAllocMaxCells;
  OrderStore os;
  os.mem = base + kScratchOrderOff;
  os.cap = kNoAllocMaxCells;
  return run_pool_with(m, a, opts, s, reinterpret_cast<unsigned long long*>(base), ts, &os,
                       false);
}

int chem_react_conserved(chem_mech m, double* cons, int64_t ld, int64_t n_cells, double dt,
                         const chem_opts* opts, void* stream, int32_t* status, int32_t* counts) {
  if (!m) return fail(CHEM_EINVAL, "chem_react_conserved: null mechanism");
  if (n_cells < 0 || ld < n_cells)
    return fail(CHEM_EINVAL, "chem_react_conserved: need 0 <= n_cells <= ld");
  if (!(dt > 0) || !std::isfinite(dt))
    return fail(CHEM_EINVAL, "chem_react_conserved: dt must be finite and > 0");
  if (n_cells > 0 && !cons) return fail(CHEM_EINVAL, "chem_react_conserved: null state");
  int rc = check_opts(opts);
  if (rc) return rc;
  if (n_cells == 0) return CHEM_OK;
  if (n_cells > 0x7fffffff) return fail(CHEM_EINVAL, "more than 2^31-1 cells in one call");
  hipStream_t s = (hipStream_t)stream;
  rc = check_capacity(m, n_cells, "chem_react_conserved");
  if (rc) return rc;
  hipError_t e = m->entry->launch_cons_to_prim(cons, ld, n_cells, m->d_prim, m->d_flag, s);
  if (e != hipSuccess) return hip_fail(e, "launch cons_to_prim");
  rc = chem_integrate(m, m->d_prim, n_cells, n_cells, dt, opts, stream, status, counts);
  if (rc) return rc;
  e = m->entry->launch_prim_to_cons(m->d_prim, m->d_flag, n_cells, cons, ld, status, s);
  if (e != hipSuccess) return hip_fail(e, "launch prim_to_cons");
  return CHEM_OK;
}

int chem_integrate_batched(chem_mech m, const chem_box* boxes, int32_t n_boxes,
                           const chem_opts* opts, void* stream) {
  if (!m) return fail(CHEM_EINVAL, "chem_integrate_batched: null mechanism");
  int rc = check_opts(opts);
  if (rc) return rc;
  std::vector<BoxDesc> table;
  int64_t total = 0;
  rc = build_table(boxes, n_boxes, table, &total);
  if (rc) return rc;
  if (total == 0) return CHEM_OK;
  hipStream_t s = (hipStream_t)stream;
  rc = check_capacity(m, total, "chem_integrate_batched");
  if (rc) return rc;
  if (table.size() > (size_t)kMaxBoxes)
    return fail(CHEM_ECAPACITY, "chem_integrate_batched: more than 4096 non-empty boxes");
  // a ring slot is free once the call that used it last has finished
  const int slot = m->box_slot;
  m->box_slot = (slot + 1) % kBoxRing;
  hipError_t e = hipEventSynchronize(m->box_done[slot]);
  if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize(box table)");
  BoxDesc* h_tab = m->h_boxes + (size_t)slot * kMaxBoxes;
  BoxDesc* d_tab = m->d_boxes + (size_t)slot * kMaxBoxes;
  memcpy(h_tab, table.data(), sizeof(BoxDesc) * table.size());
  e = hipMemcpyAsync(d_tab, h_tab, sizeof(BoxDesc) * table.size(), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(box table)");
  PoolArgs a{};
  a.one = table[0];
  a.boxes = d_tab;
  a.n_boxes = (int32_t)table.size();
  a.total = total;
  a.c = make_control(opts);
  a.fixed_steps = opts ? opts->fixed_steps : 0;
  a.scheme = opts ? opts->scheme : SCHEME_LSRK;
  rc = run_pool(m, a, opts, s);
  // recorded even when the launch failed, so the slot never waits on a stale event
  e = hipEventRecord(m->box_done[slot], s);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord(box table)");
  return CHEM_OK;
}

int chem_graph_capture_batched(chem_mech m, const chem_box* boxes, int32_t n_boxes,
                               const chem_opts* opts, void* stream, chem_graph* out) {
  if (!m || !out) return fail(CHEM_EINVAL, "chem_graph_capture_batched: null argument");
  *out = nullptr;
  int rc = check_opts(opts);
  if (rc) return rc;
  std::vector<BoxDesc> table;
  int64_t total = 0;
  rc = build_table(boxes, n_boxes, table, &total);
  if (rc) return rc;
  if (total == 0) return fail(CHEM_EINVAL, "chem_graph_capture_batched: no cells");
  if (total > 0x7fffffff) return fail(CHEM_EINVAL, "more than 2^31-1 work items in one call");
  int block, chunk;
  pick_launch(m, total, opts, &block, &chunk);
  if (m->entry->lds_per_lane() * block > 65536)
    return fail(CHEM_EINVAL, "block_size too large for this mechanism's LDS compaction slots");
  rc = check_scheme_launch(m, opts, block);
  if (rc) return rc;
  chem_graph g = new (std::nothrow) chem_graph_s();
  if (!g) return fail(CHEM_ENOMEM, "chem_graph_capture_batched: host allocation");
  auto bail = [&](hipError_t e, const char* what) {
    chem_graph_destroy(g);
    return hip_fail(e, what);
  };
  hipError_t e = hipMalloc(&g->d_boxes, sizeof(BoxDesc) * table.size());
  if (e != hipSuccess) return bail(e, "hipMalloc(graph box table)");
  e = hipMalloc(&g->d_next, sizeof(unsigned long long));
  if (e != hipSuccess) return bail(e, "hipMalloc(graph pool counter)");
  const int tail_steps = pick_tail(m, total, opts);
  if (tail_steps > 0) {
    rc = alloc_tail(g->tail, total, m->entry->tail_rd);
    if (rc) { chem_graph_destroy(g); return rc; }
  }
  const int omode = pick_order(m, total, opts);
  const bool ordered = omode != 0;
  if (ordered) {
    rc = alloc_order(g->order, total);
    if (rc) { chem_graph_destroy(g); return rc; }
  }
  e = hipMemcpy(g->d_boxes, table.data(), sizeof(BoxDesc) * table.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return bail(e, "hipMemcpy(graph box table)");
  if (stream) {
    e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return bail(e, "hipStreamSynchronize");
  }
  PoolArgs a{};
  a.one = table[0];
  a.boxes = g->d_boxes;
  a.n_boxes = (int32_t)table.size();
  a.total = total;
  a.next = g->d_next;
  a.c = make_control(opts);
  a.chunk = chunk > 0 ? chunk : kDefaultChunk;
  a.fixed_steps = opts ? opts->fixed_steps : 0;
  a.scheme = opts ? opts->scheme : SCHEME_LSRK;
  a.tail_steps = tail_steps;
  if (tail_steps > 0) {
    a.tail = g->tail.view();
    a.tail.cap = pick_cap(m, total, opts);
  }
  const int grid = grid_for(m, block, total, a.scheme);
  hipStream_t cs;
  e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return bail(e, "hipStreamCreate(capture)");
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) { (void)hipStreamDestroy(cs); return bail(e, "hipStreamBeginCapture"); }
  OrderBuf ob = ordered ? g->order.view() : OrderBuf{};
  ob.mode = omode == ORDER_RANGE_DEFER ? ORDER_RANGE : omode;
  ob.defer = omode == ORDER_RANGE_DEFER;
  ob.t_split = m->entry->t_split;
  hipError_t le = launch_step(m, a, block, grid, cs, ordered ? &ob : nullptr);
  e = hipStreamEndCapture(cs, &g->graph);
  (void)hipStreamDestroy(cs);
  if (le != hipSuccess) return bail(le, "launch integrator kernels (capture)");
  if (e != hipSuccess) return bail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return bail(e, "hipGraphInstantiate");
  *out = g;
  return CHEM_OK;
}

int chem_graph_launch(chem_graph g, void* stream) {
  if (!g || !g->exec) return fail(CHEM_EINVAL, "chem_graph_launch: null graph");
  hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return CHEM_OK;
}

void chem_graph_destroy(chem_graph g) {
  if (!g) return;
  // teardown: errors have nowhere to go
  (void)hipDeviceSynchronize();
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->d_boxes) (void)hipFree(g->d_boxes);
  if (g->d_next) (void)hipFree(g->d_next);
  if (g->tail.mem) (void)hipFree(g->tail.mem);
  if (g->order.mem) (void)hipFree(g->order.mem);
  if (g->fb_list) (void)hipFree(g->fb_list);
  if (g->fb_count) (void)hipFree(g->fb_count);
  delete g;
}

int chem_autotune(chem_mech m, const chem_box* boxes, int32_t n_boxes, const chem_opts* base,
                  int32_t reps, const char* cache_path, void* stream, chem_opts* best) {
  if (!m) return fail(CHEM_EINVAL, "chem_autotune: null mechanism");
  int rc = check_opts(base);
  if (rc) return rc;
  std::vector<BoxDesc> table;
  int64_t total = 0;
  rc = build_table(boxes, n_boxes, table, &total);
  if (rc) return rc;
  if (total == 0) return fail(CHEM_EINVAL, "chem_autotune: no cells");
  if (reps < 1) reps = 3;
  hipStream_t s = (hipStream_t)stream;
  const int bucket = size_bucket(total);
  const int tkey = tuned_key(total, base);
  char key[160];
  snprintf(key, sizeof key, "%016llx:%d:%s%s", (unsigned long long)m->entry->hash, bucket,
           arch_name(m->device).c_str(),
           (base && base->scheme == SCHEME_RKF45)  ? ":rkf45"
           : (base && base->scheme == SCHEME_ROS4) ? ":ros4"
                                                   : "");
  chem_opts o = base ? *base : chem_opts{0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<TuneEntry> cache;
  if (cache_path) {
    cache = read_cache(cache_path);
    for (const auto& en : cache)
      if (en.key == key) {
        m->tuned[tkey] = {en.block, en.chunk, en.tail, en.cap, en.order};
        if (best) {
          *best = o; best->block_size = en.block; best->chunk_steps = en.chunk;
          best->tail_steps = en.tail; best->tail_cap = en.cap; best->pool_order = en.order;
        }
        return CHEM_OK;
      }
  }
  // the trials are batched calls on the mechanism's own workspace
  if (!m->fixed_ready || total > m->reserved) {
    rc = chem_workspace_reserve(m, std::max<int64_t>(total, m->reserved));
    if (rc) return rc;
  }
  // snapshot every box so trials can restore the caller's data
  std::vector<double*> snap(table.size(), nullptr);
  std::vector<size_t> bytes(table.size());
  auto cleanup = [&]() { for (double* p : snap) if (p) (void)hipFree(p); };
  hipError_t e;
  for (size_t i = 0; i < table.size(); ++i) {
    bytes[i] = sizeof(double) * (size_t)table[i].ld * (size_t)(m->entry->ns + 3);
    e = hipMalloc(&snap[i], bytes[i]);
    if (e != hipSuccess) { cleanup(); return hip_fail(e, "hipMalloc(autotune snapshot)"); }
    e = hipMemcpyAsync(snap[i], table[i].state, bytes[i], hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) { cleanup(); return hip_fail(e, "snapshot copy"); }
  }
  auto restore = [&]() -> hipError_t {
    for (size_t i = 0; i < table.size(); ++i) {
      hipError_t r = hipMemcpyAsync(table[i].state, snap[i], bytes[i], hipMemcpyDeviceToDevice, s);
      if (r != hipSuccess) return r;
    }
    return hipSuccess;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    cleanup();
    return hip_fail(e, "hipEventCreate(autotune)");
  }
  // one timed call of a configuration from the snapshot
  auto time_one = [&](const chem_opts& t, float* el) -> int {
    if ((e = restore()) != hipSuccess) return hip_fail(e, "restore");
    if ((e = hipEventRecord(e0, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    int trc = chem_integrate_batched(m, boxes, n_boxes, &t, stream);
    if (trc != CHEM_OK) return trc;
    if ((e = hipEventRecord(e1, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if ((e = hipEventSynchronize(e1)) != hipSuccess) return hip_fail(e, "trial");
    *el = 0;
    if ((e = hipEventElapsedTime(el, e0, e1)) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    return CHEM_OK;
  };
  chem_opts found{};
  double best_ms = 0.0;
  rc = tune_search(m, o, reps, time_one, &found, &best_ms);
  if ((e = restore()) != hipSuccess && rc == CHEM_OK) rc = hip_fail(e, "restore");
  if ((e = hipStreamSynchronize(s)) != hipSuccess && rc == CHEM_OK) rc = hip_fail(e, "autotune sync");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  cleanup();
  if (rc != CHEM_OK) return rc;
  m->tuned[tkey] = {found.block_size, found.chunk_steps, found.tail_steps, found.tail_cap,
                    found.pool_order};
  if (best) *best = found;
  if (cache_path) {
    cache.push_back(TuneEntry{key, found.block_size, found.chunk_steps, found.tail_steps,
                              found.tail_cap, found.pool_order, best_ms});
    rc = write_cache(cache_path, cache);
  }
  return rc;
}

}  // extern "C"

#include "surrogate_api.hip.h"
