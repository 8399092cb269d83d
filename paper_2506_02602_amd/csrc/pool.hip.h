// pool.hip.h -- the work pool shared by the per-lane and the cooperative
// kernels: state blocks (boxes) laid out as one pool of work items, the
// tail records through which the per-lane kernel hands long-running cells
// to the cooperative kernel, the launch arguments, and the per-mechanism
// launcher of the cooperative kernel (built in its own compilation unit).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lsrk.hip.h"

namespace chemgpu {

struct BoxDesc {
  double* state;
  int64_t ld;
  int64_t n;
  int64_t start;  // first pool index of this block
  double dt;
  int32_t n_sub;
  int32_t pad;
  int32_t* status;
  int32_t* counts;
  const int32_t* index;  // NULL, or the cell index of each of this block's pool items
};

// A handed-over cell's record when the state travels with it (TailBuf::rec):
// doubles T, Y_1..Y_N, rho, h, t, then the ints item, nacc, nrej, sub, base;
// RD doubles per record, a multiple of 64 bytes, so the claim of a record in
// key order reads whole cache lines instead of one word from each state row.
template <class M>
struct TailRec {
  static constexpr int N1 = M::NS + 1;
  static constexpr int RHO = N1, H = N1 + 1, T = N1 + 2, INTS = N1 + 3;
  static constexpr int RD = (N1 + 6 + 7) / 8 * 8;
};

// Cells handed from the per-lane kernel to the cooperative one or to its
// own resumption.  With rec set, each record carries the cell's state and
// progress (TailRec) and the cell's rows are written only when it finishes;
// without (the fixed scratch of the allocation-free call), the cell's (T, Y)
// and step hint at time t go to its own state rows and its progress to the
// structure-of-arrays fields below.
struct TailBuf {
  double* rec;            // NULL, or cap records of TailRec<M>::RD doubles
  int32_t* item;          // pool index
  double* t;              // time reached within the current sub-call
  int32_t* nacc;
  int32_t* nrej;
  int32_t* sub;           // current sub-call
  int32_t* base;          // steps taken before the current sub-call
  int32_t* key;           // bucket of the cell's estimated remaining steps (tail_key)
  int32_t* order;         // record indices, largest key first (tail_count, tail_scatter)
  unsigned int* count;    // records written (zeroed before launch)
  unsigned long long* next;   // records claimed by the cooperative kernel (zeroed)
  unsigned long long* next2;  // records claimed by the per-lane resumption (zeroed)
  unsigned int* split;    // records the cooperative kernel takes: all or none (tail_scatter)
  unsigned int* btot;     // records per key bucket (zeroed before launch)
  unsigned int* bcur;     // per key bucket: records given a position so far (zeroed)
  unsigned long long* coop_steps;  // steps the cooperative kernel took (zeroed; measurement)
  int cap;                // at most this many records go to the cooperative kernel; more
                          // are resumed one per lane (the count decides, so the choice is
                          // a function of the input only)
};

struct PoolArgs {
  BoxDesc one;                 // used when boxes == nullptr
  const BoxDesc* boxes;        // device table, sorted by start
  int32_t n_boxes;
  int64_t total;               // pool size
  const unsigned int* total_dev;  // NULL, or a device word holding the pool size
  unsigned long long* next;    // pool counter (zeroed before launch)
  Control c;
  int chunk;
  int fixed_steps;
  int tail_steps;              // > 0: a cell that has taken this many steps moves to the tail
  TailBuf tail;
  int resume;                  // 1: the work items are tail records, resumed one per lane
  int scheme;                  // SCHEME_LSRK, SCHEME_RKF45 or SCHEME_ROS4
  const int32_t* order;        // NULL, or pool position -> work item (order_place)
  // Deferred cells (pool order 3): the first launch claims only positions
  // [*defer_h, pool size) of defer_order (the cells above the NASA-7 range
  // switch); the resumption claims its tail records and then positions
  // [0, *defer_h) as fresh cells, which it steps to the end.
  int defer;
  const unsigned int* defer_h;
  const int32_t* defer_order;
  const unsigned int* pool_dev;  // the resumption: the first launch's total_dev
};

__device__ __forceinline__ int find_box(const PoolArgs& a, int64_t g) {
  if (!a.boxes) return 0;
  int lo = 0, hi = a.n_boxes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.boxes[mid].start <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ const BoxDesc& box_ref(const PoolArgs& a, int b) {
  return a.boxes ? a.boxes[b] : a.one;
}

__device__ __forceinline__ int64_t cell_index(const BoxDesc& bd, int64_t g) {
  const int64_t j = g - bd.start;
  return bd.index ? (int64_t)bd.index[j] : j;
}

template <class M>
__device__ __forceinline__ void load_cell(const BoxDesc& bd, int64_t i, double (&u)[M::NS + 1],
                                          double& rho, double& h) {
  const double* s = bd.state;
#pragma unroll
  for (int v = 0; v <= M::NS; ++v) u[v] = s[v * bd.ld + i];
  rho = s[(M::NS + 1) * bd.ld + i];
  h = s[(M::NS + 2) * bd.ld + i];
}

template <class M>
__device__ __forceinline__ void store_cell(const BoxDesc& bd, int64_t i, const double (&u)[M::NS + 1],
                                           double h, int status, int nacc, int nrej) {
  double* s = bd.state;
  if (status != CELL_NONFINITE) {
#pragma unroll
    for (int v = 0; v <= M::NS; ++v) s[v * bd.ld + i] = u[v];
    s[(M::NS + 2) * bd.ld + i] = h;
  }
  if (bd.status) bd.status[i] = status;
  if (bd.counts) { bd.counts[i] = nacc; bd.counts[bd.n + i] = nrej; }
}

__device__ __forceinline__ double initial_h(double h, double dt) {
  return (h > 0.0 && h < dt) ? h : dt;
}

// Launch the cooperative kernel over the tail records of a (see TailBuf);
// defined and instantiated for every built-in mechanism in coop.hip.
template <class M>
hipError_t launch_coop(const PoolArgs& a, int n_cu, hipStream_t s);

}  // namespace chemgpu
