// Learned-surrogate kernels: BF16 MFMA (gfx950 v_mfma_f32_16x16x32_bf16,
// FP32 accumulation) for training and inference of the 3-hidden-layer SiLU
// MLP that maps (T, ln p, ln dt, Y_1..Y_N) to the increment (dT, dY) of one
// flow step, plus the FP64 feature and trust-test code around it.
//
// MFMA operand layout used throughout (one wave, D = A B, A 16x32, B 32x16):
//   lane l supplies A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16],
//   j = 0..7, and receives D[4 (l / 16) + i][l % 16], i = 0..3.
// BF16 values are kept as their 16-bit patterns (round to nearest even from
// FP32).
#pragma once

namespace surr {

constexpr int HID = 128;

typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 pattern, round to nearest even (gfx950's v_cvt_pk_bf16_f32)
__device__ __forceinline__ unsigned short f2bf(float f) {
  return __builtin_bit_cast(unsigned short, (__bf16)f);
}

__device__ __forceinline__ float bf2f(unsigned short b) {
  return __uint_as_float(((unsigned)b) << 16);
}

__device__ __forceinline__ f32x4 mfma(v8s a, v8s b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                  __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + expf(-z)); }

// SiLU for the inference epilogue: native exp2 and reciprocal (a few ulp in
// FP32), far below the BF16 rounding that follows.
__device__ __forceinline__ float silu_fast(float z) {
  return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}


// ------------------------------------------- the generic forward's GEMM
// C[M x N] = A[M x K] B[K x N] + bias with BF16 operands addressed by
// strides, one wave per 16x16 output tile; with EPI_BIAS_SILU also the BF16
// SiLU of the result (surrogate_forward on raw inputs; the training step
// has kernels of its own).
enum { EPI_BIAS_SILU = 1, EPI_BIAS = 2 };

struct GemmArgs {
  const unsigned short* A; long sam, sak;
  const unsigned short* B; long sbk, sbn;
  int M, N, K;
  float* C; long scm, scn, cz;
  unsigned short* Cb; long sbm, sbc;   // BF16 copy of the epilogue result (optional)
  const float* bias;
  int kper;                            // K range per split (multiple of 32)
};

template <int EPI>
__global__ __launch_bounds__(256) void gemm_bf16(GemmArgs g) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tiles_n = (g.N + 15) >> 4;
  const long tile = (long)blockIdx.x * 4 + wave;
  const long tm = tile / tiles_n, tn = tile % tiles_n;
  if (tm * 16 >= g.M) return;
  const int r = lane & 15, grp = lane >> 4;
  const long kbeg = (long)blockIdx.z * g.kper;
  const long kend = kbeg + g.kper < g.K ? kbeg + g.kper : g.K;
  const long m = tm * 16 + r, n = tn * 16 + r;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (long k0 = kbeg; k0 < kend; k0 += 32) {
    v8s a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const long k = k0 + grp * 8 + j;
      a[j] = (m < g.M && k < kend) ? (short)g.A[m * g.sam + k * g.sak] : (short)0;
      b[j] = (n < g.N && k < kend) ? (short)g.B[k * g.sbk + n * g.sbn] : (short)0;
    }
    acc = mfma(a, b, acc);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const long cm = tm * 16 + grp * 4 + i, cn = tn * 16 + r;
    if (cm >= g.M || cn >= g.N) continue;
    float v = acc[i];
    if (EPI == EPI_BIAS_SILU || EPI == EPI_BIAS) v += g.bias[cn];
    g.C[blockIdx.z * g.cz + cm * g.scm + cn * g.scn] = v;
    if (EPI == EPI_BIAS_SILU) g.Cb[cm * g.sbm + cn * g.sbc] = f2bf(silu_f(v));
  }
}

// batch gather through the epoch's permutation src = (pa * i + pb) mod n
__global__ void gather_batch(const float* Xn, const float* Yn, long n, int ni, int no, long first,
                             int B, unsigned long long pa, unsigned long long pb,
                             unsigned short* X0, float* Yb) {
  const int rr = blockIdx.x * blockDim.x + threadIdx.x;
  if (rr >= B) return;
  const unsigned long long idx = (unsigned long long)(first + rr);
  const long src = (long)((pa * (idx % (unsigned long long)n) + pb) % (unsigned long long)n);
  for (int k = 0; k < ni; ++k) X0[(long)rr * ni + k] = f2bf(Xn[src * ni + k]);
  for (int o = 0; o < no; ++o) Yb[(long)rr * no + o] = Yn[src * no + o];
}

__global__ void cast_bf16(const float* x, long n, unsigned short* y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

// per-column mean / std (FP64 sums) of an [n x cols] FP32 matrix; one block per column
__global__ __launch_bounds__(256) void col_moments(const float* x, long n, int cols, float* mu,
                                                   float* sd) {
  __shared__ double s1[256], s2[256];
  const int c = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (long r = threadIdx.x; r < n; r += blockDim.x) {
    const double v = x[r * cols + c];
    a += v;
    b += v * v;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) { s1[threadIdx.x] += s1[threadIdx.x + w]; s2[threadIdx.x] += s2[threadIdx.x + w]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mean = s1[0] / (double)n;
    double var = s2[0] / (double)n - mean * mean;
    double sdv = var > 0 ? sqrt(var) : 0.0;
    if (!(sdv > 1e-12 * fabs(mean))) sdv = 0.0;  // a constant column: standardised to 0
    mu[c] = (float)mean;
    sd[c] = (float)sdv;
  }
}

// standardise an [n x cols] matrix in place
__global__ void standardise(float* x, long n, int cols, const float* mu, const float* sd) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * cols) return;
  const int c = (int)(i % cols);
  x[i] = sd[c] > 0.f ? (x[i] - mu[c]) / sd[c] : 0.f;
}

// per-column min and max (the training hull); one block per column
__global__ __launch_bounds__(256) void col_minmax(const float* x, long n, int cols, float* zmin,
                                                  float* zmax) {
  __shared__ float lo[256], hi[256];
  const int c = blockIdx.x;
  float mn = 3.4e38f, mx = -3.4e38f;
  for (long r = threadIdx.x; r < n; r += blockDim.x) {
    const float z = x[r * cols + c];
    mn = fminf(mn, z);
    mx = fmaxf(mx, z);
  }
  lo[threadIdx.x] = mn;
  hi[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      lo[threadIdx.x] = fminf(lo[threadIdx.x], lo[threadIdx.x + w]);
      hi[threadIdx.x] = fmaxf(hi[threadIdx.x], hi[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) { zmin[c] = lo[0]; zmax[c] = hi[0]; }
}

// FP64 -> BF16 pattern, rounded once (nearest even) to 8 significant bits
__device__ __forceinline__ unsigned short d2bf(double x) {
  if (!(fabs(x) < 3.0e38)) return f2bf((float)x);
  unsigned long long b = (unsigned long long)__double_as_longlong(x);
  b += 0x00000FFFFFFFFFFFull + ((b >> 45) & 1ull);
  b &= ~0x00001FFFFFFFFFFFull;
  return (unsigned short)(__float_as_uint((float)__longlong_as_double((long long)b)) >> 16);
}

// Packed column order of the hidden layers: column c of a packed matrix holds
// input feature perm(c), so that a layer's MFMA output registers are already
// the next layer's B operand (no LDS round trip between layers).
__host__ __device__ constexpr int packed_feature(int c) {
  const int kc = c >> 5, rr = c & 31, gg = rr >> 3, j = rr & 7;
  return 32 * kc + (j < 4 ? 4 * gg + j : 16 + 4 * gg + (j - 4));
}

// Row strides (in BF16 elements) of the packed weights as they sit in LDS:
// each row is padded by one 16-byte chunk to an odd number of chunks, so
// the 16 rows that a wave's 16-byte operand reads touch (r16 = 0..15, one
// chunk each) start on 16 different bank groups: no bank conflicts,
// whether the LDS serves 8 or 16 such reads per clock.
constexpr int kRowPad = 8;
__host__ __device__ constexpr int w1_ld(int kc1) { return kc1 * 32 + kRowPad; }
constexpr int kWLd = HID + kRowPad;
__host__ __device__ constexpr long packed_weight_elems(int kc1, int ot4) {
  return (long)HID * w1_ld(kc1) + 2L * HID * kWLd + (long)ot4 * 16 * kWLd;
}

// theta (FP32 master, natural layout) -> BF16 packed weights (padded rows,
// padding zero) + FP32 biases; and the reciprocals of the input scales in
// FP64 (0 for a constant input), so that the inference standardises with a
// multiply
__global__ void pack_weights(const float* theta, int ni, int no, int kc1, int ot4,
                             unsigned short* wp, float* bp, const float* sd_in, double* isd) {
  if (blockIdx.x == 0 && (int)threadIdx.x < ni)
    isd[threadIdx.x] = sd_in[threadIdx.x] > 0.f ? 1.0 / (double)sd_in[threadIdx.x] : 0.0;
  const int l1 = w1_ld(kc1);
  const long w1 = (long)HID * l1, w2 = (long)HID * kWLd, w4 = (long)ot4 * 16 * kWLd;
  const long oW1 = 0, ob1 = (long)HID * ni, oW2 = ob1 + HID, ob2 = oW2 + (long)HID * HID;
  const long oW3 = ob2 + HID, ob3 = oW3 + (long)HID * HID, oW4 = ob3 + HID, ob4 = oW4 + (long)no * HID;
  const long total = w1 + 2 * w2 + w4 + 3 * HID + ot4 * 16;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x) {
    if (i < w1) {
      const long row = i / l1, k = i % l1;
      wp[i] = k < ni ? f2bf(theta[oW1 + row * ni + k]) : (unsigned short)0;
    } else if (i < w1 + 2 * w2) {
      const long j = i - w1, which = j / w2, jj = j % w2, row = jj / kWLd, c = jj % kWLd;
      const long base = which == 0 ? oW2 : oW3;
      wp[i] = c < HID ? f2bf(theta[base + row * HID + packed_feature((int)c)]) : (unsigned short)0;
    } else if (i < w1 + 2 * w2 + w4) {
      const long jj = i - w1 - 2 * w2, row = jj / kWLd, c = jj % kWLd;
      wp[i] = row < no && c < HID ? f2bf(theta[oW4 + row * HID + packed_feature((int)c)])
                                  : (unsigned short)0;
    } else {
      const long b = i - (w1 + 2 * w2 + w4);
      float v;
      if (b < HID) v = theta[ob1 + b];
      else if (b < 2 * HID) v = theta[ob2 + b - HID];
      else if (b < 3 * HID) v = theta[ob3 + b - 2 * HID];
      else v = (b - 3 * HID) < no ? theta[ob4 + b - 3 * HID] : 0.f;
      bp[b] = v;
    }
  }
}

struct InferArgs {
  double* state; long ld; long n; double dt;
  const unsigned short* wpack; const float* bpack;
  const float* norm;            // mu_in[ni] sd_in[ni] mu_out[no] sd_out[no] zmin[ni] zmax[ni]
  const double* isd;            // 1 / sd_in (0 where sd_in is 0), FP64
  double hull_margin, elem_tol, pos_tol, energy_tol;
  int32_t* fb_list; unsigned* fb_count;
  int32_t* trust_code; float* out_std;
};

enum { TRUST_HULL = 1, TRUST_ELEM = 2, TRUST_POS = 4, TRUST_ENERGY = 8, TRUST_NONFINITE = 16 };

// LDS of one inference block: the packed weights and biases (shared), then
// one staging area per wave with one row per cell of the wave's 64: first
// the cell's BF16 features, later (once they are in registers) its FP32
// network outputs.  The row length CELL_B is an odd number of 16-byte
// chunks, so the 16-byte reads and writes of 16 consecutive cells fall on
// distinct banks.  The MLP runs on the 64 cells in two halves of 32, which
// halves the accumulator registers (64 per lane instead of 128) at the
// price of reading every weight twice per tile; with the lower register
// count three waves share each SIMD instead of two.
template <class M>
struct InferShape {
  static constexpr int NS = M::NS, NI = NS + 3, NO = NS + 1;
  static constexpr int KC1 = (NI + 31) / 32, OT4 = (NO + 15) / 16;
  static constexpr int W1_LD = w1_ld(KC1);
  static constexpr long W1 = (long)HID * W1_LD, W2 = (long)HID * kWLd, W4 = (long)OT4 * 16 * kWLd;
  static constexpr long WTOT = W1 + 2 * W2 + W4;
  static constexpr long BTOT = 3 * HID + OT4 * 16;
  static constexpr int F_CHUNKS = KC1 * 4, O_CHUNKS = OT4 * 4;     // 16-byte chunks per cell
  static constexpr int CELL_CHUNKS = (F_CHUNKS > O_CHUNKS ? F_CHUNKS : O_CHUNKS) | 1;
  static constexpr int CELL_B = CELL_CHUNKS * 16;
  static constexpr long STAGE = 64L * CELL_B;                         // bytes per wave
  static constexpr long F_OFF = WTOT * 2 + BTOT * 4;
  static constexpr int WAVES = NS <= 15 ? 12 : 4, THREADS = WAVES * 64;
  static constexpr long BYTES = F_OFF + WAVES * STAGE;
  static_assert(WTOT % 8 == 0 && F_OFF % 16 == 0, "16-byte LDS alignment");
  static_assert(BYTES <= 160 * 1024, "inference block exceeds the LDS");
};

// Orders this wave's LDS writes before its later LDS reads of other lanes'
// data (a wave executes in lockstep; this keeps the compiler from moving
// the accesses across the hand-off).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Append this wave's cells with `fall` set to the fallback list (when there
// is one): one atomic per wave, positions in lane order.
__device__ __forceinline__ void append_fallback(const InferArgs& a, bool fall, int lane, long cell) {
  if (!a.fb_list) return;
  const unsigned long long ball = __ballot(fall);
  if (!ball) return;
  const int leader = __ffsll((long long)ball) - 1;
  unsigned base_idx = 0;
  if (lane == leader) base_idx = atomicAdd(a.fb_count, (unsigned)__popcll(ball));
  base_idx = __shfl(base_idx, leader);
  if (fall) a.fb_list[base_idx + __popcll(ball & ((1ull << lane) - 1ull))] = (int32_t)cell;
}

// Fused inference: FP64 features -> BF16 MFMA MLP (weights in LDS, shared by
// the block; hidden activations never leave registers) -> FP64 trust test ->
// either the new state or an entry in the fallback list for the FP64
// integrator.  Each wave runs its own 64-cell tiles through all stages with
// wave-private LDS staging, so waves overlap their FP64 and MFMA phases.
template <class M>
__global__ __launch_bounds__(InferShape<M>::THREADS) void surr_infer(InferArgs a) {
  using S = InferShape<M>;
  constexpr int NS = S::NS, NI = S::NI, NO = S::NO, KC1 = S::KC1, OT4 = S::OT4;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  unsigned short* sW = reinterpret_cast<unsigned short*>(smem);
  const unsigned short* sW1 = sW;
  const unsigned short* sW2 = sW + S::W1;
  const unsigned short* sW3 = sW2 + S::W2;
  const unsigned short* sW4 = sW3 + S::W2;
  float* sB = reinterpret_cast<float*>(smem + S::WTOT * 2);
  if (a.n <= 0) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, r16 = lane & 15;
  unsigned char* stage = smem + S::F_OFF + wave * S::STAGE;
  {
    const uint4* src = reinterpret_cast<const uint4*>(a.wpack);
    uint4* dst = reinterpret_cast<uint4*>(sW);
    for (long i = tid; i < S::WTOT / 8; i += blockDim.x) dst[i] = src[i];
    for (long i = tid; i < S::BTOT; i += blockDim.x) sB[i] = a.bpack[i];
  }
  __syncthreads();
  const float* mu_in = a.norm;
  const float* sd_in = a.norm + NI;
  const float* mu_out = a.norm + 2 * NI;
  const float* sd_out = a.norm + 2 * NI + NO;
  const float* zmin = a.norm + 2 * NI + 2 * NO;
  const float* zmax = zmin + NI;

  const double ln_dt = log(a.dt);
  const long ntiles = (a.n + 63) / 64;
  for (long tile = (long)blockIdx.x * S::WAVES + wave; tile < ntiles;
       tile += (long)gridDim.x * S::WAVES) {
    const long cell = tile * 64 + lane;
    const bool valid = cell < a.n;
    int code = 0;
    // ---- stage 0: this lane's cell features (FP64), standardised, BF16 to LDS
    {
      double f[NI];
#pragma unroll
      for (int k = 0; k < NI; ++k) f[k] = 0.0;
      if (valid) {
        const double T = a.state[cell];
        double sy = 0.0;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const double y = a.state[(k + 1) * a.ld + cell];
          f[3 + k] = y;
          sy += y * (1.0 / M::W[k]);
        }
        const double rho = a.state[(NS + 1) * a.ld + cell];
        f[0] = T;
        f[1] = log(rho * 8.31446261815324e7 * T * sy);
        f[2] = ln_dt;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
          const double z = sd_in[k] > 0.f ? (f[k] - (double)mu_in[k]) * a.isd[k] : 0.0;
          if (!(z >= (double)zmin[k] - a.hull_margin && z <= (double)zmax[k] + a.hull_margin))
            code |= TRUST_HULL;
          f[k] = z;
        }
      }
      // this lane's row of the staging area: its features, zero-padded,
      // as 16-byte stores
#pragma unroll
      for (int q = 0; q < KC1 * 4; ++q) {
        v8s v;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int k = 8 * q + j;
          v[j] = (short)((valid && k < NI) ? d2bf(f[k < NI ? k : 0]) : (unsigned short)0);
        }
        *reinterpret_cast<v8s*>(stage + lane * S::CELL_B + 16 * q) = v;
      }
    }
    // with a fallback, a cell outside the hull is decided by that criterion
    // alone (code TRUST_HULL); a tile of such cells skips the network
    const bool decided = a.fb_list && (code & TRUST_HULL);
    if (!__any(valid && !decided)) {
      if (valid && a.trust_code) a.trust_code[cell] = code;
      append_fallback(a, valid, lane, cell);
      wave_sync();
      continue;
    }
    wave_sync();
    // ---- stage 1: the MLP on this wave's 64 cells, in two halves of 32
    // (two column tiles of 16 each).  Each layer's bias is the C operand of
    // its first MFMA of every output tile, so the accumulators start from
    // the bias instead of zero.
#pragma unroll 1
    for (int half = 0; half < 2; ++half) {
      unsigned char* hs = stage + half * 32 * S::CELL_B;
      f32x4 acc[8][2];
      v8s bn[4][2];
#pragma unroll
      for (int kc = 0; kc < KC1; ++kc) {
        v8s b1[2];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
          b1[ct] = *reinterpret_cast<const v8s*>(hs + (ct * 16 + r16) * S::CELL_B + kc * 64 + 16 * g);
#pragma unroll
        for (int ot = 0; ot < 8; ++ot) {
          const v8s aw = *reinterpret_cast<const v8s*>(sW1 + (ot * 16 + r16) * S::W1_LD + kc * 32 + 8 * g);
          f32x4 bv;
          if (kc == 0) bv = *reinterpret_cast<const f32x4*>(sB + ot * 16 + 4 * g);
#pragma unroll
          for (int ct = 0; ct < 2; ++ct) acc[ot][ct] = mfma(aw, b1[ct], kc == 0 ? bv : acc[ot][ct]);
        }
      }
#pragma unroll
      for (int layer = 0; layer < 3; ++layer) {
#pragma unroll
        for (int kc = 0; kc < 4; ++kc)
#pragma unroll
          for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const int ot = 2 * kc + (j >> 2), i = j & 3;
              bn[kc][ct][j] = (short)f2bf(silu_fast(acc[ot][ct][i]));
            }
        if (layer == 2) break;
        const unsigned short* Wl = layer == 0 ? sW2 : sW3;
        const float* bias = sB + (layer + 1) * HID;
#pragma unroll
        for (int kc = 0; kc < 4; ++kc)
#pragma unroll
          for (int ot = 0; ot < 8; ++ot) {
            const v8s aw = *reinterpret_cast<const v8s*>(Wl + (ot * 16 + r16) * kWLd + kc * 32 + 8 * g);
            f32x4 bv;
            if (kc == 0) bv = *reinterpret_cast<const f32x4*>(bias + ot * 16 + 4 * g);
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
              acc[ot][ct] = mfma(aw, bn[kc][ct], kc == 0 ? bv : acc[ot][ct]);
          }
      }
      f32x4 acc4[OT4][2];
#pragma unroll
      for (int kc = 0; kc < 4; ++kc)
#pragma unroll
        for (int ot = 0; ot < OT4; ++ot) {
          const v8s aw = *reinterpret_cast<const v8s*>(sW4 + (ot * 16 + r16) * kWLd + kc * 32 + 8 * g);
          f32x4 bv;
          if (kc == 0) bv = *reinterpret_cast<const f32x4*>(sB + 3 * HID + ot * 16 + 4 * g);
#pragma unroll
          for (int ct = 0; ct < 2; ++ct)
            acc4[ot][ct] = mfma(aw, bn[kc][ct], kc == 0 ? bv : acc4[ot][ct]);
        }
      // outputs 16 ot + 4 g + (0..3) of cell 16 ct + r16, over that cell's
      // features (already in registers: the MFMAs above consumed them)
#pragma unroll
      for (int ot = 0; ot < OT4; ++ot)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
          *reinterpret_cast<f32x4*>(hs + (ct * 16 + r16) * S::CELL_B + ot * 64 + 16 * g) = acc4[ot][ct];
    }
    wave_sync();
    // ---- stage 2: de-standardise and trust-test this lane's cell (FP64)
    bool fall = false;
    if (valid && decided) {
      if (a.trust_code) a.trust_code[cell] = code;
      fall = true;
    } else if (valid) {
      double inc[NO];
      bool fin = true;
#pragma unroll
      for (int k = 0; k < NO; ++k) {
        const float o = reinterpret_cast<const float*>(stage + lane * S::CELL_B)[k];
        if (a.out_std) a.out_std[cell * NO + k] = o;
        inc[k] = (double)o * (double)sd_out[k] + (double)mu_out[k];
        fin = fin && isfinite(inc[k]);
      }
      const double T = a.state[cell];
      double Y[NS], Y1[NS];
      double ymin = 1e300;
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        Y[k] = a.state[(k + 1) * a.ld + cell];
        Y1[k] = Y[k] + inc[1 + k];
        ymin = Y1[k] < ymin ? Y1[k] : ymin;
      }
      const double T1 = T + inc[0];
      if (!fin) {
        code |= TRUST_NONFINITE;
      } else {
#pragma unroll
        for (int e = 0; e < M::NE; ++e) {
          double s = 0.0;
#pragma unroll
          for (int k = 0; k < NS; ++k) s += M::ELEM[e][k] * (Y1[k] - Y[k]);
          if (fabs(s) > a.elem_tol) code |= TRUST_ELEM;
        }
        if (ymin < -a.pos_tol) code |= TRUST_POS;
        double e0, cv0, e1, cv1;
        M::energy_cv(T, Y, e0, cv0);
        M::energy_cv(T1, Y1, e1, cv1);
        if (!(fabs(e1 - e0) / cv0 <= a.energy_tol)) code |= TRUST_ENERGY;
      }
      if (a.trust_code) a.trust_code[cell] = code;
      if (code == 0) {
        // a trusted cell's Y + dY >= -pos_tol; what lies below zero is
        // written as zero, so no negative mass fraction reaches the state
        a.state[cell] = T1;
#pragma unroll
        for (int k = 0; k < NS; ++k) a.state[(k + 1) * a.ld + cell] = fmax(Y1[k], 0.0);
      } else {
        fall = true;
      }
    }
    append_fallback(a, fall, lane, cell);
    wave_sync();
  }
}

// raw features and increments of (state_before -> state_after) pairs
template <class M>
__global__ void make_pairs(const double* before, const double* after, long ld, long n, double dt,
                           const double* dt_cells, float* X, float* Yd) {
  constexpr int NS = M::NS, NI = NS + 3, NO = NS + 1;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double T = before[i];
  double sy = 0.0;
  for (int k = 0; k < NS; ++k) {
    const double y = before[(k + 1) * ld + i];
    sy += y * (1.0 / M::W[k]);
    X[i * NI + 3 + k] = (float)y;
    Yd[i * NO + 1 + k] = (float)(after[(k + 1) * ld + i] - y);
  }
  const double rho = before[(NS + 1) * ld + i];
  X[i * NI + 0] = (float)T;
  X[i * NI + 1] = (float)log(rho * 8.31446261815324e7 * T * sy);
  X[i * NI + 2] = (float)log(dt_cells ? dt_cells[i] : dt);
  Yd[i * NO + 0] = (float)(after[i] - T);
}

__global__ void zero_u32(unsigned* p) { *p = 0u; }

}  // namespace surr

template <class M>
hipError_t launch_surr_infer(const surr::InferArgs& a, int grid, hipStream_t s) {
  using S = surr::InferShape<M>;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)surr::surr_infer<M>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)S::BYTES);
    attr = true;
  }
  // at most `grid` blocks (one per CU), fewer when the cells do not fill them
  const long need = (a.n + S::THREADS - 1) / S::THREADS;
  grid = (int)(need < grid ? (need > 0 ? need : 1) : grid);
  hipLaunchKernelGGL(surr::surr_infer<M>, dim3(grid), dim3(S::THREADS), S::BYTES, s, a);
  return hipGetLastError();
}

template <class M>
hipError_t launch_make_pairs(const double* before, const double* after, long ld, long n, double dt,
                             const double* dt_cells, float* X, float* Y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(surr::make_pairs<M>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     before, after, ld, n, dt, dt_cells, X, Y);
  return hipGetLastError();
}
