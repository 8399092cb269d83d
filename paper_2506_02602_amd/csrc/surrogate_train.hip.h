// Training step of the surrogate MLP in three kernels per batch (BF16 MFMA,
// FP32 accumulation; the BF16 rounding points are those of the forward and
// backward passes the oracle emulates):
//
//   train_fwd  per 16-sample wave tile: gather the batch rows through the
//              epoch's permutation, the forward pass on the packed weights
//              in LDS (as the inference kernel), the loss and its gradient;
//              keeps what the backward pass needs: the pre-activations Z_l
//              in the wave's own register order, and the BF16 activations
//              H_l, inputs and output gradient feature-major (one row of
//              samples per feature);
//   train_bwd  per 16-sample wave tile: dZ_3, dZ_2, dZ_1 through the
//              transposed packed weights, each dZ_l = BF16(dH_l * silu'(Z_l)),
//              written feature-major;
//   train_dw   one block per 16 x 16 tile of a weight gradient: the
//              batch's dZ_l^T H_(l-1) as MFMA chains over the samples, split
//              over the block's waves and added in wave order (both operands
//              sample-contiguous rows), the bias gradient from
//              the same dZ rows, then either the gradient itself or the Adam
//              update of those parameters, written to the FP32 masters, the
//              BF16 natural copy and both packed layouts (no reduction or
//              repacking pass).
#pragma once

namespace surr {

// inverse of packed_feature: the packed column of hidden feature f
__host__ __device__ constexpr int packed_column(int f) {
  return (f & ~31) + (((f & 31) < 16) ? 8 * ((f & 15) >> 2) + (f & 3)
                                      : 8 * ((f & 15) >> 2) + 4 + (f & 3));
}

constexpr bool packed_column_inverts() {
  for (int c = 0; c < HID; ++c)
    if (packed_column(packed_feature(c)) != c) return false;
  return true;
}
static_assert(packed_column_inverts(), "packed_column is the inverse of packed_feature");

struct TrainArgs {
  // batch rows: sample s of the batch is row (pa ((first + s) mod n) + pb) mod n
  const float* Xn; const float* Yn; long n; long first; unsigned long long pa, pb;
  int B, Bp;                         // batch size, and rounded up to 32 (row stride)
  const unsigned short* wpack; const float* bpack;   // forward (inference) layout
  const unsigned short* wtpack;                      // transposed layout for dH = W^T dZ
  unsigned short* Xfm;               // [NI16][Bp] BF16 inputs, feature-major
  unsigned short* Hfm;               // [3][HID][Bp] BF16 activations
  float* Zd;                         // [3][Bp/TS][ZQ][64] pre-activations, register order
  unsigned short* dZfm;              // [3][HID][Bp] BF16 pre-activation gradients
  unsigned short* doutfm;            // [NO16][Bp] BF16 output gradient
  double* sse; float scale;          // sum of squared errors; 2 / (B NO)
  // train_dw
  float* theta; float* m; float* v; float* grad; unsigned short* wbf;
  unsigned short* wpack_w; float* bpack_w; unsigned short* wtpack_w;
  int adam; float lr, b1, b2, c1, c2, eps;
  long oW[4], ob[4];
};

template <class M>
struct TrainShape {
  using S = InferShape<M>;
  static constexpr int NI = S::NI, NO = S::NO, KC1 = S::KC1, OT4 = S::OT4;
  static constexpr int NI16 = (NI + 15) / 16 * 16, NO16 = OT4 * 16;
  static constexpr int KO = (NO + 31) / 32;            // k chunks of dH_3 = W4^T dout
  static constexpr int W4T_LD = KO * 32 + kRowPad;
  static constexpr long WT4 = (long)HID * W4T_LD, WT2 = (long)HID * kWLd;
  static constexpr long WTTOT = WT4 + 2 * WT2;         // [W4^T][W3^T][W2^T]
  // waves per block of train_fwd and train_bwd: each block loads the
  // weights into its LDS once, so more waves per block share that load
  // (8: 1.33 s for the benchmark's 12 epochs, 4: 1.41 s, 16: spills)
  static constexpr int WAVES = 8;
  // a wave takes CT column tiles of 16 samples (TS samples); its
  // pre-activations are ZQ floats per lane per layer
  static constexpr int CT = 1, TS = 16 * CT, ZQ = 8 * CT * 4;
  // train_fwd LDS: the inference weights and biases, then per wave the
  // TS cells' staging rows and their source rows
  static constexpr long F_STAGE = (long)TS * S::CELL_B + TS * 8;
  static constexpr long F_BYTES = S::F_OFF + WAVES * F_STAGE;
  static constexpr long B_BYTES = WTTOT * 2;
  static_assert(F_BYTES <= 160 * 1024 && B_BYTES <= 160 * 1024, "training block exceeds the LDS");
  // train_dw work items: (layer, out tile, in tile)
  static constexpr int IT1 = NI16 / 16, OTH = HID / 16, ITH = HID / 16;
  static constexpr int N1 = OTH * IT1, N2 = OTH * ITH, N4 = OT4 * ITH;
  static constexpr int ITEMS = N1 + 2 * N2 + N4;
};

__device__ __forceinline__ float dsilu_fast(float z) {
  const float s = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
  return s * (1.0f + z * (1.0f - s));
}

__device__ __forceinline__ long batch_row(const TrainArgs& a, int s) {
  const unsigned long long idx = (unsigned long long)(a.first + s);
  return (long)((a.pa * (idx % (unsigned long long)a.n) + a.pb) % (unsigned long long)a.n);
}

template <class M>
__global__ __launch_bounds__(64 * TrainShape<M>::WAVES) void train_fwd(TrainArgs a) {
  using T = TrainShape<M>;
  using S = typename T::S;
  constexpr int NI = T::NI, NO = T::NO, KC1 = T::KC1, OT4 = T::OT4;
  constexpr int CT = T::CT, TS = T::TS, ZQ = T::ZQ;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  unsigned short* sW = reinterpret_cast<unsigned short*>(smem);
  const unsigned short* sW1 = sW;
  const unsigned short* sW2 = sW + S::W1;
  const unsigned short* sW3 = sW2 + S::W2;
  const unsigned short* sW4 = sW3 + S::W2;
  float* sB = reinterpret_cast<float*>(smem + S::WTOT * 2);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, r16 = lane & 15;
  unsigned char* hs = smem + S::F_OFF + wave * T::F_STAGE;
  long* srow = reinterpret_cast<long*>(hs + (long)TS * S::CELL_B);
  {
    const uint4* src = reinterpret_cast<const uint4*>(a.wpack);
    uint4* dst = reinterpret_cast<uint4*>(sW);
    for (long i = tid; i < S::WTOT / 8; i += blockDim.x) dst[i] = src[i];
    for (long i = tid; i < S::BTOT; i += blockDim.x) sB[i] = a.bpack[i];
  }
  __syncthreads();
  const int tile = blockIdx.x * T::WAVES + wave;
  const int s0 = tile * TS;
  if (s0 >= a.Bp) return;
  // ---- the wave's TS samples: inputs to the staging rows (BF16) and to Xfm
  if (lane < TS) {
    const int s = s0 + lane;
    const bool in = s < a.B;
    const long row = in ? batch_row(a, s) : 0;
    srow[lane] = row;
#pragma unroll
    for (int q = 0; q < KC1 * 4; ++q) {
      v8s v;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = 8 * q + j;
        v[j] = (short)((in && k < NI) ? f2bf(a.Xn[row * NI + k]) : (unsigned short)0);
      }
      *reinterpret_cast<v8s*>(hs + lane * S::CELL_B + 16 * q) = v;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (8 * q + j < T::NI16) (a.Xfm + (long)(8 * q + j) * a.Bp)[s] = (unsigned short)v[j];
    }
  }
  wave_sync();
  // this lane's targets for the loss, loaded now: a load issued after the
  // activation stores below would wait for all of them
  float yv[OT4][CT][4];
#pragma unroll
  for (int ot = 0; ot < OT4; ++ot)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int o = ot * 16 + 4 * g + i, c = ct * 16 + r16;
        yv[ot][ct][i] = (o < NO && s0 + c < a.B) ? a.Yn[srow[c] * NO + o] : 0.f;
      }
  f32x4 acc[8][CT];
  v8s bn[4][CT];
#pragma unroll
  for (int kc = 0; kc < KC1; ++kc) {
    v8s b1[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
      b1[ct] = *reinterpret_cast<const v8s*>(hs + (ct * 16 + r16) * S::CELL_B + kc * 64 + 16 * g);
#pragma unroll
    for (int ot = 0; ot < 8; ++ot) {
      const v8s aw = *reinterpret_cast<const v8s*>(sW1 + (ot * 16 + r16) * S::W1_LD + kc * 32 + 8 * g);
      f32x4 bv;
      if (kc == 0) bv = *reinterpret_cast<const f32x4*>(sB + ot * 16 + 4 * g);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[ot][ct] = mfma(aw, b1[ct], kc == 0 ? bv : acc[ot][ct]);
    }
  }
  float* zd = a.Zd + (long)tile * ZQ * 64;
  // a feature-major row is a uniform pointer (feature 16 ot + i) plus this
  // lane's offset (its group's 4 g rows further, its cell's column)
  const int loff = 4 * g * a.Bp + s0 + r16;
#pragma unroll
  for (int layer = 0; layer < 3; ++layer) {
    float* zl = zd + (long)layer * (a.Bp / TS) * ZQ * 64;
    unsigned short* hl = a.Hfm + (long)layer * HID * a.Bp;
#pragma unroll
    for (int kc = 0; kc < 4; ++kc)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int ot = 2 * kc + (j >> 2), i = j & 3;
          const float z = acc[ot][ct][i];
          (zl + ((ot * CT + ct) * 4 + i) * 64)[lane] = z;
          const unsigned short h = s0 + ct * 16 + r16 < a.B ? f2bf(silu_fast(z)) : (unsigned short)0;
          bn[kc][ct][j] = (short)h;
          (hl + (long)(ot * 16 + i) * a.Bp)[loff + ct * 16] = h;
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
        for (int ct = 0; ct < CT; ++ct) acc[ot][ct] = mfma(aw, bn[kc][ct], kc == 0 ? bv : acc[ot][ct]);
      }
  }
  f32x4 acc4[OT4][CT];
#pragma unroll
  for (int kc = 0; kc < 4; ++kc)
#pragma unroll
    for (int ot = 0; ot < OT4; ++ot) {
      const v8s aw = *reinterpret_cast<const v8s*>(sW4 + (ot * 16 + r16) * kWLd + kc * 32 + 8 * g);
      f32x4 bv;
      if (kc == 0) bv = *reinterpret_cast<const f32x4*>(sB + 3 * HID + ot * 16 + 4 * g);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc4[ot][ct] = mfma(aw, bn[kc][ct], kc == 0 ? bv : acc4[ot][ct]);
    }
  // ---- loss and its gradient dL/dout = 2 (out - y) / (B NO), BF16
  double se = 0.0;
#pragma unroll
  for (int ot = 0; ot < OT4; ++ot)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int o = ot * 16 + 4 * g + i, c = ct * 16 + r16, s = s0 + c;
        unsigned short d16 = 0;
        if (o < NO && s < a.B) {
          const float d = acc4[ot][ct][i] - yv[ot][ct][i];
          d16 = f2bf(a.scale * d);
          se += (double)d * d;
        }
        (a.doutfm + (long)(ot * 16 + i) * a.Bp)[loff + ct * 16] = d16;
      }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) se += __shfl_xor(se, off);
  if (lane == 0) atomicAdd(a.sse, se);
}

template <class M>
__global__ __launch_bounds__(64 * TrainShape<M>::WAVES) void train_bwd(TrainArgs a) {
  using T = TrainShape<M>;
  constexpr int NO = T::NO, KO = T::KO;
  constexpr int CT = T::CT, TS = T::TS, ZQ = T::ZQ;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  unsigned short* sT = reinterpret_cast<unsigned short*>(smem);
  const unsigned short* sT4 = sT;                  // W4^T [HID][W4T_LD]
  const unsigned short* sT3 = sT + T::WT4;         // W3^T, packed columns
  const unsigned short* sT2 = sT3 + T::WT2;        // W2^T, packed columns
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, r16 = lane & 15;
  {
    const uint4* src = reinterpret_cast<const uint4*>(a.wtpack);
    uint4* dst = reinterpret_cast<uint4*>(sT);
    for (long i = tid; i < T::WTTOT / 8; i += blockDim.x) dst[i] = src[i];
  }
  __syncthreads();
  const int tile = blockIdx.x * T::WAVES + wave;
  const int s0 = tile * TS;
  if (s0 >= a.Bp) return;
  f32x4 acc[8][CT];
  v8s bz[4][CT];
  // this wave's pre-activations of the current and the next layer, in the
  // register order the forward kernel stored them
  const float* zd = a.Zd + (long)tile * ZQ * 64;
  float zcur[ZQ], znext[ZQ];
  {
    const float* z3 = zd + 2L * (a.Bp / TS) * ZQ * 64;
#pragma unroll
    for (int q = 0; q < ZQ; ++q) zcur[q] = (z3 + q * 64)[lane];
  }
  // dH_3 = W4^T dout: the output gradient as the B operand (k = output)
#pragma unroll
  for (int ot = 0; ot < 8; ++ot)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ot][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kc = 0; kc < KO; ++kc) {
    v8s bo[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int o = kc * 32 + 8 * g + j;
        bo[ct][j] = o < NO ? (short)(a.doutfm + (long)(kc * 32 + j) * a.Bp)[8 * g * a.Bp + s0 + ct * 16 + r16]
                           : (short)0;
      }
#pragma unroll
    for (int ot = 0; ot < 8; ++ot) {
      const v8s aw = *reinterpret_cast<const v8s*>(sT4 + (ot * 16 + r16) * T::W4T_LD + kc * 32 + 8 * g);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[ot][ct] = mfma(aw, bo[ct], acc[ot][ct]);
    }
  }
  const int loff = 4 * g * a.Bp + s0 + r16;
#pragma unroll
  for (int layer = 2; layer >= 0; --layer) {
    unsigned short* dzl = a.dZfm + (long)layer * HID * a.Bp;
    // the next layer's pre-activations are loaded before this layer's
    // gradient stores: a load issued after stores would wait for them too
    // (one counter covers both), a load issued before them does not
    if (layer > 0) {
      const float* zn = zd + (long)(layer - 1) * (a.Bp / TS) * ZQ * 64;
#pragma unroll
      for (int q = 0; q < ZQ; ++q) znext[q] = (zn + q * 64)[lane];
    }
    // dZ_l = BF16(dH_l * silu'(Z_l)), in the next product's B-operand order
#pragma unroll
    for (int kc = 0; kc < 4; ++kc)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int ot = 2 * kc + (j >> 2), i = j & 3;
          const float z = zcur[(ot * CT + ct) * 4 + i];
          const unsigned short dz =
              s0 + ct * 16 + r16 < a.B ? f2bf(acc[ot][ct][i] * dsilu_fast(z)) : (unsigned short)0;
          bz[kc][ct][j] = (short)dz;
          (dzl + (long)(ot * 16 + i) * a.Bp)[loff + ct * 16] = dz;
        }
    if (layer == 0) break;
    // dH_(l-1) = W_l^T dZ_l
    const unsigned short* Wt = layer == 2 ? sT3 : sT2;
#pragma unroll
    for (int ot = 0; ot < 8; ++ot)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[ot][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc)
#pragma unroll
      for (int ot = 0; ot < 8; ++ot) {
        const v8s aw = *reinterpret_cast<const v8s*>(Wt + (ot * 16 + r16) * kWLd + kc * 32 + 8 * g);
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[ot][ct] = mfma(aw, bz[kc][ct], acc[ot][ct]);
      }
#pragma unroll
    for (int q = 0; q < ZQ; ++q) zcur[q] = znext[q];
  }
}

// Adam on one FP32 master parameter (the moment decay rates and the bias
// corrections as FP32 numbers); returns the new value
__device__ __forceinline__ float adam_one(const TrainArgs& a, long p, float gr) {
  const float mi = a.b1 * a.m[p] + (1.f - a.b1) * gr;
  const float vi = a.b2 * a.v[p] + (1.f - a.b2) * gr * gr;
  a.m[p] = mi;
  a.v[p] = vi;
  const float th = a.theta[p] - a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + a.eps);
  a.theta[p] = th;
  return th;
}

constexpr int kDwWaves = 16;

template <class M>
__global__ __launch_bounds__(64 * kDwWaves) void train_dw(TrainArgs a) {
  using T = TrainShape<M>;
  using S = typename T::S;
  constexpr int NI = T::NI, NO = T::NO;
  __shared__ float red[kDwWaves][5][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, r16 = lane & 15;
  // one block per item: layer l (0-based: W1..W4), out tile ot, in tile it
  int item = blockIdx.x;
  int l, ot, it;
  if (item < T::N1) { l = 0; ot = item / T::IT1; it = item % T::IT1; }
  else if ((item -= T::N1) < 2 * T::N2) { l = 1 + item / T::N2; item %= T::N2; ot = item / T::ITH; it = item % T::ITH; }
  else { item -= 2 * T::N2; l = 3; ot = item / T::ITH; it = item % T::ITH; }
  const int out_dim = l == 3 ? NO : HID, in_dim = l == 0 ? NI : HID;
  const unsigned short* A = l == 3 ? a.doutfm : a.dZfm + (long)l * HID * a.Bp;     // [out][Bp]
  const unsigned short* Bm = l == 0 ? a.Xfm : a.Hfm + (long)(l - 1) * HID * a.Bp;  // [in][Bp]
  const unsigned short* arow = A + (long)(ot * 16 + r16) * a.Bp + 8 * g;
  const unsigned short* brow = Bm + (long)(it * 16 + r16) * a.Bp + 8 * g;
  // the waves split the samples; each sums its share, the first wave adds
  // the shares in wave order
  const int per = (a.Bp / 32 + kDwWaves - 1) / kDwWaves * 32;
  const int kb = wave * per, ke = min(kb + per, a.Bp);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  const bool bias_tile = it == 0;
#pragma unroll 4
  for (int k0 = kb; k0 < ke; k0 += 32) {
    const v8s av = *reinterpret_cast<const v8s*>(arow + k0);
    const v8s bv = *reinterpret_cast<const v8s*>(brow + k0);
    acc = mfma(av, bv, acc);
    if (bias_tile) {
#pragma unroll
      for (int j = 0; j < 8; ++j) bsum += bf2f((unsigned short)av[j]);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) red[wave][i][lane] = acc[i];
  red[wave][4][lane] = bsum;
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = red[0][i][lane];
  bsum = red[0][4][lane];
  for (int w = 1; w < kDwWaves; ++w) {
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += red[w][i][lane];
    bsum += red[w][4][lane];
  }
  // D[4g + i][r16] = dW[out = 16 ot + 4g + i][in = 16 it + r16]
  const long oWl = a.oW[l];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int o = ot * 16 + 4 * g + i, in = it * 16 + r16;
    if (o >= out_dim || in >= in_dim) continue;
    const long p = oWl + (long)o * in_dim + in;
    if (!a.adam) { a.grad[p] = acc[i]; continue; }
    const float th = adam_one(a, p, acc[i]);
    const unsigned short b16 = f2bf(th);
    a.wbf[p] = b16;
    // the forward (inference) layout and the transposed backward one
    if (l == 0) {
      a.wpack_w[(long)o * S::W1_LD + in] = b16;
    } else {
      a.wpack_w[S::W1 + (long)(l - 1) * S::W2 + (long)o * kWLd + packed_column(in)] = b16;
      if (l == 3) a.wtpack_w[(long)in * T::W4T_LD + o] = b16;
      else a.wtpack_w[T::WT4 + (long)(2 - l) * T::WT2 + (long)in * kWLd + packed_column(o)] = b16;
    }
  }
  if (bias_tile) {
    // the four lanes of one out row (g = 0..3) hold its partial sums
    bsum += __shfl_xor(bsum, 16);
    bsum += __shfl_xor(bsum, 32);
    const int o = ot * 16 + r16;
    if (g == 0 && o < out_dim) {
      const long p = a.ob[l] + o;
      if (!a.adam) {
        a.grad[p] = bsum;
      } else {
        const float th = adam_one(a, p, bsum);
        a.wbf[p] = f2bf(th);
        a.bpack_w[l * HID + o] = th;
      }
    }
  }
}

// theta -> the transposed backward layout (initial packing; the training
// step keeps it current for the parameters it updates)
__global__ void pack_transposed(const float* theta, int ni, int no, long oW2, long oW3, long oW4,
                                int w4t_ld, long wt4, long wt2, unsigned short* wt) {
  const long total = wt4 + 2 * wt2;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x) {
    unsigned short v = 0;
    if (i < wt4) {
      const long in = i / w4t_ld, o = i % w4t_ld;
      if (o < no) v = f2bf(theta[oW4 + o * HID + in]);
    } else {
      const long j = i - wt4, which = j / wt2, jj = j % wt2, in = jj / kWLd, c = jj % kWLd;
      const long base = which == 0 ? oW3 : oW2;
      if (c < HID) v = f2bf(theta[base + (long)packed_feature((int)c) * HID + in]);
    }
    wt[i] = v;
  }
}

}  // namespace surr

template <class M>
hipError_t launch_train(const surr::TrainArgs& a, int phase, hipStream_t s) {
  using T = surr::TrainShape<M>;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)surr::train_fwd<M>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)T::F_BYTES);
    (void)hipFuncSetAttribute((const void*)surr::train_bwd<M>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)T::B_BYTES);
    attr = true;
  }
  const unsigned tiles = (unsigned)(a.Bp / T::TS);
  const unsigned blocks = (tiles + T::WAVES - 1) / T::WAVES;
  if (phase == 0)
    hipLaunchKernelGGL(surr::train_fwd<M>, dim3(blocks), dim3(64 * T::WAVES), T::F_BYTES, s, a);
  else if (phase == 1)
    hipLaunchKernelGGL(surr::train_bwd<M>, dim3(blocks), dim3(64 * T::WAVES), T::B_BYTES, s, a);
  else
    hipLaunchKernelGGL(surr::train_dw<M>, dim3(T::ITEMS), dim3(64 * surr::kDwWaves), 0, s, a);
  return hipGetLastError();
}

template <class M>
struct TrainSizes {
  using T = surr::TrainShape<M>;
  static constexpr long wtpack_elems = T::WTTOT;
  static constexpr int ni16 = T::NI16, no16 = T::NO16, w4t_ld = T::W4T_LD;
  static constexpr long wt4 = T::WT4, wt2 = T::WT2;
};
