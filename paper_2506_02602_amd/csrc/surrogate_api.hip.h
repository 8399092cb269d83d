// Host side of the learned surrogate: the chem_surr handle and its C ABI.
#pragma once

struct chem_surr_s {
  chem_mech mech = nullptr;
  int ni = 0, no = 0;
  long P = 0;
  long oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0, oW4 = 0, ob4 = 0;
  float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
  unsigned short* wbf = nullptr;          // BF16 copy of theta (natural layout)
  float* norm = nullptr;                  // mu_in sd_in mu_out sd_out zmin zmax
  bool norm_set = false;
  unsigned short* wpack = nullptr;        // inference layout
  float* bpack = nullptr;
  double* isd = nullptr;                  // 1 / input scale, FP64 (inference)
  bool packed = false;
  long adam_t = 0;
  // training data (standardised) and per-batch buffers
  float *Xn = nullptr, *Yn = nullptr;
  long ncap = 0;
  int bcap = 0;
  // the generic forward's batch (surrogate_forward)
  unsigned short *X0 = nullptr, *H1 = nullptr, *H2 = nullptr, *H3 = nullptr;
  float *Z1 = nullptr, *Z2 = nullptr, *Z3 = nullptr, *out = nullptr, *Yb = nullptr;
  // the training step's batch (rows padded to a multiple of 32 samples)
  int tcap = 0;
  unsigned short *Xfm = nullptr, *Hfm = nullptr, *dZfm = nullptr, *doutfm = nullptr;
  float* Zd = nullptr;
  unsigned short* wtpack = nullptr;       // transposed packed weights (backward)
  float* fwd_tmp = nullptr;               // surrogate_forward's standardised chunk
  double* sse = nullptr;
  // the fallback list: the cells failing the trust test, appended by the
  // inference kernel; one pool of the FP64 integrator takes the whole list
  // (allocated by surrogate_reserve; surrogate_infer allocates nothing)
  int32_t* fb_list = nullptr;
  unsigned* fb_count = nullptr;
  int64_t reserved = 0;
};

namespace {

uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double uniform01(uint64_t& x) { return (splitmix64(x) >> 11) * (1.0 / 9007199254740992.0); }

template <class T>
hipError_t dalloc(T** p, long count) {
  *p = nullptr;
  return hipMalloc(p, sizeof(T) * (size_t)(count > 0 ? count : 1));
}

void surr_free_batch(chem_surr s) {
  for (void* p : {(void*)s->X0, (void*)s->H1, (void*)s->H2, (void*)s->H3, (void*)s->Z1,
                  (void*)s->Z2, (void*)s->Z3, (void*)s->out, (void*)s->Yb, (void*)s->fwd_tmp,
                  (void*)s->Xfm, (void*)s->Hfm, (void*)s->dZfm, (void*)s->doutfm, (void*)s->Zd})
    if (p) (void)hipFree(p);
  s->X0 = s->H1 = s->H2 = s->H3 = nullptr;
  s->Z1 = s->Z2 = s->Z3 = s->out = s->Yb = s->fwd_tmp = nullptr;
  s->Xfm = s->Hfm = s->dZfm = s->doutfm = nullptr;
  s->Zd = nullptr;
  s->bcap = 0;
  s->tcap = 0;
}

// The training step's buffers for batches of up to B samples.
int surr_ensure_train(chem_surr s, int B) {
  const int Bp = (B + 31) / 32 * 32;
  if (Bp <= s->tcap) return CHEM_OK;
  for (void* p : {(void*)s->Xfm, (void*)s->Hfm, (void*)s->dZfm, (void*)s->doutfm, (void*)s->Zd})
    if (p) (void)hipFree(p);
  s->Xfm = s->Hfm = s->dZfm = s->doutfm = nullptr;
  s->Zd = nullptr;
  s->tcap = 0;
  const long H = surr::HID;
  const int ni16 = (s->ni + 15) / 16 * 16, no16 = (s->no + 15) / 16 * 16;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) { if (e == hipSuccess) e = r; };
  A(dalloc(&s->Xfm, (long)ni16 * Bp));
  A(dalloc(&s->Hfm, 3 * H * Bp));
  A(dalloc(&s->dZfm, 3 * H * Bp));
  A(dalloc(&s->doutfm, (long)no16 * Bp));
  A(dalloc(&s->Zd, 3 * H * Bp));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(surrogate training batch)");
  s->tcap = Bp;
  return CHEM_OK;
}

int surr_ensure_batch(chem_surr s, int B) {
  if (B <= s->bcap) return CHEM_OK;
  surr_free_batch(s);
  const long H = surr::HID;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) { if (e == hipSuccess) e = r; };
  A(dalloc(&s->X0, (long)B * s->ni));
  A(dalloc(&s->H1, (long)B * H)); A(dalloc(&s->H2, (long)B * H)); A(dalloc(&s->H3, (long)B * H));
  A(dalloc(&s->Z1, (long)B * H)); A(dalloc(&s->Z2, (long)B * H)); A(dalloc(&s->Z3, (long)B * H));
  A(dalloc(&s->out, (long)B * s->no)); A(dalloc(&s->Yb, (long)B * s->no));
  A(dalloc(&s->fwd_tmp, (long)B * s->ni));
  if (e != hipSuccess) { surr_free_batch(s); return hip_fail(e, "hipMalloc(surrogate batch)"); }
  s->bcap = B;
  return CHEM_OK;
}

template <int EPI>
hipError_t gemm(surr::GemmArgs g, int splits, hipStream_t st) {
  if (splits < 1) splits = 1;
  g.kper = ((g.K + splits - 1) / splits + 31) / 32 * 32;
  const long tiles = (long)((g.M + 15) / 16) * ((g.N + 15) / 16);
  hipLaunchKernelGGL(surr::gemm_bf16<EPI>, dim3((unsigned)((tiles + 3) / 4), 1, splits), dim3(256),
                     0, st, g);
  return hipGetLastError();
}

surr::GemmArgs gargs(const unsigned short* A, long sam, long sak, const unsigned short* B, long sbk,
                     long sbn, int M, int N, int K, float* C, long scm, long scn) {
  surr::GemmArgs g{};
  g.A = A; g.sam = sam; g.sak = sak; g.B = B; g.sbk = sbk; g.sbn = sbn;
  g.M = M; g.N = N; g.K = K; g.C = C; g.scm = scm; g.scn = scn; g.cz = 0;
  return g;
}

// Forward pass of a batch already gathered into X0 (BF16 [B x ni]); keeps the
// pre-activations Z and BF16 activations H for the backward pass.
hipError_t surr_forward_batch(chem_surr s, int B, hipStream_t st) {
  const int H = surr::HID, ni = s->ni, no = s->no;
  hipError_t e;
  const unsigned short* Hin[3] = {s->X0, s->H1, s->H2};
  unsigned short* Hout[3] = {s->H1, s->H2, s->H3};
  float* Zs[3] = {s->Z1, s->Z2, s->Z3};
  const long oW[3] = {s->oW1, s->oW2, s->oW3}, ob[3] = {s->ob1, s->ob2, s->ob3};
  for (int l = 0; l < 3; ++l) {
    const int K = l == 0 ? ni : H;
    surr::GemmArgs g = gargs(Hin[l], K, 1, s->wbf + oW[l], 1, K, B, H, K, Zs[l], H, 1);
    g.Cb = Hout[l]; g.sbm = H; g.sbc = 1; g.bias = s->theta + ob[l];
    if ((e = gemm<surr::EPI_BIAS_SILU>(g, 1, st)) != hipSuccess) return e;
  }
  surr::GemmArgs g = gargs(s->H3, H, 1, s->wbf + s->oW4, 1, H, B, no, H, s->out, no, 1);
  g.bias = s->theta + s->ob4;
  return gemm<surr::EPI_BIAS>(g, 1, st);
}

// The arguments of the training step's kernels for a batch of B samples:
// rows (pa ((first + s) mod n) + pb) mod n of Xn / Yn.
surr::TrainArgs train_args(chem_surr s, const float* Xn, const float* Yn, long n, long first,
                           unsigned long long pa, unsigned long long pb, int B) {
  surr::TrainArgs a{};
  a.Xn = Xn; a.Yn = Yn; a.n = n; a.first = first; a.pa = pa; a.pb = pb;
  a.B = B; a.Bp = (B + 31) / 32 * 32;
  a.wpack = s->wpack; a.bpack = s->bpack; a.wtpack = s->wtpack;
  a.Xfm = s->Xfm; a.Hfm = s->Hfm; a.Zd = s->Zd; a.dZfm = s->dZfm; a.doutfm = s->doutfm;
  a.sse = s->sse;
  a.scale = 2.0f / ((float)B * (float)s->no);
  a.theta = s->theta; a.m = s->m; a.v = s->v; a.grad = s->grad; a.wbf = s->wbf;
  a.wpack_w = s->wpack; a.bpack_w = s->bpack; a.wtpack_w = s->wtpack;
  a.oW[0] = s->oW1; a.oW[1] = s->oW2; a.oW[2] = s->oW3; a.oW[3] = s->oW4;
  a.ob[0] = s->ob1; a.ob[1] = s->ob2; a.ob[2] = s->ob3; a.ob[3] = s->ob4;
  return a;
}

// One training step's kernels: forward + loss, backward, weight gradients
// (and, with a.adam, the Adam update of every parameter).
hipError_t train_step(chem_surr s, const surr::TrainArgs& a, hipStream_t st) {
  const MechEntry* en = s->mech->entry;
  hipError_t e = en->launch_train(a, 0, st);
  if (e == hipSuccess) e = en->launch_train(a, 1, st);
  if (e == hipSuccess) e = en->launch_train(a, 2, st);
  return e;
}

int surr_pack(chem_surr s, hipStream_t st) {
  const int kc1 = (s->ni + 31) / 32, ot4 = (s->no + 15) / 16;
  hipLaunchKernelGGL(surr::pack_weights, dim3(256), dim3(256), 0, st, s->theta, s->ni, s->no, kc1,
                     ot4, s->wpack, s->bpack, s->norm + s->ni, s->isd);
  const MechEntry* en = s->mech->entry;
  hipLaunchKernelGGL(surr::pack_transposed, dim3(256), dim3(256), 0, st, s->theta, s->ni, s->no,
                     s->oW2, s->oW3, s->oW4, en->train_w4t_ld, en->train_wt4, en->train_wt2,
                     s->wtpack);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "launch pack_weights");
  s->packed = true;
  return CHEM_OK;
}

// Where one surrogate step keeps its fallback list and the fallback pool's
// counter, tail records and order: the surrogate's and mechanism's own for
// surrogate_infer, a graph's own for a captured step.
struct StepBufs {
  int32_t* fb_list;
  unsigned* fb_count;
  unsigned long long* next;
  TailStore* tail;
  OrderStore* order;
};

// Enqueue one surrogate step on `st`: zero the list, the fused inference
// (appending untrusted cells when `fallback`), then one FP64 pool over the
// list, its size read on the device.
int enqueue_step(chem_surr s, chem_mech m, double* state, int64_t ld, int64_t n_cells, double dt,
                 const double trust[4], bool fallback, const chem_opts* opts, hipStream_t st,
                 int32_t* trust_code, float* out_std, int32_t* status, int32_t* counts,
                 const StepBufs& b, bool timed) {
  hipLaunchKernelGGL(surr::zero_u32, dim3(1), dim3(1), 0, st, b.fb_count);
  if (n_cells <= 0) return CHEM_OK;
  surr::InferArgs a{};
  a.state = state; a.ld = ld; a.n = n_cells; a.dt = dt;
  a.wpack = s->wpack; a.bpack = s->bpack; a.norm = s->norm; a.isd = s->isd;
  a.hull_margin = trust[0]; a.elem_tol = trust[1]; a.pos_tol = trust[2]; a.energy_tol = trust[3];
  a.fb_list = fallback ? b.fb_list : nullptr;
  a.fb_count = b.fb_count;
  a.trust_code = trust_code;
  a.out_std = out_std;
  hipError_t e = m->entry->launch_surr_infer(a, m->n_cu, st);
  if (e != hipSuccess) return hip_fail(e, "launch surr_infer");
  if (!fallback) return CHEM_OK;
  PoolArgs pa{};
  pa.one = BoxDesc{state, ld, n_cells, 0, dt, 1, 0, status, counts, b.fb_list};
  pa.boxes = nullptr;
  pa.n_boxes = 1;
  pa.total = n_cells;
  pa.total_dev = b.fb_count;
  pa.c = make_control(opts);
  pa.fixed_steps = opts ? opts->fixed_steps : 0;
  pa.scheme = opts ? opts->scheme : SCHEME_LSRK;
  return run_pool_with(m, pa, opts, st, b.next, *b.tail, b.order, timed);
}

}  // namespace

extern "C" {

int surrogate_create(chem_mech mech, int32_t hidden, int32_t depth, uint64_t seed, chem_surr* out) {
  if (!mech || !out) return fail(CHEM_EINVAL, "surrogate_create: null argument");
  *out = nullptr;
  if (hidden != surr::HID || depth != 3)
    return fail(CHEM_EINVAL, "surrogate_create: only hidden = 128, depth = 3 are built");
  chem_surr s = new (std::nothrow) chem_surr_s();
  if (!s) return fail(CHEM_ENOMEM, "surrogate_create: host allocation");
  s->mech = mech;
  s->ni = mech->entry->ns + 3;
  s->no = mech->entry->ns + 1;
  const long H = surr::HID;
  s->oW1 = 0; s->ob1 = H * s->ni; s->oW2 = s->ob1 + H; s->ob2 = s->oW2 + H * H;
  s->oW3 = s->ob2 + H; s->ob3 = s->oW3 + H * H; s->oW4 = s->ob3 + H; s->ob4 = s->oW4 + (long)s->no * H;
  s->P = s->ob4 + s->no;
  const int kc1 = (s->ni + 31) / 32, ot4 = (s->no + 15) / 16;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) { if (e == hipSuccess) e = r; };
  A(dalloc(&s->theta, s->P)); A(dalloc(&s->m, s->P)); A(dalloc(&s->v, s->P));
  A(dalloc(&s->grad, s->P)); A(dalloc(&s->wbf, s->P));
  A(dalloc(&s->norm, 4L * s->ni + 2L * s->no));
  A(dalloc(&s->wpack, surr::packed_weight_elems(kc1, ot4)));
  A(dalloc(&s->bpack, 3 * H + ot4 * 16));
  A(dalloc(&s->isd, s->ni));
  A(dalloc(&s->wtpack, mech->entry->train_wtpack_elems));
  A(dalloc(&s->sse, 1));
  A(dalloc(&s->fb_count, 1));
  if (e != hipSuccess) { surrogate_free(s); return hip_fail(e, "hipMalloc(surrogate)"); }
  // He-uniform init (bound sqrt(6 / fan_in)), zero biases, from splitmix64(seed)
  std::vector<float> th(s->P, 0.f);
  uint64_t x = seed;
  const long oW[4] = {s->oW1, s->oW2, s->oW3, s->oW4};
  const long rows[4] = {H, H, H, s->no}, cols[4] = {s->ni, H, H, H};
  for (int l = 0; l < 4; ++l) {
    const double lim = sqrt(6.0 / (double)cols[l]);
    for (long i = 0; i < rows[l] * cols[l]; ++i) th[oW[l] + i] = (float)((2.0 * uniform01(x) - 1.0) * lim);
  }
  std::vector<float> nm(4 * s->ni + 2 * s->no, 0.f);
  for (int k = 0; k < s->ni; ++k) { nm[s->ni + k] = 1.f; nm[2 * s->ni + 2 * s->no + k] = -1e30f;
                                    nm[3 * s->ni + 2 * s->no + k] = 1e30f; }
  for (int k = 0; k < s->no; ++k) nm[2 * s->ni + s->no + k] = 1.f;
  A(hipMemcpy(s->theta, th.data(), sizeof(float) * s->P, hipMemcpyHostToDevice));
  A(hipMemcpy(s->norm, nm.data(), sizeof(float) * nm.size(), hipMemcpyHostToDevice));
  A(hipMemset(s->m, 0, sizeof(float) * s->P));
  A(hipMemset(s->v, 0, sizeof(float) * s->P));
  if (e != hipSuccess) { surrogate_free(s); return hip_fail(e, "surrogate_create: upload"); }
  hipLaunchKernelGGL(surr::cast_bf16, dim3((unsigned)((s->P + 255) / 256)), dim3(256), 0, 0, s->theta,
                     s->P, s->wbf);
  int rc = surr_pack(s, 0);
  if (rc == CHEM_OK && (e = hipDeviceSynchronize()) != hipSuccess) rc = hip_fail(e, "surrogate_create");
  if (rc) { surrogate_free(s); return rc; }
  *out = s;
  return CHEM_OK;
}

void surrogate_free(chem_surr s) {
  if (!s) return;
  (void)hipDeviceSynchronize();  // teardown: nothing to report an error to
  surr_free_batch(s);
  for (void* p : {(void*)s->theta, (void*)s->m, (void*)s->v, (void*)s->grad, (void*)s->wbf,
                  (void*)s->norm, (void*)s->wpack, (void*)s->bpack, (void*)s->isd,
                  (void*)s->wtpack,
                  (void*)s->Xn, (void*)s->Yn,
                  (void*)s->sse, (void*)s->fb_list, (void*)s->fb_count})
    if (p) (void)hipFree(p);
  delete s;
}

int surrogate_query(chem_surr s, int32_t* n_in, int32_t* n_out, int64_t* n_params) {
  if (!s) return fail(CHEM_EINVAL, "surrogate_query: null handle");
  if (n_in) *n_in = s->ni;
  if (n_out) *n_out = s->no;
  if (n_params) *n_params = s->P;
  return CHEM_OK;
}

int surrogate_get_params(chem_surr s, float* theta_host, float* norm_host) {
  if (!s) return fail(CHEM_EINVAL, "surrogate_get_params: null handle");
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess && theta_host)
    e = hipMemcpy(theta_host, s->theta, sizeof(float) * s->P, hipMemcpyDeviceToHost);
  if (e == hipSuccess && norm_host)
    e = hipMemcpy(norm_host, s->norm, sizeof(float) * (4 * s->ni + 2 * s->no), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "surrogate_get_params");
  return CHEM_OK;
}

int surrogate_set_params(chem_surr s, const float* theta_host, const float* norm_host) {
  if (!s) return fail(CHEM_EINVAL, "surrogate_set_params: null handle");
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess && theta_host)
    e = hipMemcpy(s->theta, theta_host, sizeof(float) * s->P, hipMemcpyHostToDevice);
  if (e == hipSuccess && norm_host) {
    e = hipMemcpy(s->norm, norm_host, sizeof(float) * (4 * s->ni + 2 * s->no), hipMemcpyHostToDevice);
    s->norm_set = true;
  }
  if (e != hipSuccess) return hip_fail(e, "surrogate_set_params");
  hipLaunchKernelGGL(surr::cast_bf16, dim3((unsigned)((s->P + 255) / 256)), dim3(256), 0, 0, s->theta,
                     s->P, s->wbf);
  int rc = surr_pack(s, 0);
  if (rc) return rc;
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "surrogate_set_params");
  return CHEM_OK;
}

int surrogate_make_pairs(chem_mech m, const double* before, const double* after, int64_t ld,
                         int64_t n, double dt, const double* dt_cells, float* X, float* Y,
                         void* stream) {
  if (!m || n < 0 || ld < n) return fail(CHEM_EINVAL, "surrogate_make_pairs: bad argument");
  if (n > 0 && (!before || !after || !X || !Y)) return fail(CHEM_EINVAL, "surrogate_make_pairs: null");
  if (!dt_cells && !(dt > 0)) return fail(CHEM_EINVAL, "surrogate_make_pairs: dt must be > 0");
  hipError_t e = m->entry->launch_make_pairs(before, after, ld, n, dt, dt_cells, X, Y,
                                             (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "launch make_pairs");
  return CHEM_OK;
}

int surrogate_grad(chem_surr s, const float* Xn, const float* Yn, int32_t B, float* grad_out,
                   float* loss_host, void* stream) {
  if (!s || !Xn || !Yn || B <= 0) return fail(CHEM_EINVAL, "surrogate_grad: bad argument");
  int rc = surr_ensure_train(s, B);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemsetAsync(s->sse, 0, sizeof(double), st);
  if (e != hipSuccess) return hip_fail(e, "surrogate_grad clear");
  surr::TrainArgs a = train_args(s, Xn, Yn, B, 0, 1ull, 0ull, B);
  a.adam = 0;
  e = train_step(s, a, st);
  if (e == hipSuccess && grad_out)
    e = hipMemcpyAsync(grad_out, s->grad, sizeof(float) * s->P, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "surrogate_grad");
  if (loss_host) {
    double sse = 0;
    if ((e = hipMemcpyAsync(&sse, s->sse, sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess)
      return hip_fail(e, "surrogate_grad loss copy");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "surrogate_grad sync");
    *loss_host = (float)(sse / ((double)B * s->no));
  }
  return CHEM_OK;
}

int surrogate_forward(chem_surr s, const float* X, int64_t n, float* out, void* stream) {
  if (!s || n < 0 || (n > 0 && (!X || !out))) return fail(CHEM_EINVAL, "surrogate_forward: bad argument");
  const int B = 4096;
  int rc = surr_ensure_batch(s, B);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  float* tmp = s->fwd_tmp;
  hipError_t e = hipSuccess;
  for (long c0 = 0; c0 < n && e == hipSuccess; c0 += B) {
    const int b = (int)std::min<long>(B, n - c0);
    e = hipMemcpyAsync(tmp, X + c0 * s->ni, sizeof(float) * b * s->ni, hipMemcpyDeviceToDevice, st);
    hipLaunchKernelGGL(surr::standardise, dim3((unsigned)((b * s->ni + 255) / 256)), dim3(256), 0, st,
                       tmp, (long)b, s->ni, s->norm, s->norm + s->ni);
    hipLaunchKernelGGL(surr::gather_batch, dim3((b + 255) / 256), dim3(256), 0, st, tmp, tmp, (long)b,
                       s->ni, 0, 0L, b, 1ull, 0ull, s->X0, s->Yb);
    if (e == hipSuccess) e = surr_forward_batch(s, b, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(out + c0 * s->no, s->out, sizeof(float) * b * s->no, hipMemcpyDeviceToDevice, st);
  }
  const hipError_t es = hipStreamSynchronize(st);
  if (e == hipSuccess) e = es;
  if (e != hipSuccess) return hip_fail(e, "surrogate_forward");
  return CHEM_OK;
}

int surrogate_train(chem_surr s, const float* X, const float* Y, int64_t n, int32_t epochs,
                    int32_t batch, float lr, uint64_t seed, void* stream, float* loss_host) {
  if (!s || !X || !Y || n <= 0 || epochs < 0 || batch <= 0)
    return fail(CHEM_EINVAL, "surrogate_train: bad argument");
  if (n < batch) return fail(CHEM_EINVAL, "surrogate_train: fewer samples than one batch");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if (n > s->ncap) {
    if (s->Xn) (void)hipFree(s->Xn);
    if (s->Yn) (void)hipFree(s->Yn);
    s->Xn = s->Yn = nullptr;
    s->ncap = 0;
    if ((e = dalloc(&s->Xn, n * s->ni)) != hipSuccess) return hip_fail(e, "hipMalloc(train X)");
    if ((e = dalloc(&s->Yn, n * s->no)) != hipSuccess) return hip_fail(e, "hipMalloc(train Y)");
    s->ncap = n;
  }
  if ((e = hipMemcpyAsync(s->Xn, X, sizeof(float) * n * s->ni, hipMemcpyDeviceToDevice, st)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(s->Yn, Y, sizeof(float) * n * s->no, hipMemcpyDeviceToDevice, st)) !=
          hipSuccess)
    return hip_fail(e, "surrogate_train copy");
  float* mu_in = s->norm;
  float* sd_in = s->norm + s->ni;
  float* mu_out = s->norm + 2 * s->ni;
  float* sd_out = mu_out + s->no;
  float* zmin = sd_out + s->no;
  float* zmax = zmin + s->ni;
  if (!s->norm_set) {  // the normaliser and hull are fitted on the first call's data
    hipLaunchKernelGGL(surr::col_moments, dim3(s->ni), dim3(256), 0, st, s->Xn, (long)n, s->ni, mu_in, sd_in);
    hipLaunchKernelGGL(surr::col_moments, dim3(s->no), dim3(256), 0, st, s->Yn, (long)n, s->no, mu_out, sd_out);
  }
  hipLaunchKernelGGL(surr::standardise, dim3((unsigned)((n * s->ni + 255) / 256)), dim3(256), 0, st,
                     s->Xn, (long)n, s->ni, mu_in, sd_in);
  hipLaunchKernelGGL(surr::standardise, dim3((unsigned)((n * s->no + 255) / 256)), dim3(256), 0, st,
                     s->Yn, (long)n, s->no, mu_out, sd_out);
  if (!s->norm_set) {
    hipLaunchKernelGGL(surr::col_minmax, dim3(s->ni), dim3(256), 0, st, s->Xn, (long)n, s->ni, zmin, zmax);
    s->norm_set = true;
  }
  int rc = surr_ensure_train(s, batch);
  if (rc) return rc;
  const long steps = n / batch;
  const long total = steps * (long)epochs;
  uint64_t x = seed ^ 0x5DEECE66Dull;
  long t = 0;
  for (int ep = 0; ep < epochs; ++ep) {
    // epoch permutation: i -> (pa i + pb) mod n with pa coprime to n
    unsigned long long pa, pb = splitmix64(x) % (unsigned long long)n;
    for (;;) {
      pa = (splitmix64(x) % (unsigned long long)n) | 1ull;
      unsigned long long a0 = pa, b0 = (unsigned long long)n;
      while (b0) { const unsigned long long r = a0 % b0; a0 = b0; b0 = r; }
      if (a0 == 1) break;
    }
    if ((e = hipMemsetAsync(s->sse, 0, sizeof(double), st)) != hipSuccess)
      return hip_fail(e, "surrogate_train clear");
    surr::TrainArgs a = train_args(s, s->Xn, s->Yn, n, 0, pa, pb, batch);
    a.adam = 1;
    // the decay rates are the FP32 values the moment updates use; the bias
    // corrections 1 - beta^t are taken with those same values
    a.b1 = 0.9f; a.b2 = 0.999f; a.eps = 1e-8f;
    for (long k = 0; k < steps; ++k, ++t) {
      s->adam_t += 1;
      a.first = k * batch;
      a.lr = (float)(lr * 0.5 * (1.0 + cos(3.14159265358979323846 * (double)t / (double)total)));
      a.c1 = (float)(1.0 - pow((double)a.b1, (double)s->adam_t));
      a.c2 = (float)(1.0 - pow((double)a.b2, (double)s->adam_t));
      if ((e = train_step(s, a, st)) != hipSuccess) return hip_fail(e, "surrogate_train step");
    }
    if (loss_host) {
      double sse = 0;
      if ((e = hipMemcpyAsync(&sse, s->sse, sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return hip_fail(e, "surrogate_train loss copy");
      if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "surrogate_train sync");
      loss_host[ep] = (float)(sse / ((double)steps * batch * s->no));
    }
  }
  rc = surr_pack(s, st);
  if (rc) return rc;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "surrogate_train");
  return CHEM_OK;
}

int surrogate_reserve(chem_surr s, int64_t max_cells) {
  if (!s || max_cells < 0) return fail(CHEM_EINVAL, "surrogate_reserve: bad argument");
  if (max_cells <= s->reserved && s->fb_list) return CHEM_OK;
  hipError_t e;
  // growing: calls still queued may use the old list
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize(surrogate)");
  if (s->fb_list) (void)hipFree(s->fb_list);
  s->fb_list = nullptr;
  s->reserved = 0;
  const int64_t cap = std::max<int64_t>(max_cells, 1);
  if ((e = dalloc(&s->fb_list, cap)) != hipSuccess) return hip_fail(e, "hipMalloc(fallback list)");
  s->reserved = max_cells;
  return CHEM_OK;
}

int surrogate_infer(chem_surr s, chem_mech m, double* state, int64_t ld, int64_t n_cells, double dt,
                    const double trust[4], int32_t fallback, const chem_opts* opts, void* stream,
                    int32_t* trust_code, float* out_std, int32_t* status, int32_t* counts,
                    int64_t* n_fallback_host) {
  if (!s || !m || !trust) return fail(CHEM_EINVAL, "surrogate_infer: null argument");
  if (m->entry != s->mech->entry) return fail(CHEM_EINVAL, "surrogate_infer: surrogate built for another mechanism");
  if (n_cells < 0 || ld < n_cells) return fail(CHEM_EINVAL, "surrogate_infer: need 0 <= n_cells <= ld");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(CHEM_EINVAL, "surrogate_infer: dt must be finite and > 0");
  if (n_cells > 0 && !state) return fail(CHEM_EINVAL, "surrogate_infer: null state");
  if (n_cells > 0x7fffffff) return fail(CHEM_EINVAL, "surrogate_infer: more than 2^31-1 cells");
  int rc = check_opts(opts);
  if (rc) return rc;
  if (!s->packed) return fail(CHEM_EINVAL, "surrogate_infer: weights not packed");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (fallback) {
    // the fallback list is the surrogate's, the integrator's workspace the
    // mechanism's: both reservations must cover n_cells
    if (!s->fb_list || n_cells > s->reserved) {
      char msg[200];
      snprintf(msg, sizeof msg, "surrogate_infer: %lld cells but the surrogate is reserved for "
               "%lld (call surrogate_reserve first)", (long long)n_cells,
               (long long)(s->fb_list ? s->reserved : 0));
      return fail(CHEM_ECAPACITY, msg);
    }
    rc = check_capacity(m, n_cells, "surrogate_infer fallback");
    if (rc) return rc;
  }
  StepBufs b{s->fb_list, s->fb_count, m->d_next, &m->tail, &m->order};
  rc = enqueue_step(s, m, state, ld, n_cells, dt, trust, fallback != 0, opts, st, trust_code,
                    out_std, status, counts, b, true);
  if (rc) return rc;
  if (n_fallback_host) {
    unsigned cnt = 0;
    e = hipMemcpyAsync(&cnt, s->fb_count, sizeof(unsigned), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_fail(e, "surrogate_infer count copy");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "surrogate_infer sync");
    *n_fallback_host = (int64_t)cnt;
  }
  return CHEM_OK;
}

int surrogate_autotune(chem_surr s, chem_mech m, double* state, int64_t ld, int64_t n_cells,
                       double dt, const double trust[4], const chem_opts* base, int32_t reps,
                       const char* cache_path, void* stream, chem_opts* best) {
  if (!s || !m || !trust || !best) return fail(CHEM_EINVAL, "surrogate_autotune: null argument");
  if (m->entry != s->mech->entry)
    return fail(CHEM_EINVAL, "surrogate_autotune: surrogate built for another mechanism");
  if (n_cells <= 0 || ld < n_cells || !state)
    return fail(CHEM_EINVAL, "surrogate_autotune: need 0 < n_cells <= ld and a state");
  int rc = check_opts(base);
  if (rc) return rc;
  if (reps < 1) reps = 3;
  hipStream_t st = (hipStream_t)stream;
  char key[180];
  snprintf(key, sizeof key, "%016llx:%d:%s%s:surrogate", (unsigned long long)m->entry->hash,
           size_bucket(n_cells), arch_name(m->device).c_str(),
           (base && base->scheme == SCHEME_RKF45)  ? ":rkf45"
           : (base && base->scheme == SCHEME_ROS4) ? ":ros4"
                                                   : "");
  const chem_opts o = base ? *base : chem_opts{0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<TuneEntry> cache;
  if (cache_path) {
    cache = read_cache(cache_path);
    for (const auto& en : cache)
      if (en.key == key) {
        *best = o; best->block_size = en.block; best->chunk_steps = en.chunk;
        best->tail_steps = en.tail; best->tail_cap = en.cap; best->pool_order = en.order;
        return CHEM_OK;
      }
  }
  // the trials are surrogate_infer calls: both reservations must cover them
  if (!m->fixed_ready || n_cells > m->reserved) {
    rc = chem_workspace_reserve(m, std::max<int64_t>(n_cells, m->reserved));
    if (rc) return rc;
  }
  if (!s->fb_list || n_cells > s->reserved) {
    rc = surrogate_reserve(s, std::max<int64_t>(n_cells, s->reserved));
    if (rc) return rc;
  }
  // a snapshot of the caller's state, restored before every trial and at
  // the end
  const size_t bytes = sizeof(double) * (size_t)ld * (size_t)(m->entry->ns + 3);
  double* snap = nullptr;
  hipError_t e = hipMalloc(&snap, bytes);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(surrogate_autotune snapshot)");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(snap);
  };
  if ((e = hipMemcpyAsync(snap, state, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess ||
      (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipStreamSynchronize(st);
    cleanup();
    return hip_fail(e, "surrogate_autotune set-up");
  }
  auto time_one = [&](const chem_opts& t, float* el) -> int {
    if ((e = hipMemcpyAsync(state, snap, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess)
      return hip_fail(e, "restore");
    if ((e = hipEventRecord(e0, st)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    const int trc = surrogate_infer(s, m, state, ld, n_cells, dt, trust, 1, &t, stream, nullptr,
                                    nullptr, nullptr, nullptr, nullptr);
    if (trc != CHEM_OK) return trc;
    if ((e = hipEventRecord(e1, st)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if ((e = hipEventSynchronize(e1)) != hipSuccess) return hip_fail(e, "trial");
    *el = 0;
    if ((e = hipEventElapsedTime(el, e0, e1)) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    return CHEM_OK;
  };
  chem_opts found{};
  double best_ms = 0.0;
  rc = tune_search(m, o, reps, time_one, &found, &best_ms);
  if ((e = hipMemcpyAsync(state, snap, bytes, hipMemcpyDeviceToDevice, st)) != hipSuccess &&
      rc == CHEM_OK)
    rc = hip_fail(e, "restore");
  if ((e = hipStreamSynchronize(st)) != hipSuccess && rc == CHEM_OK)
    rc = hip_fail(e, "surrogate_autotune sync");
  cleanup();
  if (rc != CHEM_OK) return rc;
  *best = found;
  if (cache_path) {
    cache.push_back(TuneEntry{key, found.block_size, found.chunk_steps, found.tail_steps,
                              found.tail_cap, found.pool_order, best_ms});
    rc = write_cache(cache_path, cache);
  }
  return rc;
}

int surrogate_graph_capture(chem_surr s, chem_mech m, double* state, int64_t ld, int64_t n_cells,
                            double dt, const double trust[4], const chem_opts* opts, void* stream,
                            chem_graph* out) {
  if (!s || !m || !trust || !out) return fail(CHEM_EINVAL, "surrogate_graph_capture: null argument");
  *out = nullptr;
  if (m->entry != s->mech->entry)
    return fail(CHEM_EINVAL, "surrogate_graph_capture: surrogate built for another mechanism");
  if (n_cells <= 0 || ld < n_cells || !state)
    return fail(CHEM_EINVAL, "surrogate_graph_capture: need 0 < n_cells <= ld and a state");
  if (n_cells > 0x7fffffff) return fail(CHEM_EINVAL, "more than 2^31-1 cells");
  int rc = check_opts(opts);
  if (rc) return rc;
  if (!s->packed) return fail(CHEM_EINVAL, "surrogate_graph_capture: weights not packed");
  chem_graph g = new (std::nothrow) chem_graph_s();
  if (!g) return fail(CHEM_ENOMEM, "surrogate_graph_capture: host allocation");
  auto bail = [&](hipError_t e, const char* what) {
    chem_graph_destroy(g);
    return hip_fail(e, what);
  };
  // the graph's own list, pool counter, tail records and order, so that its
  // launches and eager calls on the same handles do not share them
  hipError_t e;
  if ((e = dalloc(&g->fb_list, n_cells)) != hipSuccess) return bail(e, "hipMalloc(graph fallback list)");
  if ((e = dalloc(&g->fb_count, 1)) != hipSuccess) return bail(e, "hipMalloc(graph list length)");
  if ((e = hipMalloc(&g->d_next, sizeof(unsigned long long))) != hipSuccess)
    return bail(e, "hipMalloc(graph pool counter)");
  if ((rc = alloc_tail(g->tail, n_cells, m->entry->tail_rd)) != CHEM_OK) { chem_graph_destroy(g); return rc; }
  if ((rc = alloc_order(g->order, n_cells)) != CHEM_OK) { chem_graph_destroy(g); return rc; }
  if (stream && (e = hipStreamSynchronize((hipStream_t)stream)) != hipSuccess)
    return bail(e, "hipStreamSynchronize");
  hipStream_t cs;
  if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess)
    return bail(e, "hipStreamCreate(capture)");
  // one empty inference launch outside the capture sets the kernel's LDS
  // attribute, which is a set-up call
  {
    surr::InferArgs a0{};
    a0.n = 0;
    a0.dt = dt;
    a0.wpack = s->wpack; a0.bpack = s->bpack; a0.norm = s->norm; a0.isd = s->isd;
    if ((e = m->entry->launch_surr_infer(a0, 1, cs)) != hipSuccess ||
        (e = hipStreamSynchronize(cs)) != hipSuccess) {
      (void)hipStreamDestroy(cs);
      return bail(e, "surrogate_graph_capture set-up");
    }
  }
  if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return bail(e, "hipStreamBeginCapture");
  }
  StepBufs b{g->fb_list, g->fb_count, g->d_next, &g->tail, &g->order};
  rc = enqueue_step(s, m, state, ld, n_cells, dt, trust, true, opts, cs, nullptr, nullptr,
                    nullptr, nullptr, b, false);
  e = hipStreamEndCapture(cs, &g->graph);
  (void)hipStreamDestroy(cs);
  if (rc) { chem_graph_destroy(g); return rc; }
  if (e != hipSuccess) return bail(e, "hipStreamEndCapture");
  if ((e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess)
    return bail(e, "hipGraphInstantiate");
  *out = g;
  return CHEM_OK;
}

int surrogate_save(chem_surr s, const char* path) {
  if (!s || !path) return fail(CHEM_EINVAL, "surrogate_save: null argument");
  std::vector<float> th(s->P), nm(4 * s->ni + 2 * s->no);
  int rc = surrogate_get_params(s, th.data(), nm.data());
  if (rc) return rc;
  FILE* f = fopen(path, "wb");
  if (!f) return fail(CHEM_EINVAL, std::string("cannot write ") + path);
  const char magic[8] = {'C', 'H', 'S', 'U', 'R', 'R', '0', '1'};
  const uint64_t hsh = s->mech->entry->hash;
  const int32_t dims[3] = {s->ni, s->no, surr::HID};
  bool ok = fwrite(magic, 1, 8, f) == 8 && fwrite(&hsh, 8, 1, f) == 1 && fwrite(dims, 4, 3, f) == 3 &&
            fwrite(th.data(), 4, th.size(), f) == th.size() && fwrite(nm.data(), 4, nm.size(), f) == nm.size();
  ok = (fclose(f) == 0) && ok;
  if (!ok) return fail(CHEM_EINVAL, std::string("short write to ") + path);
  return CHEM_OK;
}

int surrogate_load(chem_mech m, const char* path, chem_surr* out) {
  if (!m || !path || !out) return fail(CHEM_EINVAL, "surrogate_load: null argument");
  *out = nullptr;
  FILE* f = fopen(path, "rb");
  if (!f) return fail(CHEM_EPARSE, std::string("cannot open ") + path);
  char magic[8];
  uint64_t hsh = 0;
  int32_t dims[3] = {0, 0, 0};
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "CHSURR01", 8) == 0 &&
            fread(&hsh, 8, 1, f) == 1 && fread(dims, 4, 3, f) == 3;
  if (!ok || hsh != m->entry->hash || dims[0] != m->entry->ns + 3 || dims[1] != m->entry->ns + 1 ||
      dims[2] != surr::HID) {
    fclose(f);
    return fail(CHEM_EPARSE, std::string(path) + ": not a surrogate for this mechanism");
  }
  chem_surr s = nullptr;
  int rc = surrogate_create(m, surr::HID, 3, 0, &s);
  if (rc) { fclose(f); return rc; }
  std::vector<float> th(s->P), nm(4 * s->ni + 2 * s->no);
  ok = fread(th.data(), 4, th.size(), f) == th.size() && fread(nm.data(), 4, nm.size(), f) == nm.size();
  fclose(f);
  if (!ok) { surrogate_free(s); return fail(CHEM_EPARSE, std::string(path) + ": truncated"); }
  rc = surrogate_set_params(s, th.data(), nm.data());
  if (rc) { surrogate_free(s); return rc; }
  *out = s;
  return CHEM_OK;
}

}  // extern "C"
