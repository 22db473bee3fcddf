// C entry points of the surrogate MLP (declared in include/sugg.h): workspace
// object, forward (inference or training), MSE, hand-written backward, Adam
// and the fused training step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>

#include "ctx.hpp"

using namespace sugg;

struct sugg_mlp {
  sugg_ctx* ctx = nullptr;   // identity only
  int device = 0;
  int in = 0, hid = 0, out = 0, bm = 0;   // bm: max batch, multiple of 8
  int64_t off_w1 = 0, off_b1 = 0, off_w2 = 0, off_b2 = 0, off_w3 = 0, off_b3 = 0, nparam = 0;
  // BF16 working weights: row-major [out][in] and, where the backward needs
  // it, transposed [in][out]
  __bf16 *w1 = nullptr, *w2 = nullptr, *w2t = nullptr, *w3 = nullptr, *w3t = nullptr;
  // activations (row-major [batch][features]; transposed [features][bm])
  __bf16 *xb = nullptr, *xt = nullptr, *h1 = nullptr, *h1t = nullptr, *h2 = nullptr, *h2t = nullptr;
  __bf16 *dy = nullptr, *dyt = nullptr, *da2 = nullptr, *da2t = nullptr, *da1t = nullptr;
  float *a1 = nullptr, *a2 = nullptr, *part = nullptr, *loss_part = nullptr, *ybuf = nullptr;
  int32_t* trow = nullptr;      // training rows of the current mini-batch (sugg_mlp_train_epoch)
  int64_t part_n = 0;
  int64_t part_off[3] = {};   // partial regions of the weight gradients of layers 3, 2, 1
  float* frozen = nullptr;      // inference copy of the parameters (sugg_mlp_freeze)
  bool packed_frozen = false;   // the BF16 working weights hold the frozen parameters
  int32_t info[8][4] = {};   // launched GEMM instances: forward layers 1-3, then the backward's five
  int kept_batch = -1;    // batch of the last forward that kept activations
  bool have_dy = false;   // dY of that batch is in dy/dyt (from sugg_mlp_loss)
  ~sugg_mlp() {
    dfree(w1); dfree(w2); dfree(w2t); dfree(w3); dfree(w3t);
    dfree(xb); dfree(xt); dfree(h1); dfree(h1t); dfree(h2); dfree(h2t);
    dfree(dy); dfree(dyt); dfree(da2); dfree(da2t); dfree(da1t);
    dfree(a1); dfree(a2); dfree(part); dfree(loss_part); dfree(ybuf); dfree(frozen); dfree(trow);
  }
};

namespace {

int splits_for(int M, int N, int K) {
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  int s = std::max(1, 256 / std::max(1, tiles));
  s = std::min(s, std::max(1, K / 256));
  return s;
}

GemmArgs gemm(const __bf16* A, int lda, const __bf16* Bt, int ldb, int M, int N, int K) {
  GemmArgs g{};
  g.A = A;
  g.lda = lda;
  g.Bt = Bt;
  g.ldb = ldb;
  g.M = M;
  g.N = N;
  g.K = K;
  g.k_per_split = (K + 31) / 32 * 32;
  return g;
}

// weight gradient dW[M x N] = A[M x K] . Bt[N x K]^T with K split across
// workgroups into partial region `region` of the layer, and its finishing
// job: the split sums into dW and the bias gradient db[M] = row sums of A (the
// transposed activation gradient, K = batch)
GemmArgs wgrad_args(sugg_mlp* m, int region, const __bf16* A, int lda, const __bf16* Bt, int ldb, int M, int N, int K,
                    float* dW, float* db, int* splits, WgradJob* job) {
  GemmArgs g = gemm(A, lda, Bt, ldb, M, N, K);
  const int sp = splits_for(M, N, K);
  g.k_per_split = ((K + sp - 1) / sp + 31) / 32 * 32;
  *splits = (K + g.k_per_split - 1) / g.k_per_split;
  g.Cf = m->part + m->part_off[region];
  *job = WgradJob{g.Cf, (int64_t)M * N, *splits, dW, A, M, K, lda, db};
  return g;
}

int check_mlp(sugg_ctx* ctx, sugg_mlp* m, int batch) {
  if (!m || m->ctx != ctx) return ctx->fail(SUGG_E_ARG, "mlp missing or from another context");
  if (batch < 1 || batch > m->bm) return ctx->fail(SUGG_E_SHAPE, "batch %d outside [1, %d]", batch, m->bm);
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  return SUGG_OK;
}

// forward pass; target (nullable) adds the squared-error loss and dY
hipError_t pack_weights(sugg_mlp* m, const float* params, hipStream_t s) {
  const int in = m->in, hid = m->hid, out = m->out;
  hipError_t e = launch_pack(params + m->off_w1, hid, in, m->w1, in, nullptr, 0, s);
  if (e == hipSuccess) e = launch_pack(params + m->off_w2, hid, hid, m->w2, hid, m->w2t, hid, s);
  if (e == hipSuccess) e = launch_pack(params + m->off_w3, out, hid, m->w3, hid, m->w3t, out, s);
  m->packed_frozen = params == m->frozen;
  return e;
}

// x == nullptr: the batch is already packed in xb and xt; trow (nullable):
// row r's target is target row trow[r]
// defer_loss: the caller sums the loss partials (in the backward's finishing
// launch)
int forward(sugg_ctx* ctx, sugg_mlp* m, const float* params, const float* x, int B, float* y, bool keep,
            const float* target, float* loss, hipStream_t s, bool pack_w = true, const int32_t* trow = nullptr,
            bool defer_loss = false) {
  const int in = m->in, hid = m->hid, out = m->out, bm = m->bm;
  hipError_t e = hipSuccess;
  if (pack_w) e = pack_weights(m, params, s);
  if (e == hipSuccess && x) e = launch_pack(x, B, in, m->xb, in, keep ? m->xt : nullptr, bm, s);
  if (e != hipSuccess) return ctx->hip(e, "mlp pack");
  GemmArgs g = gemm(m->xb, in, m->w1, in, B, hid, in);
  g.bias = params + m->off_b1;
  g.Cf = keep ? m->a1 : nullptr;
  g.ldcf = hid;
  g.Cb = m->h1;
  g.ldcb = hid;
  g.Ct = keep ? m->h1t : nullptr;
  g.ldct = bm;
  e = launch_gemm(g, kEpiFwdHidden, 1, s, m->info[0]);
  if (e != hipSuccess) return ctx->hip(e, "mlp layer 1");
  g = gemm(m->h1, hid, m->w2, hid, B, hid, hid);
  g.bias = params + m->off_b2;
  g.Cf = keep ? m->a2 : nullptr;
  g.ldcf = hid;
  g.Cb = m->h2;
  g.ldcb = hid;
  g.Ct = keep ? m->h2t : nullptr;
  g.ldct = bm;
  e = launch_gemm(g, kEpiFwdHidden, 1, s, m->info[1]);
  if (e != hipSuccess) return ctx->hip(e, "mlp layer 2");
  g = gemm(m->h2, hid, m->w3, hid, B, out, hid);
  g.bias = params + m->off_b3;
  g.Cf = y;
  g.ldcf = out;
  if (target) {
    g.target = target;
    g.ldt = out;
    g.trow = trow;
    g.Cb = m->dy;
    g.ldcb = out;
    g.Ct = m->dyt;
    g.ldct = bm;
    g.loss_part = m->loss_part;
    g.scale = 2.0f / ((float)B * (float)out);
  }
  e = launch_gemm(g, kEpiFwdOut, 1, s, m->info[2]);
  if (e != hipSuccess) return ctx->hip(e, "mlp layer 3");
  if (target && !defer_loss) {
    const int tiles = ((B + 63) / 64) * ((out + 63) / 64);
    e = launch_loss_sum(m->loss_part, tiles, 1.0f / ((float)B * (float)out), loss, s);
    if (e != hipSuccess) return ctx->hip(e, "mlp loss");
  }
  m->kept_batch = keep ? B : -1;
  m->have_dy = keep && target;
  return SUGG_OK;
}

// Three launches and the finish: each layer's weight gradient shares a launch
// with the backward through that layer (they do not depend on each other),
// and one launch finishes all three weight and bias gradients (and, with
// loss non-null, sums the loss partials of the forward that kept dY).
int backward(sugg_ctx* ctx, sugg_mlp* m, const float* params, int B, float* grads, hipStream_t s,
             float* loss = nullptr) {
  (void)params;
  const int in = m->in, hid = m->hid, out = m->out, bm = m->bm;
  FinishArgs fa{};
  fa.njobs = 3;
  int sp = 1;
  GemmArgs gw = wgrad_args(m, 0, m->dyt, bm, m->h2t, bm, out, hid, B, grads + m->off_w3, grads + m->off_b3, &sp,
                           &fa.job[0]);
  GemmArgs g = gemm(m->dy, out, m->w3t, out, B, hid, out);
  g.gact = m->a2;
  g.ldg = hid;
  g.Cb = m->da2;
  g.ldcb = hid;
  g.Ct = m->da2t;
  g.ldct = bm;
  hipError_t e = launch_gemm_pair(gw, sp, g, s, m->info[3], m->info[4]);
  if (e != hipSuccess) return ctx->hip(e, "mlp backward layer 3");
  gw = wgrad_args(m, 1, m->da2t, bm, m->h1t, bm, hid, hid, B, grads + m->off_w2, grads + m->off_b2, &sp, &fa.job[1]);
  g = gemm(m->da2, hid, m->w2t, hid, B, hid, hid);
  g.gact = m->a1;
  g.ldg = hid;
  g.Ct = m->da1t;
  g.ldct = bm;
  e = launch_gemm_pair(gw, sp, g, s, m->info[5], m->info[6]);
  if (e != hipSuccess) return ctx->hip(e, "mlp backward layer 2");
  gw = wgrad_args(m, 2, m->da1t, bm, m->xt, bm, hid, in, B, grads + m->off_w1, grads + m->off_b1, &sp, &fa.job[2]);
  e = launch_gemm(gw, kEpiWgrad, sp, s, m->info[7]);
  if (e != hipSuccess) return ctx->hip(e, "mlp backward layer 1");
  if (loss) {
    fa.loss_part = m->loss_part;
    fa.loss_n = ((B + 63) / 64) * ((out + 63) / 64);
    fa.loss_scale = 1.0f / ((float)B * (float)out);
    fa.loss = loss;
  }
  e = launch_wgrad_finish(fa, s);
  if (e != hipSuccess) return ctx->hip(e, "mlp gradients");
  return SUGG_OK;
}

}  // namespace

// Inference with the frozen parameters (packed once, repacked only after a
// call with other parameters overwrote the working weights).
int mlp_infer(sugg_ctx* ctx, sugg_mlp* m, const float* x, int B, float* y, hipStream_t s) {
  if (!m || m->ctx != ctx) return ctx->fail(SUGG_E_ARG, "mlp missing or from another context");
  if (!m->frozen) return ctx->fail(SUGG_E_STATE, "mlp has no frozen parameters (sugg_mlp_freeze)");
  if (B < 1 || B > m->bm) return ctx->fail(SUGG_E_SHAPE, "batch %d outside [1, %d]", B, m->bm);
  return forward(ctx, m, m->frozen, x, B, y, false, nullptr, nullptr, s, !m->packed_frozen);
}

namespace {

// Inference and each row's top n of the outputs in columns >= skip above
// tau: the output layer's epilogue ranks where the output width is 64 or
// 128 (a tile row), otherwise the outputs go through the row ranking kernel.
// x == nullptr: the input is already in the BF16 input buffer (mlp_input)
int infer_rank(sugg_ctx* ctx, sugg_mlp* m, const float* x, int B, int skip, int n, float tau, float* y,
               int32_t* idx, float* score, int32_t* count, hipStream_t s) {
  const int in = m->in, hid = m->hid, out = m->out;
  hipError_t e = hipSuccess;
  if (!m->packed_frozen) e = pack_weights(m, m->frozen, s);
  if (e == hipSuccess && x) e = launch_pack(x, B, in, m->xb, in, nullptr, m->bm, s);
  if (e != hipSuccess) return ctx->hip(e, "mlp pack");
  const float* params = m->frozen;
  GemmArgs g = gemm(m->xb, in, m->w1, in, B, hid, in);
  g.bias = params + m->off_b1;
  g.Cb = m->h1;
  g.ldcb = hid;
  e = launch_gemm(g, kEpiFwdHidden, 1, s, m->info[0]);
  if (e != hipSuccess) return ctx->hip(e, "mlp layer 1");
  g = gemm(m->h1, hid, m->w2, hid, B, hid, hid);
  g.bias = params + m->off_b2;
  g.Cb = m->h2;
  g.ldcb = hid;
  e = launch_gemm(g, kEpiFwdHidden, 1, s, m->info[1]);
  if (e != hipSuccess) return ctx->hip(e, "mlp layer 2");
  g = gemm(m->h2, hid, m->w3, hid, B, out, hid);
  g.bias = params + m->off_b3;
  g.Cf = y;
  g.ldcf = out;
  if (out == 64 || out == 128) {
    g.idx_out = idx;
    g.score_out = score;
    g.count_out = count;
    g.n = n;
    g.skip = skip;
    g.tau = tau;
    e = launch_gemm_rank(g, s, m->info[2]);
    if (e != hipSuccess) return ctx->hip(e, "mlp layer 3 with ranking");
  } else {
    if (!y) g.Cf = m->ybuf;
    e = launch_gemm(g, kEpiFwdOut, 1, s, m->info[2]);
    if (e == hipSuccess)
      e = launch_rank<float>(g.Cf, nullptr, B, skip, n, tau, idx, score, count, s, (int64_t)out);
    if (e != hipSuccess) return ctx->hip(e, "mlp layer 3 and ranking");
  }
  m->kept_batch = -1;
  m->have_dy = false;
  return SUGG_OK;
}

}  // namespace

void mlp_dims(const sugg_mlp* m, int* in, int* out, int* max_batch) {
  *in = m->in;
  *out = m->out;
  *max_batch = m->bm;
}

__bf16* mlp_input(sugg_mlp* m) { return m->xb; }

int mlp_infer_rank_input(sugg_ctx* ctx, sugg_mlp* m, int B, int skip, int n, float tau, float* y, int32_t* idx,
                         float* score, int32_t* count, hipStream_t s) {
  if (!m->frozen) return ctx->fail(SUGG_E_STATE, "mlp has no frozen parameters (sugg_mlp_freeze)");
  return infer_rank(ctx, m, nullptr, B, skip, n, tau, y, idx, score, count, s);
}

extern "C" {

int32_t sugg_mlp_create(sugg_ctx* ctx, int32_t in, int32_t hidden, int32_t out, int32_t max_batch, sugg_mlp** res) {
  if (!ctx || !res) return SUGG_E_ARG;
  *res = nullptr;
  if (in < 8 || hidden < 8 || out < 8 || in % 8 || hidden % 8 || out % 8 || in > 4096 || hidden > 4096 || out > 4096)
    return ctx->fail(SUGG_E_SHAPE, "layer widths must be multiples of 8 in [8, 4096]");
  if (max_batch < 1 || max_batch > (1 << 20)) return ctx->fail(SUGG_E_SHAPE, "max_batch outside [1, 2^20]");
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  sugg_mlp* m = new (std::nothrow) sugg_mlp();
  if (!m) return ctx->fail(SUGG_E_BUDGET, "out of host memory");
  m->ctx = ctx;
  m->device = ctx->device;
  m->in = in;
  m->hid = hidden;
  m->out = out;
  m->bm = (max_batch + 7) / 8 * 8;
  m->off_w1 = 0;
  m->off_b1 = m->off_w1 + (int64_t)hidden * in;
  m->off_w2 = m->off_b1 + hidden;
  m->off_b2 = m->off_w2 + (int64_t)hidden * hidden;
  m->off_w3 = m->off_b2 + hidden;
  m->off_b3 = m->off_w3 + (int64_t)out * hidden;
  m->nparam = m->off_b3 + out;
  const size_t bm = m->bm, bf = sizeof(__bf16);
  // one region per layer (the three weight gradients are finished together);
  // a smaller batch uses no more splits than the largest
  int64_t part = 0;
  int li = 0;
  for (auto mn : {std::pair<int, int>(out, hidden), {hidden, hidden}, {hidden, in}}) {
    m->part_off[li++] = part;
    part += (int64_t)splits_for(mn.first, mn.second, m->bm) * mn.first * mn.second;
  }
  m->part_n = part;
  hipError_t e = hipSuccess;
  auto A = [&](auto*& p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc((void**)&p, std::max<size_t>(bytes, 16));
  };
  A(m->w1, bf * hidden * in);
  A(m->w2, bf * hidden * hidden);
  A(m->w2t, bf * hidden * hidden);
  A(m->w3, bf * out * hidden);
  A(m->w3t, bf * out * hidden);
  A(m->xb, bf * bm * in);
  A(m->xt, bf * bm * in);
  A(m->h1, bf * bm * hidden);
  A(m->h1t, bf * bm * hidden);
  A(m->h2, bf * bm * hidden);
  A(m->h2t, bf * bm * hidden);
  A(m->dy, bf * bm * out);
  A(m->dyt, bf * bm * out);
  A(m->da2, bf * bm * hidden);
  A(m->da2t, bf * bm * hidden);
  A(m->da1t, bf * bm * hidden);
  A(m->a1, sizeof(float) * bm * hidden);
  A(m->a2, sizeof(float) * bm * hidden);
  A(m->part, sizeof(float) * part);
  A(m->loss_part, sizeof(float) * ((bm + 63) / 64) * ((out + 63) / 64));
  A(m->ybuf, sizeof(float) * bm * out);
  A(m->trow, sizeof(int32_t) * bm);
  if (e != hipSuccess) {
    delete m;
    return ctx->hip(e, "mlp workspace");
  }
  *res = m;
  return SUGG_OK;
}

void sugg_mlp_destroy(sugg_mlp* mlp) {
  if (!mlp) return;
  int cur = -1;
  if (hipGetDevice(&cur) == hipSuccess && cur != mlp->device) (void)hipSetDevice(mlp->device);
  delete mlp;
}

int64_t sugg_mlp_param_count(const sugg_mlp* mlp) { return mlp ? mlp->nparam : -1; }

int32_t sugg_mlp_launch_info(const sugg_mlp* mlp, int32_t* info) {
  if (!mlp || !info) return SUGG_E_ARG;
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 4; ++j) info[4 * i + j] = mlp->info[i][j];
  return SUGG_OK;
}

int32_t sugg_mlp_freeze(sugg_ctx* ctx, sugg_mlp* mlp, const float* params, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (!mlp || mlp->ctx != ctx || !params) return ctx->fail(SUGG_E_ARG, "mlp or params missing");
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  if (!mlp->frozen) {
    const hipError_t e = hipMalloc((void**)&mlp->frozen, sizeof(float) * mlp->nparam);
    if (e != hipSuccess) return ctx->hip(e, "frozen parameters");
  }
  hipError_t e = hipMemcpyAsync(mlp->frozen, params, sizeof(float) * mlp->nparam, hipMemcpyDeviceToDevice, stream);
  if (e != hipSuccess) return ctx->hip(e, "frozen parameters");
  mlp->packed_frozen = false;
  return SUGG_OK;
}

int32_t sugg_mlp_forward(sugg_ctx* ctx, sugg_mlp* mlp, const float* params, const float* x, int32_t batch,
                         float* y, int32_t keep, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  int rc = check_mlp(ctx, mlp, batch);
  if (rc) return rc;
  if (!params || !x || !y) return ctx->fail(SUGG_E_ARG, "null argument");
  return forward(ctx, mlp, params, x, batch, y, keep != 0, nullptr, nullptr, stream);
}

int32_t sugg_mlp_loss(sugg_ctx* ctx, sugg_mlp* mlp, const float* params, const float* x, const float* target,
                      int32_t batch, float* y, float* loss, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  int rc = check_mlp(ctx, mlp, batch);
  if (rc) return rc;
  if (!params || !x || !target || !loss) return ctx->fail(SUGG_E_ARG, "null argument");
  return forward(ctx, mlp, params, x, batch, y ? y : mlp->ybuf, true, target, loss, stream);
}

int32_t sugg_mlp_backward(sugg_ctx* ctx, sugg_mlp* mlp, const float* params, const float* dy, int32_t batch,
                          float* grads, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  int rc = check_mlp(ctx, mlp, batch);
  if (rc) return rc;
  if (!params || !grads) return ctx->fail(SUGG_E_ARG, "null argument");
  if (mlp->kept_batch != batch) return ctx->fail(SUGG_E_STATE, "backward needs a forward of this batch that kept activations");
  if (dy) {
    hipError_t e = launch_pack(dy, batch, mlp->out, mlp->dy, mlp->out, mlp->dyt, mlp->bm, stream);
    if (e != hipSuccess) return ctx->hip(e, "mlp pack dY");
  } else if (!mlp->have_dy) {
    return ctx->fail(SUGG_E_STATE, "no dY: pass dy or run sugg_mlp_loss first");
  }
  return backward(ctx, mlp, params, batch, grads, stream);
}

int32_t sugg_mlp_adam(sugg_ctx* ctx, sugg_mlp* mlp, float* params, const float* grads, float* m, float* v,
                      int32_t step, float lr, float beta1, float beta2, float eps, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (!mlp || mlp->ctx != ctx) return ctx->fail(SUGG_E_ARG, "mlp missing or from another context");
  if (!params || !grads || !m || !v) return ctx->fail(SUGG_E_ARG, "null argument");
  if (step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return ctx->fail(SUGG_E_ARG, "bad Adam hyper-parameters");
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  return ctx->hip(launch_adam(params, grads, m, v, mlp->nparam, lr, beta1, beta2, eps, step, stream), "adam");
}

int32_t sugg_mlp_train_step(sugg_ctx* ctx, sugg_mlp* mlp, float* params, float* grads, float* m, float* v,
                            int32_t step, float lr, const float* x, const float* target, int32_t batch, float* loss,
                            hipStream_t stream) {
  int rc = sugg_mlp_loss(ctx, mlp, params, x, target, batch, nullptr, loss, stream);
  if (rc) return rc;
  rc = backward(ctx, mlp, params, batch, grads, stream);
  if (rc) return rc;
  return sugg_mlp_adam(ctx, mlp, params, grads, m, v, step, lr, 0.9f, 0.999f, 1e-8f, stream);
}

int32_t sugg_mlp_infer(sugg_ctx* ctx, sugg_mlp* mlp, const float* x, int32_t batch, float* y, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (!x || !y) return ctx->fail(SUGG_E_ARG, "null argument");
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  return mlp_infer(ctx, mlp, x, batch, y, stream);
}

int32_t sugg_mlp_infer_rank(sugg_ctx* ctx, sugg_mlp* mlp, const float* x, int32_t batch, int32_t skip, int32_t n,
                            float tau, float* y, int32_t* idx, float* score, int32_t* count, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (!mlp || mlp->ctx != ctx) return ctx->fail(SUGG_E_ARG, "mlp missing or from another context");
  if (!mlp->frozen) return ctx->fail(SUGG_E_STATE, "mlp has no frozen parameters (sugg_mlp_freeze)");
  if (batch < 1 || batch > mlp->bm) return ctx->fail(SUGG_E_SHAPE, "batch %d outside [1, %d]", batch, mlp->bm);
  if (!x || !idx || !score || !count) return ctx->fail(SUGG_E_ARG, "null argument");
  if (n < 1 || n > SUGG_MAX_SUGGEST || skip < 0 || skip >= mlp->out || !std::isfinite(tau))
    return ctx->fail(SUGG_E_ARG, "bad n, skip or tau");
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  return infer_rank(ctx, mlp, x, batch, skip, n, tau, y, idx, score, count, stream);
}

int32_t sugg_mlp_train_epoch(sugg_ctx* ctx, sugg_mlp* mlp, float* params, float* grads, float* m, float* v,
                             int32_t step0, float lr, const float* X, const float* Y, int64_t n_rows,
                             const int32_t* perm, int32_t batch, int32_t steps, float* losses, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  int rc = check_mlp(ctx, mlp, batch);
  if (rc) return rc;
  if (!params || !grads || !m || !v || !X || !Y || !perm || (steps > 0 && !losses))
    return ctx->fail(SUGG_E_ARG, "null argument");
  if (steps < 0 || step0 < 0 || n_rows < 1 || n_rows > INT32_MAX || !(lr > 0.f))
    return ctx->fail(SUGG_E_ARG, "bad steps, step0, n_rows or lr");
  if (steps == 0) return SUGG_OK;
  hipError_t e = pack_weights(mlp, params, stream);
  if (e != hipSuccess) return ctx->hip(e, "mlp pack");
  AdamPackArgs ap{};
  ap.p = params;
  ap.g = grads;
  ap.m = m;
  ap.v = v;
  ap.n = mlp->nparam;
  ap.lr = lr;
  ap.b1 = 0.9f;
  ap.b2 = 0.999f;
  ap.eps = 1e-8f;
  const int64_t offs[3] = {mlp->off_w1, mlp->off_w2, mlp->off_w3};
  const int rows[3] = {mlp->hid, mlp->hid, mlp->out}, cols[3] = {mlp->in, mlp->hid, mlp->hid};
  __bf16* w[3] = {mlp->w1, mlp->w2, mlp->w3};
  __bf16* wt[3] = {nullptr, mlp->w2t, mlp->w3t};
  for (int l = 0; l < 3; ++l) {
    ap.off[l] = offs[l];
    ap.rows[l] = rows[l];
    ap.cols[l] = cols[l];
    ap.w[l] = w[l];
    ap.wt[l] = wt[l];
  }
  // mini-batch s: rows perm[s*batch ..) gathered into the packed input (the
  // gather of step s + 1 shares Adam's launch of step s)
  auto gather = [&](int s) {
    return GatherArgs{X, n_rows, mlp->in, perm + (int64_t)s * batch, batch, mlp->xb, mlp->in, mlp->xt, mlp->bm,
                      mlp->trow, ctx->d_status};
  };
  e = launch_gather_pack(gather(0), stream);
  if (e != hipSuccess) return ctx->hip(e, "mlp gather");
  for (int s = 0; s < steps; ++s) {
    rc = forward(ctx, mlp, params, nullptr, batch, mlp->ybuf, true, Y, nullptr, stream, false, mlp->trow, true);
    if (rc) return rc;
    rc = backward(ctx, mlp, params, batch, grads, stream, losses + s);
    if (rc) return rc;
    e = s + 1 < steps ? launch_adam_gather(ap, step0 + s + 1, gather(s + 1), stream)
                      : launch_adam_pack(ap, step0 + s + 1, stream);
    if (e != hipSuccess) return ctx->hip(e, "mlp adam");
  }
  mlp->packed_frozen = false;
  return SUGG_OK;
}

}  // extern "C"
