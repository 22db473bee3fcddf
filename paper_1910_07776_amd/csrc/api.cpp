// Host side of the C ABI declared in include/sugg.h: contexts, plans (the
// ragged work lists), argument validation and kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "sugg.h"

using namespace sugg;

#include "ctx.hpp"

#include "plan.hpp"

namespace {

int cu_count(int device) {
  int c = 0;
  if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c <= 0) c = 256;
  return c;
}

template <typename V>
hipError_t upload(V*& dst, const void* src, size_t bytes) {
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc((void**)&dst, bytes);
  if (e != hipSuccess) return e;
  if (src) e = hipMemcpy((void*)dst, src, bytes, hipMemcpyHostToDevice);
  return e;
}

int check_params(sugg_ctx* ctx, const sugg_params& p) {
  if (!(p.lambda >= 0.0) || !std::isfinite(p.lambda)) return ctx->fail(SUGG_E_ARG, "lambda must be finite and >= 0");
  if (std::isnan(p.tau)) return ctx->fail(SUGG_E_ARG, "tau is NaN");
  if (p.n_suggest < 1 || p.n_suggest > SUGG_MAX_SUGGEST)
    return ctx->fail(SUGG_E_ARG, "n_suggest must be in [1, %d]", SUGG_MAX_SUGGEST);
  return SUGG_OK;
}

// Build the ragged work list: kernels grouped by B (largest first, a greedy
// longest-processing-time order), small kernels packed into items of about
// `target` rows, kernels of >= target rows alone.
void build_items(const std::vector<int32_t>& nopts, const std::vector<int64_t>& row_off, int target,
                 std::vector<Item>& items, std::vector<int32_t>& item_kernels, int& max_rows, int& max_nk) {
  const int K = (int)nopts.size();
  std::vector<int32_t> order(K);
  for (int k = 0; k < K; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nopts[a] > nopts[b]; });
  items.clear();
  item_kernels = order;
  max_rows = 1;
  max_nk = 1;
  int i = 0;
  while (i < K) {
    const int B = nopts[order[i]];
    const int rows = 1 << B;
    const int per = rows >= target ? 1 : target / rows;
    int j = i;
    while (j < K && j - i < per && nopts[order[j]] == B) ++j;
    Item it;
    std::memset(&it, 0, sizeof it);
    it.first = i;
    it.nk = j - i;
    it.B = B;
    it.R = it.nk << B;
    bool adjacent = true;
    for (int t = i; t + 1 < j; ++t) adjacent &= order[t + 1] == order[t] + 1;
    it.row0 = adjacent ? row_off[order[i]] : -1;
    items.push_back(it);
    max_rows = std::max(max_rows, it.R);
    max_nk = std::max(max_nk, it.nk);
    i = j;
  }
}

// The plan's work list for items of about `target` rows (build_items), the
// arithmetic geometry of batches whose kernels all have one B, and the
// kernel records; replaces a previous list.  Synchronous.
hipError_t plan_items(sugg_plan* p, int target) {
  const int K = p->K;
  std::vector<Item> items;
  std::vector<int32_t> ik;
  build_items(p->nopts, p->row_off, target, items, ik, p->max_item_rows, p->max_item_kernels);
  p->item_rows = target;
  // a batch whose kernels all have the same B gets arithmetic item geometry
  p->uni_B = -1;
  p->uni_nk = 0;
  p->uni_ops = 0;
  p->uni_opt_lo = p->uni_opt_hi = 0;
  if (K > 0 && std::all_of(p->nopts.begin(), p->nopts.end(), [&](int32_t b) { return b == p->nopts[0]; })) {
    p->uni_B = p->nopts[0];
    p->uni_nk = items[0].nk;
    // and when every kernel also carries the same optimisation ids
    bool same = true;
    for (int k = 1; k < K && same; ++k)
      for (int b = 0; b < p->uni_B; ++b) same &= p->opt_ids[p->opt_off[k] + b] == p->opt_ids[b];
    if (same) {
      p->uni_ops = 1;
      for (int b = 0; b < p->uni_B; ++b) {
        const uint64_t o = (uint64_t)(uint8_t)p->opt_ids[b];
        if (b < 8) p->uni_opt_lo |= o << (8 * b);
        else p->uni_opt_hi |= o << (8 * (b - 8));
      }
    }
  }
  p->n_items = (int)items.size();
  std::vector<KRec> recs(ik.size());
  for (size_t i = 0; i < ik.size(); ++i) {
    const int k = ik[i];
    KRec& r = recs[i];
    std::memset(&r, 0, sizeof r);
    r.row_off = p->row_off[k];
    r.kid = k;
    for (int b = 0; b < p->nopts[k]; ++b) r.opt[b] = (uint8_t)p->opt_ids[p->opt_off[k] + b];
  }
  // streaming form: consecutive whole kernels in memory order, a chunk closed
  // before it would pass `target` rows (a larger kernel is a chunk alone).
  // The kernels of the last tenth of the rows go into chunks of a quarter of
  // the target, and the chunks are dispatched largest first: the workgroups
  // that start last are then short, and the device stays nearly full until
  // the end of the launch (with equal chunks throughout, the last round of
  // workgroups drained over most of a chunk's lifetime).
  std::vector<Chunk> chunks;
  std::vector<CRec> crec(K);
  p->chunk_max_rows = 1;
  p->chunk_max_nk = 1;
  const int64_t n_rows = K > 0 ? p->row_off[K] : 0;
  const int tail_target = std::max(target / 4, 128);
  for (int k = 0; k < K;) {
    Chunk c;
    std::memset(&c, 0, sizeof c);
    c.row0 = p->row_off[k];
    c.k0 = k;
    const int64_t cap = 10 * c.row0 >= 9 * n_rows ? std::min(target, tail_target) : target;
    int64_t rows = 0;
    while (k < K && (c.nk == 0 || rows + ((int64_t)1 << p->nopts[k]) <= cap)) {
      CRec& r = crec[k];
      std::memset(&r, 0, sizeof r);
      r.rel = (int16_t)rows;   // < max(target, 2^SUGG_MAX_OPTS) <= 4096
      r.B = (int8_t)p->nopts[k];
      for (int b = 0; b < p->nopts[k]; ++b) r.op[b] = (uint8_t)p->opt_ids[p->opt_off[k] + b];
      rows += (int64_t)1 << p->nopts[k];
      ++c.nk;
      ++k;
    }
    c.R = (int32_t)rows;
    p->chunk_max_rows = std::max(p->chunk_max_rows, c.R);
    p->chunk_max_nk = std::max(p->chunk_max_nk, c.nk);
    chunks.push_back(c);
  }
  std::stable_sort(chunks.begin(), chunks.end(), [](const Chunk& x, const Chunk& y) { return x.R > y.R; });
  p->n_chunks = (int)chunks.size();
  dfree(p->d_items);
  dfree(p->d_recs);
  dfree(p->d_chunks);
  dfree(p->d_crec);
  hipError_t e = upload(p->d_items, items.data(), sizeof(Item) * items.size());
  if (e == hipSuccess) e = upload(p->d_recs, recs.data(), sizeof(KRec) * recs.size());
  if (e == hipSuccess) e = upload(p->d_chunks, chunks.data(), sizeof(Chunk) * chunks.size());
  if (e == hipSuccess) e = upload(p->d_crec, crec.data(), sizeof(CRec) * crec.size());
  return e;
}

template <typename T>
const T* model_mu(sugg_ctx* c);
template <>
const float* model_mu<float>(sugg_ctx* c) { return c->mu32; }
template <>
const double* model_mu<double>(sugg_ctx* c) { return c->mu64; }
template <typename T>
const T* model_isg(sugg_ctx* c);
template <>
const float* model_isg<float>(sugg_ctx* c) { return c->isg32; }
template <>
const double* model_isg<double>(sugg_ctx* c) { return c->isg64; }
template <typename T>
const T* model_W(sugg_ctx* c);
template <>
const float* model_W<float>(sugg_ctx* c) { return c->W32; }
template <>
const double* model_W<double>(sugg_ctx* c) { return c->W64; }

__global__ void inv_kernel(const double* sig, double* isg, int E) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < E) isg[j] = 1.0 / sig[j];
}

__global__ void stats_to_f32_kernel(const double* mu, const double* sig, float* mu32, float* isg32, int E) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < E) {
    mu32[j] = (float)mu[j];
    isg32[j] = (float)(1.0 / sig[j]);
  }
}

int ensure_stat_ws(sugg_ctx* ctx, sugg_plan* p) {
  if (p->d_stat_partial) return SUGG_OK;
  return ctx->hip(hipMalloc((void**)&p->d_stat_partial, sizeof(double) * 2 * p->E * p->stat_chunks),
                  "statistics workspace");
}

int prepare_fit(sugg_ctx* ctx, sugg_plan* p) {
  if (p->fit_ready) return SUGG_OK;
  const int E = p->E, D = p->D;
  // per-optimisation list of (kernel, local bit); pair space prefix sums
  std::vector<std::vector<std::pair<int, int>>> lists(D);
  for (int k = 0; k < p->K; ++k)
    for (int b = 0; b < p->nopts[k]; ++b) lists[p->opt_ids[p->opt_off[k] + b]].push_back({k, b});
  int64_t total = 0;
  for (int o = 0; o < D; ++o) total += p->opt_pairs[o];
  const int target_items = 4 * cu_count(ctx->device);
  int64_t chunk = total / std::max(1, target_items);
  chunk = std::max<int64_t>(chunk, 256);
  chunk = (chunk + 31) / 32 * 32;
  std::vector<int64_t> pbase, prow0;
  std::vector<int32_t> pbit, owb(D + 1, 0);
  std::vector<GramWork> work;
  for (int o = 0; o < D; ++o) {
    owb[o] = (int)work.size();
    const int lb = (int)pbase.size();
    int64_t acc = 0;
    for (auto& kb : lists[o]) {
      pbase.push_back(acc);
      prow0.push_back(p->row_off[kb.first]);
      pbit.push_back(kb.second);
      acc += (int64_t)1 << (p->nopts[kb.first] - 1);
    }
    const int le = (int)pbase.size();
    for (int64_t s0 = 0; s0 < acc; s0 += chunk) {
      GramWork w;
      w.opt = o;
      w.list_begin = lb;
      w.list_end = le;
      w.pad = 0;
      w.s_begin = s0;
      w.s_end = std::min(acc, s0 + chunk);
      work.push_back(w);
    }
  }
  owb[D] = (int)work.size();
  hipError_t e = hipSuccess;
  const size_t stride = (size_t)E * E + 2 * E + 2;
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_z64, sizeof(double) * std::max<int64_t>(1, p->N * E));
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_lcyc64, sizeof(double) * std::max<int64_t>(1, p->N));
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_gram_partial, sizeof(double) * stride * std::max<size_t>(1, work.size()));
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_reduced, sizeof(double) * stride * std::max(1, D));
  if (e == hipSuccess && sizeof(double) * (size_t)(E + 1) * (E + 1) > 150 * 1024)
    e = hipMalloc((void**)&p->d_solveA, sizeof(double) * (size_t)(E + 1) * (E + 1) * std::max(1, D));
  if (e == hipSuccess) e = upload(p->d_gwork, work.data(), sizeof(GramWork) * work.size());
  if (e == hipSuccess) e = upload(p->d_pair_base, pbase.data(), sizeof(int64_t) * pbase.size());
  if (e == hipSuccess) e = upload(p->d_pair_row0, prow0.data(), sizeof(int64_t) * prow0.size());
  if (e == hipSuccess) e = upload(p->d_pair_bit, pbit.data(), sizeof(int32_t) * pbit.size());
  if (e == hipSuccess) e = upload(p->d_opt_work_begin, owb.data(), sizeof(int32_t) * owb.size());
  if (e != hipSuccess) return ctx->hip(e, "fit workspace");
  p->n_gwork = (int)work.size();
  p->fit_ready = true;
  return SUGG_OK;
}

template <typename T>
int run_fit(sugg_ctx* ctx, sugg_plan* p, const T* c, const T* cyc, hipStream_t s) {
  int rc = prepare_fit(ctx, p);
  if (!rc) rc = ensure_stat_ws(ctx, p);
  if (rc) return rc;
  rc = ctx->ensure_model(p->E, p->D);
  if (rc) return rc;
  T* mu_t = (T*)(sizeof(T) == 4 ? (void*)ctx->mu32 : (void*)ctx->mu64);
  T* isg_t = (T*)(sizeof(T) == 4 ? (void*)ctx->isg32 : (void*)ctx->isg64);
  rc = ctx->hip(launch_colstats<T>(c, cyc, p->N, p->E, p->d_stat_partial, p->stat_chunks, ctx->mu64,
                                   ctx->sig64, mu_t, isg_t, ctx->d_status, s), "column statistics");
  if (rc) return rc;
  (void)hipGetLastError();
  hipLaunchKernelGGL(inv_kernel, dim3((p->E + 255) / 256), dim3(256), 0, s, ctx->sig64, ctx->isg64, p->E);
  hipLaunchKernelGGL(stats_to_f32_kernel, dim3((p->E + 255) / 256), dim3(256), 0, s, ctx->mu64, ctx->sig64,
                     ctx->mu32, ctx->isg32, p->E);
  rc = ctx->hip(hipGetLastError(), "statistics");
  if (rc) return rc;
  rc = ctx->hip(launch_zfeat64<T>(c, cyc, p->N, p->E, ctx->mu64, ctx->sig64, p->d_z64, p->d_lcyc64, s), "features");
  if (rc) return rc;
  GramArgs g;
  g.z64 = p->d_z64;
  g.lcyc64 = p->d_lcyc64;
  g.E = p->E;
  g.work = p->d_gwork;
  g.n_work = p->n_gwork;
  g.pair_base = p->d_pair_base;
  g.pair_row0 = p->d_pair_row0;
  g.pair_bit = p->d_pair_bit;
  g.partial = p->d_gram_partial;
  rc = ctx->hip(launch_gram(g, s), "gram");
  if (rc) return rc;
  SolveArgs sa;
  sa.partial = p->d_gram_partial;
  sa.opt_work_begin = p->d_opt_work_begin;
  sa.E = p->E;
  sa.D = p->D;
  sa.lambda = ctx->params.lambda;
  sa.A = p->d_solveA;
  sa.reduced = p->d_reduced;
  sa.W64 = ctx->W64;
  sa.W32 = ctx->W32;
  sa.status = ctx->d_status;
  rc = ctx->hip(launch_solve(sa, s), "solve");
  if (rc) return rc;
  for (int o = 0; o < p->D; ++o) ctx->counts[o] = p->opt_pairs[o];
  ctx->has_stats = ctx->has_model = true;
  return SUGG_OK;
}

int check_model_for(sugg_ctx* ctx, const sugg_plan* p) {
  if (!ctx->has_model) return ctx->fail(SUGG_E_STATE, "no fitted model");
  if (ctx->E != p->E) return ctx->fail(SUGG_E_SHAPE, "plan has E=%d, model E=%d", p->E, ctx->E);
  for (int o = 0; o < p->D; ++o)
    // the plan uses o exactly when it has before/after pairs for it
    if (p->opt_pairs[o] > 0 && (o >= ctx->D || ctx->counts[o] == 0))
      return ctx->fail(SUGG_E_UNTRAINED_OPT, "optimisation id %d has no fitted model", o);
  return SUGG_OK;
}

// Upper bound of the fused kernel's dynamic LDS (weights, per-item tables,
// metadata, cross-wave lists) for the widest configuration.
size_t path_lds_bound(size_t tsize, int D, int E, int max_rows, int max_nk, int max_B) {
  const int vpl = E <= 64 ? 4 : (E <= 128 ? 8 : 16);
  return tsize * ((size_t)D * 16 * vpl + D + 2 * 16 * vpl + 2 * (size_t)max_rows) + 16 * (size_t)max_nk * (1 + max_B) +
         (tsize + 8) * 8 * 8 + 256;
}

constexpr size_t kLdsPerWorkgroup = 160 * 1024;
constexpr int kTuneItems[] = {64, 128, 256, 512, 1024};
constexpr int kTuneWaves[] = {2, 4, 8};
constexpr int kTuneUnroll[] = {1, 2, 4};
constexpr int kTuneFinalists = 4;   // candidates timed again before the choice
static_assert(5 * (3 * 3 + 3) + 1 == SUGG_TUNE_CANDIDATES, "autotuner candidate count");

template <typename T>
int run_path(sugg_ctx* ctx, const sugg_plan* p, const T* c, const T* cyc, T* grid, T* table,
             int32_t* idx, T* score, int32_t* count, int n, hipStream_t s, const int32_t* kmask = nullptr) {
  if (p->K == 0) return SUGG_OK;
  if (path_lds_bound(sizeof(T), ctx->D, p->E, p->max_item_rows, p->max_item_kernels, p->Bmax) > kLdsPerWorkgroup)
    return ctx->fail(SUGG_E_BUDGET, "model of %d optimisations x %d events does not fit in LDS", ctx->D, p->E);
  PathArgs<T> a;
  a.judge = nullptr;
  a.kmask = kmask;
  a.counters = c;
  a.cycles = cyc;
  a.E = p->E;
  a.D = ctx->D;
  a.items = p->d_items;
  a.recs = p->d_recs;
  a.K = p->K;
  a.uni_B = p->uni_B;
  a.uni_nk = p->uni_nk;
  a.uni_ops = p->uni_ops;
  a.uni_opt_lo = p->uni_opt_lo;
  a.uni_opt_hi = p->uni_opt_hi;
  a.n_items = p->n_items;
  a.queue = p->d_queue;
  a.mu = model_mu<T>(ctx);
  a.isg = model_isg<T>(ctx);
  a.W = model_W<T>(ctx);
  a.ldw = sizeof(T) == 4 ? w32_ld(p->E) : p->E + 1;
  a.grid = grid;
  a.grid_ld = p->Bmax;
  a.table = table;
  a.idx_out = idx;
  a.score_out = score;
  a.count_out = count;
  a.n = n;
  a.tau = (T)ctx->params.tau;
  a.status = ctx->d_status;
  if (p->cfg.unroll == 0 && p->split_ok() && !grid && !kmask)
    return ctx->hip(launch_path_split<T>(a, p->d_arrivals, (T*)p->d_split_edges, s), "scoring kernel");
  if (p->cfg.unroll < 0 && !grid && !kmask &&
      path_chunk_lds(sizeof(T), ctx->D, p->E, p->chunk_max_rows, p->chunk_max_nk) <= kLdsPerWorkgroup) {
    ChunkArgs<T> ch;
    ch.counters = c;
    ch.cycles = cyc;
    ch.E = p->E;
    ch.D = ctx->D;
    ch.W = a.W;
    ch.ldw = a.ldw;
    ch.mu = a.mu;
    ch.isg = a.isg;
    ch.recs = p->d_crec;
    ch.chunks = p->d_chunks;
    ch.n_chunks = p->n_chunks;
    ch.max_rows = p->chunk_max_rows;
    ch.max_nk = p->chunk_max_nk;
    ch.table = table;
    ch.idx_out = idx;
    ch.score_out = score;
    ch.count_out = count;
    ch.n = n;
    ch.tau = (T)ctx->params.tau;
    ch.status = ctx->d_status;
    return ctx->hip(launch_path_chunks<T>(ch, -p->cfg.unroll, s), "scoring kernel (streaming form)");
  }
  PathLaunch cfg = p->cfg;
  if (cfg.unroll <= 0) cfg.unroll = 1;   // the split or streaming form does not apply: fused, one row per stage
  return ctx->hip(launch_path<T>(a, p->max_item_rows, p->max_item_kernels, std::max(1, p->Bmax), cfg, s),
                  "scoring kernel");
}

}  // namespace

namespace {

template <typename T>
int run_judge(sugg_ctx* ctx, const sugg_plan* p, const T* c, const T* cyc, const int32_t* cand, int32_t C,
                     T* out, const T* ref, double tol, int32_t* flag, int32_t accumulate, hipStream_t s,
                     int32_t C2 = 0, const int32_t* cand2 = nullptr, T* out2 = nullptr, const T* ref2 = nullptr) {
  JudgeArgs<T> j;
  j.counters = c;
  j.cycles = cyc;
  j.E = p->E;
  j.D = ctx->D;
  j.W = model_W<T>(ctx);
  j.ldw = sizeof(T) == 4 ? w32_ld(p->E) : p->E + 1;
  j.mu = model_mu<T>(ctx);
  j.isg = model_isg<T>(ctx);
  j.row_off = p->d_row_off;
  j.nopts = p->d_nopts;
  j.opt_off = p->d_opt_off;
  j.opt_ids = p->d_opt_ids;
  j.K = p->K;
  j.C = C;
  j.cand = cand;
  j.out = out;
  j.ref = ref;
  j.tol = tol;
  j.flag = flag;
  j.accumulate = accumulate;
  j.status = ctx->d_status;
  j.C2 = C2;
  j.cand2 = cand2;
  j.out2 = out2;
  j.ref2 = ref2;
  PathArgs<T> a{};
  a.judge = &j;
  a.E = p->E;
  return ctx->hip(launch_path<T>(a, 1, 1, 1, p->cfg, s), "judge");
}


template <typename T>
int run_paths(sugg_ctx* ctx, const sugg_plan* p, const T* c, const T* cyc, bool greedy, T* table, int32_t* idx,
              T* score, int32_t* count, int32_t* path, int32_t* steps, T* gain, hipStream_t s) {
  PathsArgs<T> a{};
  a.counters = c;
  a.cycles = cyc;
  a.E = p->E;
  a.D = ctx->D;
  a.ldw = sizeof(T) == 4 ? w32_ld(p->E) : p->E + 1;
  a.W = model_W<T>(ctx);
  a.mu = model_mu<T>(ctx);
  a.isg = model_isg<T>(ctx);
  a.row_off = p->d_row_off;
  a.nopts = p->d_nopts;
  a.opt_off = p->d_opt_off;
  a.opt_ids = p->d_opt_ids;
  a.K = p->K;
  a.Bmax = p->Bmax;
  a.n = ctx->params.n_suggest;
  a.tau = (T)ctx->params.tau;
  a.table = table;
  a.idx_out = idx;
  a.score_out = score;
  a.count_out = count;
  a.path_out = path;
  a.steps_out = steps;
  a.gain_out = gain;
  a.status = ctx->d_status;
  return ctx->hip(launch_paths<T>(a, greedy, s), greedy ? "greedy" : "all-paths");
}

int paths_checks(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles) {
  if (!plan || plan->ctx != ctx) return ctx->fail(SUGG_E_ARG, "plan missing or from another context");
  if (plan->N > 0 && (!counters || !cycles)) return ctx->fail(SUGG_E_ARG, "null counters or cycles");
  int rc = check_model_for(ctx, plan);
  if (rc) return rc;
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  return SUGG_OK;
}
}  // namespace

extern "C" {

int32_t sugg_create(sugg_ctx** out, int32_t device, const sugg_params* params) {
  if (!out) return SUGG_E_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SUGG_E_ARG;
  sugg_ctx* c = new (std::nothrow) sugg_ctx();
  if (!c) return SUGG_E_BUDGET;
  c->device = device;
  c->params.lambda = 1e-2;
  c->params.tau = std::log(1.05);
  c->params.n_suggest = 3;
  if (params) {
    if (check_params(c, *params)) {
      delete c;
      return SUGG_E_ARG;
    }
    c->params = *params;
  }
  if (hipSetDevice(device) != hipSuccess || hipMalloc((void**)&c->d_status, sizeof(int32_t)) != hipSuccess ||
      hipMemset(c->d_status, 0, sizeof(int32_t)) != hipSuccess || noalloc_scratch_setup(device) != SUGG_OK) {
    delete c;
    return SUGG_E_HIP;
  }
  *out = c;
  return SUGG_OK;
}

void sugg_destroy(sugg_ctx* ctx) {
  if (!ctx) return;
  (void)device_ok(ctx);
  ctx->free_model();
  ibk_model_free(ctx->ibk);
  m5p_model_free(ctx->m5p);
  dfree(ctx->d_status);
  delete ctx;
}

const char* sugg_last_error(const sugg_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int32_t sugg_set_params(sugg_ctx* ctx, const sugg_params* params) {
  if (!ctx || !params) return SUGG_E_ARG;
  int rc = check_params(ctx, *params);
  if (rc) return rc;
  ctx->params = *params;
  return SUGG_OK;
}

int32_t sugg_get_params(const sugg_ctx* ctx, sugg_params* out) {
  if (!ctx || !out) return SUGG_E_ARG;
  *out = ctx->params;
  return SUGG_OK;
}

int32_t sugg_plan_create(sugg_ctx* ctx, int32_t K, int32_t E, int32_t D, int32_t dtype, const int32_t* nopts,
                         const int32_t* opt_ids, sugg_plan** out) {
  if (!ctx || !out) return SUGG_E_ARG;
  *out = nullptr;
  if (K < 0 || (K > 0 && !nopts)) return ctx->fail(SUGG_E_ARG, "bad K or null nopts");
  if (E < 1 || E > SUGG_MAX_EVENTS) return ctx->fail(SUGG_E_SHAPE, "E=%d outside [1, %d]", E, SUGG_MAX_EVENTS);
  if (D < 0 || D > SUGG_MAX_GLOBAL_OPTS) return ctx->fail(SUGG_E_SHAPE, "D=%d outside [0, %d]", D, SUGG_MAX_GLOBAL_OPTS);
  if (dtype != SUGG_F32 && dtype != SUGG_F64) return ctx->fail(SUGG_E_ARG, "bad dtype %d", dtype);
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device %d", ctx->device);
  sugg_plan* p = new (std::nothrow) sugg_plan();
  if (!p) return ctx->fail(SUGG_E_BUDGET, "out of host memory");
  p->ctx = ctx;
  p->device = ctx->device;
  p->K = K;
  p->E = E;
  p->D = D;
  p->dtype = dtype;
  p->nopts.assign(nopts, nopts + K);
  p->row_off.assign(K + 1, 0);
  p->opt_off.assign(K + 1, 0);
  for (int k = 0; k < K; ++k) {
    const int B = p->nopts[k];
    if (B < 0 || B > SUGG_MAX_OPTS) {
      delete p;
      return ctx->fail(SUGG_E_SHAPE, "kernel %d has %d optimisations (max %d)", k, B, SUGG_MAX_OPTS);
    }
    p->Bmax = std::max(p->Bmax, B);
    p->row_off[k + 1] = p->row_off[k] + ((int64_t)1 << B);
    p->opt_off[k + 1] = p->opt_off[k] + B;
  }
  p->N = p->row_off[K];
  const int64_t nid = p->opt_off[K];
  if (nid > 0 && !opt_ids) {
    delete p;
    return ctx->fail(SUGG_E_ARG, "null opt_ids");
  }
  p->opt_ids.assign(opt_ids, opt_ids + nid);
  p->opt_pairs.assign(D, 0);
  for (int k = 0; k < K; ++k) {
    for (int64_t i = p->opt_off[k]; i < p->opt_off[k + 1]; ++i) {
      const int o = p->opt_ids[i];
      if (o < 0 || o >= D || (i > p->opt_off[k] && o <= p->opt_ids[i - 1])) {
        delete p;
        return ctx->fail(SUGG_E_SHAPE, "kernel %d: optimisation ids must ascend strictly within [0, %d)", k, D);
      }
      p->opt_pairs[o] += (int64_t)1 << (p->nopts[k] - 1);
    }
  }
  // item size: enough items to spread over the chip, at most 256 rows packed
  const int cus = cu_count(ctx->device);
  int target = 256;
  while (target > 64 && p->N / target < 2 * cus) target >>= 1;
  p->stat_chunks = colstats_chunks(std::max<int64_t>(p->N, 1));
  hipError_t e = plan_items(p, target);
  if (e == hipSuccess) e = upload(p->d_row_off, p->row_off.data(), sizeof(int64_t) * (K + 1));
  if (e == hipSuccess) e = upload(p->d_opt_off, p->opt_off.data(), sizeof(int64_t) * (K + 1));
  if (e == hipSuccess) e = upload(p->d_opt_ids, p->opt_ids.data(), sizeof(int32_t) * nid);
  if (e == hipSuccess) e = upload(p->d_nopts, p->nopts.data(), sizeof(int32_t) * K);
  if (e == hipSuccess) e = upload(p->d_queue, nullptr, 64);
  if (e == hipSuccess) e = hipMemset(p->d_queue, 0, 64);
  if (e == hipSuccess && p->uni_B >= 0 && p->uni_B <= 6 && p->uni_ops) {
    e = upload(p->d_arrivals, nullptr, sizeof(int32_t) * K);
    if (e == hipSuccess) e = hipMemset(p->d_arrivals, 0, sizeof(int32_t) * K);
    if (e == hipSuccess) e = upload(p->d_split_edges, nullptr, (dtype == SUGG_F32 ? 4 : 8) * (size_t)p->N);
  }
  if (e != hipSuccess) {
    delete p;
    return ctx->hip(e, "plan upload");
  }
  *out = p;
  return SUGG_OK;
}

void sugg_plan_destroy(sugg_plan* plan) {
  if (!plan) return;
  int cur = -1;
  if (hipGetDevice(&cur) == hipSuccess && cur != plan->device) (void)hipSetDevice(plan->device);
  delete plan;
}

int64_t sugg_plan_rows(const sugg_plan* plan) { return plan ? plan->N : -1; }
int32_t sugg_plan_max_opts(const sugg_plan* plan) { return plan ? plan->Bmax : -1; }

}  // extern "C"

// sugg_load_features and its variant without allocation: with partial ==
// nullptr the column-statistics partials go to the plan's workspace and the
// model storage is (re)allocated as needed; otherwise they go to `partial`
// (a device buffer of at least 2 * E * stat_chunks doubles) and the call
// allocates nothing, so the model storage must already hold E columns.
int load_features_core(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles, int32_t mode,
                       void* z_out, hipStream_t stream, double* partial) {
  if (!ctx) return SUGG_E_ARG;
  if (!plan || plan->ctx != ctx) return ctx->fail(SUGG_E_ARG, "plan missing or from another context");
  if (mode & ~(SUGG_FIT_STATS | SUGG_APPLY | SUGG_BASELINE) || mode == 0 ||
      ((mode & SUGG_BASELINE) && !(mode & SUGG_APPLY)))
    return ctx->fail(SUGG_E_ARG, "bad mode %d", mode);
  if (plan->N > 0 && (!counters || !cycles)) return ctx->fail(SUGG_E_ARG, "null counters or cycles");
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  sugg_plan* p = const_cast<sugg_plan*>(plan);
  int rc = SUGG_OK;
  if (mode & SUGG_FIT_STATS) {
    if (p->N == 0) return ctx->fail(SUGG_E_SHAPE, "statistics need at least one row");
    if (partial) {
      if (!ctx->mu64 || ctx->E != p->E)
        return ctx->fail(SUGG_E_STATE, "model storage for E=%d not set up (one sugg_load_features, sugg_fit or "
                         "sugg_model_set of this E first)", p->E);
    } else {
      rc = ctx->ensure_model(p->E, (ctx->has_model && ctx->E == p->E) ? ctx->D : 0);
      if (!rc) rc = ensure_stat_ws(ctx, p);
      if (rc) return rc;
      partial = p->d_stat_partial;
    }
    if (p->dtype == SUGG_F32)
      rc = ctx->hip(launch_colstats<float>((const float*)counters, (const float*)cycles, p->N, p->E, partial,
                                           p->stat_chunks, ctx->mu64, ctx->sig64, ctx->mu32, ctx->isg32,
                                           ctx->d_status, stream), "column statistics");
    else
      rc = ctx->hip(launch_colstats<double>((const double*)counters, (const double*)cycles, p->N, p->E,
                                            partial, p->stat_chunks, ctx->mu64, ctx->sig64, ctx->mu64,
                                            ctx->isg64, ctx->d_status, stream), "column statistics");
    if (rc) return rc;
    (void)hipGetLastError();
    hipLaunchKernelGGL(inv_kernel, dim3((p->E + 255) / 256), dim3(256), 0, stream, ctx->sig64, ctx->isg64, p->E);
    hipLaunchKernelGGL(stats_to_f32_kernel, dim3((p->E + 255) / 256), dim3(256), 0, stream, ctx->mu64, ctx->sig64,
                       ctx->mu32, ctx->isg32, p->E);
    rc = ctx->hip(hipGetLastError(), "statistics");
    if (rc) return rc;
    ctx->has_stats = true;
    // new statistics invalidate fitted weights
    ctx->has_model = false;
  }
  if (mode & SUGG_APPLY) {
    if (!ctx->has_stats) return ctx->fail(SUGG_E_STATE, "no column statistics");
    if (ctx->E != p->E) return ctx->fail(SUGG_E_SHAPE, "plan E=%d, statistics E=%d", p->E, ctx->E);
    if (z_out && (mode & SUGG_BASELINE)) {
      if (p->dtype == SUGG_F32)
        rc = ctx->hip(launch_standardize_rows<float>((const float*)counters, (const float*)cycles, p->d_row_off, p->K,
                                                     p->E, ctx->mu32, ctx->isg32, (float*)z_out, ctx->d_status, stream),
                      "standardize");
      else
        rc = ctx->hip(launch_standardize_rows<double>((const double*)counters, (const double*)cycles, p->d_row_off,
                                                      p->K, p->E, ctx->mu64, ctx->isg64, (double*)z_out, ctx->d_status,
                                                      stream),
                      "standardize");
    } else if (z_out) {
      if (p->dtype == SUGG_F32)
        rc = ctx->hip(launch_standardize<float>((const float*)counters, (const float*)cycles, p->N, p->E, ctx->mu32,
                                                ctx->isg32, (float*)z_out, ctx->d_status, stream), "standardize");
      else
        rc = ctx->hip(launch_standardize<double>((const double*)counters, (const double*)cycles, p->N, p->E,
                                                 ctx->mu64, ctx->isg64, (double*)z_out, ctx->d_status, stream),
                      "standardize");
    }
  }
  return rc;
}

extern "C" {

int32_t sugg_load_features(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles,
                           int32_t mode, void* z_out, hipStream_t stream) {
  return load_features_core(ctx, plan, counters, cycles, mode, z_out, stream, nullptr);
}

int32_t sugg_fit(sugg_ctx* ctx, const sugg_plan* train, const void* counters, const void* cycles, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (!train || train->ctx != ctx) return ctx->fail(SUGG_E_ARG, "plan missing or from another context");
  if (train->N == 0) return ctx->fail(SUGG_E_SHAPE, "empty training batch");
  if (!counters || !cycles) return ctx->fail(SUGG_E_ARG, "null counters or cycles");
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  sugg_plan* p = const_cast<sugg_plan*>(train);
  if (p->dtype == SUGG_F32) return run_fit<float>(ctx, p, (const float*)counters, (const float*)cycles, stream);
  return run_fit<double>(ctx, p, (const double*)counters, (const double*)cycles, stream);
}

int32_t sugg_predict(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles, void* grid_out,
                     void* table_out, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (!plan || plan->ctx != ctx) return ctx->fail(SUGG_E_ARG, "plan missing or from another context");
  if (plan->N > 0 && (!counters || !cycles || !table_out)) return ctx->fail(SUGG_E_ARG, "null counters, cycles or table");
  int rc = check_model_for(ctx, plan);
  if (rc) return rc;
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  if (plan->dtype == SUGG_F32)
    return run_path<float>(ctx, plan, (const float*)counters, (const float*)cycles, (float*)grid_out,
                           (float*)table_out, nullptr, nullptr, nullptr, 0, stream);
  return run_path<double>(ctx, plan, (const double*)counters, (const double*)cycles, (double*)grid_out,
                          (double*)table_out, nullptr, nullptr, nullptr, 0, stream);
}

int32_t sugg_suggest(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles, void* table_out,
                     int32_t* idx_out, void* score_out, int32_t* count_out, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (!plan || plan->ctx != ctx) return ctx->fail(SUGG_E_ARG, "plan missing or from another context");
  if (plan->K > 0 && (!counters || !cycles || !idx_out || !score_out || !count_out))
    return ctx->fail(SUGG_E_ARG, "null argument");
  int rc = check_model_for(ctx, plan);
  if (rc) return rc;
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  const int n = ctx->params.n_suggest;
  if (plan->dtype == SUGG_F32)
    return run_path<float>(ctx, plan, (const float*)counters, (const float*)cycles, nullptr, (float*)table_out,
                           idx_out, (float*)score_out, count_out, n, stream);
  return run_path<double>(ctx, plan, (const double*)counters, (const double*)cycles, nullptr, (double*)table_out,
                          idx_out, (double*)score_out, count_out, n, stream);
}

int32_t sugg_suggest_subset(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles,
                            const int32_t* kmask, void* table_out, int32_t* idx_out, void* score_out,
                            int32_t* count_out, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (!plan || plan->ctx != ctx) return ctx->fail(SUGG_E_ARG, "plan missing or from another context");
  if (plan->K > 0 && (!counters || !cycles || !kmask || !idx_out || !score_out || !count_out))
    return ctx->fail(SUGG_E_ARG, "null argument");
  int rc = check_model_for(ctx, plan);
  if (rc) return rc;
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  const int n = ctx->params.n_suggest;
  if (plan->dtype == SUGG_F32)
    return run_path<float>(ctx, plan, (const float*)counters, (const float*)cycles, nullptr, (float*)table_out,
                           idx_out, (float*)score_out, count_out, n, stream, kmask);
  return run_path<double>(ctx, plan, (const double*)counters, (const double*)cycles, nullptr, (double*)table_out,
                          idx_out, (double*)score_out, count_out, n, stream, kmask);
}

int32_t sugg_judge(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles,
                   const int32_t* cand, int32_t C, void* out, const void* ref, double tol, int32_t* flag_out,
                   int32_t accumulate, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (!plan || plan->ctx != ctx) return ctx->fail(SUGG_E_ARG, "plan missing or from another context");
  if (C < 1 || C > 64) return ctx->fail(SUGG_E_ARG, "candidates per kernel must be in [1, 64]");
  if (plan->K == 0) return SUGG_OK;
  if (!counters || !cycles || !cand || !out) return ctx->fail(SUGG_E_ARG, "null argument");
  if ((ref == nullptr) != (flag_out == nullptr) || (flag_out && !(tol >= 0.0)))
    return ctx->fail(SUGG_E_ARG, "ref and flag_out go together, with tol >= 0");
  int rc = check_model_for(ctx, plan);
  if (rc) return rc;
  if (path_lds_bound(plan->dtype == SUGG_F32 ? 4 : 8, ctx->D, plan->E, 1, 1, 1) > kLdsPerWorkgroup)
    return ctx->fail(SUGG_E_BUDGET, "model does not fit in LDS");
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  if (plan->dtype == SUGG_F32)
    return run_judge<float>(ctx, plan, (const float*)counters, (const float*)cycles, cand, C, (float*)out,
                            (const float*)ref, tol, flag_out, accumulate, stream);
  return run_judge<double>(ctx, plan, (const double*)counters, (const double*)cycles, cand, C, (double*)out,
                           (const double*)ref, tol, flag_out, accumulate, stream);
}

int32_t sugg_rank_suggest(sugg_ctx* ctx, int32_t dtype, const void* scores, const int64_t* seg_off, int32_t nseg,
                          int32_t skip_head, int32_t n, double tau, int32_t* idx_out, void* score_out,
                          int32_t* count_out, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (dtype != SUGG_F32 && dtype != SUGG_F64) return ctx->fail(SUGG_E_ARG, "bad dtype %d", dtype);
  if (nseg < 0 || skip_head < 0) return ctx->fail(SUGG_E_ARG, "negative nseg or skip_head");
  if (n < 1 || n > SUGG_MAX_SUGGEST) return ctx->fail(SUGG_E_ARG, "n must be in [1, %d]", SUGG_MAX_SUGGEST);
  if (std::isnan(tau)) return ctx->fail(SUGG_E_ARG, "tau is NaN");
  if (nseg == 0) return SUGG_OK;
  if (!scores || !seg_off || !idx_out || !score_out || !count_out) return ctx->fail(SUGG_E_ARG, "null argument");
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  if (dtype == SUGG_F32)
    return ctx->hip(launch_rank<float>((const float*)scores, seg_off, nseg, skip_head, n, (float)tau, idx_out,
                                       (float*)score_out, count_out, stream), "rank");
  return ctx->hip(launch_rank<double>((const double*)scores, seg_off, nseg, skip_head, n, tau, idx_out,
                                      (double*)score_out, count_out, stream), "rank");
}

int32_t sugg_band_select(sugg_ctx* ctx, int32_t dtype, const void* scores, const int64_t* seg_off, int32_t nseg,
                         int32_t skip_head, const int32_t* top_idx, const int32_t* top_count, int32_t n,
                         double tau, double band, int32_t C, int32_t* cand_out, void* ref_out, int32_t* flag_out,
                         hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (dtype != SUGG_F32 && dtype != SUGG_F64) return ctx->fail(SUGG_E_ARG, "bad dtype %d", dtype);
  if (nseg < 0 || skip_head < 0) return ctx->fail(SUGG_E_ARG, "negative nseg or skip_head");
  if (n < 1 || n > SUGG_MAX_SUGGEST) return ctx->fail(SUGG_E_ARG, "n must be in [1, %d]", SUGG_MAX_SUGGEST);
  if (C < 1 || C > 64) return ctx->fail(SUGG_E_ARG, "band capacity must be in [1, 64]");
  if (!std::isfinite(tau) || !(band >= 0.0) || !std::isfinite(band))
    return ctx->fail(SUGG_E_ARG, "tau must be finite and band finite and >= 0");
  if (nseg == 0) return SUGG_OK;
  if (!scores || !seg_off || !top_idx || !top_count || !cand_out || !ref_out || !flag_out)
    return ctx->fail(SUGG_E_ARG, "null argument");
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  const double lo = tau - band;
  if (dtype == SUGG_F32)
    return ctx->hip(launch_band<float>((const float*)scores, seg_off, nseg, skip_head, top_idx, top_count, n, lo, C,
                                       cand_out, (float*)ref_out, flag_out, stream), "band");
  return ctx->hip(launch_band<double>((const double*)scores, seg_off, nseg, skip_head, top_idx, top_count, n, lo, C,
                                      cand_out, (double*)ref_out, flag_out, stream), "band");
}

int32_t sugg_predict_allpaths(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles,
                              void* table_out, int32_t* idx_out, void* score_out, int32_t* count_out,
                              hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (plan && plan->K > 0 && !table_out) return ctx->fail(SUGG_E_ARG, "table_out is required");
  if (idx_out && (!score_out || !count_out)) return ctx->fail(SUGG_E_ARG, "idx_out needs score_out and count_out");
  if (plan && plan->Bmax > 10) return ctx->fail(SUGG_E_SHAPE, "all-paths composition supports B <= 10");
  int rc = paths_checks(ctx, plan, counters, cycles);
  if (rc || plan->K == 0) return rc;
  const size_t lds = plan->dtype == SUGG_F32 ? paths_lds_bytes<float>(ctx->D, plan->E, plan->Bmax)
                                             : paths_lds_bytes<double>(ctx->D, plan->E, plan->Bmax);
  if (lds > kLdsPerWorkgroup) return ctx->fail(SUGG_E_BUDGET, "model and tables do not fit in LDS");
  if (plan->dtype == SUGG_F32)
    return run_paths<float>(ctx, plan, (const float*)counters, (const float*)cycles, false, (float*)table_out,
                            idx_out, (float*)score_out, count_out, nullptr, nullptr, nullptr, stream);
  return run_paths<double>(ctx, plan, (const double*)counters, (const double*)cycles, false, (double*)table_out,
                           idx_out, (double*)score_out, count_out, nullptr, nullptr, nullptr, stream);
}

int32_t sugg_greedy(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles,
                    int32_t* path_out, int32_t* steps_out, void* gain_out, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (plan && plan->K > 0 && (!path_out || !steps_out || !gain_out))
    return ctx->fail(SUGG_E_ARG, "path_out, steps_out and gain_out are required");
  int rc = paths_checks(ctx, plan, counters, cycles);
  if (rc || plan->K == 0) return rc;
  if (path_lds_bound(plan->dtype == SUGG_F32 ? 4 : 8, ctx->D, plan->E, 1, 1, 1) > kLdsPerWorkgroup)
    return ctx->fail(SUGG_E_BUDGET, "model does not fit in LDS");
  if (plan->dtype == SUGG_F32)
    return run_paths<float>(ctx, plan, (const float*)counters, (const float*)cycles, true, nullptr, nullptr, nullptr,
                            nullptr, path_out, steps_out, (float*)gain_out, stream);
  return run_paths<double>(ctx, plan, (const double*)counters, (const double*)cycles, true, nullptr, nullptr,
                           nullptr, nullptr, path_out, steps_out, (double*)gain_out, stream);
}

int32_t sugg_surrogate_suggest(sugg_ctx* ctx, const sugg_plan* plan, sugg_mlp* mlp, const void* counters,
                               const void* cycles, void* table_out, int32_t* idx_out, void* score_out,
                               int32_t* count_out, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (!plan || plan->ctx != ctx) return ctx->fail(SUGG_E_ARG, "plan missing or from another context");
  if (plan->dtype != SUGG_F32) return ctx->fail(SUGG_E_ARG, "the surrogate runs on FP32 plans");
  if (plan->K == 0) return SUGG_OK;
  if (plan->uni_B < 0) return ctx->fail(SUGG_E_SHAPE, "the surrogate needs one B for all kernels");
  if (!counters || !cycles || !idx_out || !score_out || !count_out) return ctx->fail(SUGG_E_ARG, "null argument");
  if (!mlp) return ctx->fail(SUGG_E_ARG, "null mlp");
  int in = 0, out = 0, bm = 0;
  mlp_dims(mlp, &in, &out, &bm);
  const int B = plan->uni_B, K = plan->K;
  if (in != plan->E || out != (1 << B)) return ctx->fail(SUGG_E_SHAPE, "mlp %d -> %d does not map E=%d to 2^%d", in, out, plan->E, B);
  if (K > bm) return ctx->fail(SUGG_E_SHAPE, "%d kernels above the mlp's batch %d", K, bm);
  int rc = check_model_for(ctx, plan);
  if (rc) return rc;
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  // Tier 1 of each kernel's baseline version, rounded to BF16 into the
  // network's input, then the network with Tier 3 in its output layer
  rc = ctx->hip(launch_standardize_rows_bf16((const float*)counters, (const float*)cycles, plan->d_row_off, K,
                                             plan->E, ctx->mu32, ctx->isg32, mlp_input(mlp), in, ctx->d_status, stream),
                "surrogate: baseline features");
  if (rc) return rc;
  return mlp_infer_rank_input(ctx, mlp, K, 1, ctx->params.n_suggest, (float)ctx->params.tau, (float*)table_out,
                              idx_out, (float*)score_out, count_out, stream);
}

int32_t sugg_serve_query(sugg_ctx* ctx, const sugg_plan* plan, sugg_mlp* mlp, const void* counters,
                         const void* cycles, double tol, double band, int32_t cap, int32_t* idx_out, void* score_out,
                         int32_t* count_out, int32_t* flag_out, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (!plan || plan->ctx != ctx) return ctx->fail(SUGG_E_ARG, "plan missing or from another context");
  if (plan->dtype != SUGG_F32) return ctx->fail(SUGG_E_ARG, "serving runs on FP32 plans");
  if (plan->K == 0) return SUGG_OK;
  if (plan->uni_B < 0) return ctx->fail(SUGG_E_SHAPE, "a serving query has one B for all its kernels");
  if (!counters || !cycles || !idx_out || !score_out || !count_out || !flag_out)
    return ctx->fail(SUGG_E_ARG, "null argument");
  if (!(tol >= 0.0) || !(band >= 0.0) || cap < 1 || cap > 64) return ctx->fail(SUGG_E_ARG, "bad tol, band or cap");
  int in = 0, out = 0, bm = 0;
  if (!mlp) return ctx->fail(SUGG_E_ARG, "null mlp");
  mlp_dims(mlp, &in, &out, &bm);
  const int B = plan->uni_B, K = plan->K, n = ctx->params.n_suggest;
  if (in != plan->E || out != (1 << B)) return ctx->fail(SUGG_E_SHAPE, "mlp %d -> %d does not map E=%d to 2^%d", in, out, plan->E, B);
  if (K > bm) return ctx->fail(SUGG_E_SHAPE, "query of %d kernels above the mlp's batch %d", K, bm);
  int rc = check_model_for(ctx, plan);
  if (rc) return rc;
  if (path_lds_bound(4, ctx->D, plan->E, plan->max_item_rows, plan->max_item_kernels, plan->Bmax) > kLdsPerWorkgroup)
    return ctx->fail(SUGG_E_BUDGET, "model does not fit in LDS");
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  sugg_plan* p = const_cast<sugg_plan*>(plan);
  if (!p->serve || p->serve->cap < cap) {
    delete p->serve;
    p->serve = new (std::nothrow) ServeWs();
    if (!p->serve) return ctx->fail(SUGG_E_BUDGET, "out of host memory");
    ServeWs& w = *p->serve;
    w.cap = cap;
    std::vector<int64_t> seg(K + 1);
    for (int k = 0; k <= K; ++k) seg[k] = (int64_t)k << B;
    hipError_t e = hipMalloc((void**)&w.ys, sizeof(float) * ((size_t)K << B));
    if (e == hipSuccess) e = hipMalloc((void**)&w.sc, sizeof(float) * (size_t)K * n);
    if (e == hipSuccess) e = hipMalloc((void**)&w.br, sizeof(float) * (size_t)K * cap);
    if (e == hipSuccess) e = hipMalloc((void**)&w.bout, sizeof(float) * (size_t)K * cap);
    if (e == hipSuccess) e = hipMalloc((void**)&w.bc, sizeof(int32_t) * (size_t)K * cap);
    if (e == hipSuccess) e = upload(w.seg, seg.data(), sizeof(int64_t) * (K + 1));
    if (e != hipSuccess) {
      delete p->serve;
      p->serve = nullptr;
      return ctx->hip(e, "serving workspace");
    }
  }
  ServeWs& w = *p->serve;
  const float* c = (const float*)counters;
  const float* cy = (const float*)cycles;
  // 1. standardised baseline rows, rounded to BF16 into the network's input;
  // 2. the surrogate's tables and 3. their top n (the output layer ranks in
  // its epilogue where the table is 64 or 128 wide)
  rc = ctx->hip(launch_standardize_rows_bf16(c, cy, p->d_row_off, K, p->E, ctx->mu32, ctx->isg32, mlp_input(mlp),
                                             in, ctx->d_status, stream),
                "serve: baseline features");
  if (!rc) rc = mlp_infer_rank_input(ctx, mlp, K, 1, n, (float)ctx->params.tau, w.ys, idx_out, w.sc, count_out, stream);
  // 4. the threshold band of short lists (overflow flags)
  if (!rc)
    rc = ctx->hip(launch_band<float>(w.ys, w.seg, K, 1, idx_out, count_out, n, ctx->params.tau - band, cap, w.bc,
                                     w.br, flag_out, stream), "serve: band");
  // 5. the judge on both, in one launch (plain values of the listed subsets
  // are the answer's scores)
  if (!rc)
    rc = run_judge<float>(ctx, p, c, cy, idx_out, n, (float*)score_out, w.sc, tol, flag_out, 1, stream, cap, w.bc,
                          w.bout, w.br);
  // 6. Tier 3's contract by the plain values: listed subsets above the
  // threshold, no band subset above it; kept lists sorted by plain value
  if (!rc)
    rc = ctx->hip(launch_confirm(K, n, idx_out, (float*)score_out, count_out, w.bc, w.bout, cap,
                                 (float)ctx->params.tau, flag_out, stream), "serve: confirm");
  // 7. the plain path for the flagged kernels
  if (!rc)
    rc = run_path<float>(ctx, p, c, cy, nullptr, nullptr, idx_out, (float*)score_out, count_out, n, stream, flag_out);
  return rc;
}

int32_t sugg_sync(sugg_ctx* ctx, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  int rc = ctx->hip(hipStreamSynchronize(stream), "stream synchronize");
  if (rc) return rc;
  int32_t st = 0;
  rc = ctx->hip(hipMemcpy(&st, ctx->d_status, sizeof st, hipMemcpyDeviceToHost), "status read");
  if (rc) return rc;
  if (st) {
    rc = ctx->hip(hipMemset(ctx->d_status, 0, sizeof(int32_t)), "status clear");
    if (rc) return rc;
  }
  if (st & kStatusBadCounter) return ctx->fail(SUGG_E_BAD_COUNTER, "a counter or cycle count is <= 0, NaN or Inf");
  if (st & kStatusSingular) return ctx->fail(SUGG_E_SINGULAR, "a regression system is not positive definite");
  if (st & kStatusBadIndex) return ctx->fail(SUGG_E_ARG, "a training row index is outside the training set");
  return SUGG_OK;
}

int32_t sugg_plan_set_launch(sugg_plan* plan, int32_t waves, int32_t unroll, int32_t grid) {
  if (!plan) return SUGG_E_ARG;
  if (waves < 1 || waves > 8 || grid < 0) return SUGG_E_ARG;
  if (unroll != 0 && unroll != 1 && unroll != 2 && unroll != 4 && unroll != -1 && unroll != -2 && unroll != -4)
    return SUGG_E_ARG;
  plan->cfg.waves = waves;
  plan->cfg.unroll = unroll;
  plan->cfg.grid = grid;
  return SUGG_OK;
}

int32_t sugg_plan_set_items(sugg_ctx* ctx, sugg_plan* plan, int32_t rows) {
  if (!ctx) return SUGG_E_ARG;
  if (!plan || plan->ctx != ctx) return ctx->fail(SUGG_E_ARG, "plan missing or from another context");
  if (rows < 16 || rows > 4096) return ctx->fail(SUGG_E_ARG, "item rows %d outside [16, 4096]", rows);
  if (rows == plan->item_rows) return SUGG_OK;
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  return ctx->hip(plan_items(plan, rows), "plan items");
}

int32_t sugg_plan_get_items(const sugg_plan* plan) { return plan ? plan->item_rows : -1; }

int32_t sugg_plan_get_launch(const sugg_plan* plan, int32_t* waves, int32_t* unroll, int32_t* grid) {
  if (!plan || !waves || !unroll || !grid) return SUGG_E_ARG;
  *waves = plan->cfg.waves;
  *unroll = plan->cfg.unroll;
  *grid = plan->cfg.grid;
  return SUGG_OK;
}

int32_t sugg_autotune(sugg_ctx* ctx, sugg_plan* plan, const void* counters, const void* cycles, int32_t reps,
                      float* times_ms, int32_t times_cap, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (!plan || plan->ctx != ctx) return ctx->fail(SUGG_E_ARG, "plan missing or from another context");
  if (plan->K == 0) return SUGG_OK;
  if (!counters || !cycles || reps < 1) return ctx->fail(SUGG_E_ARG, "null input or reps < 1");
  if (times_ms && times_cap < SUGG_TUNE_CANDIDATES)
    return ctx->fail(SUGG_E_ARG, "times_ms holds %d entries, %d needed", times_cap, SUGG_TUNE_CANDIDATES);
  int rc = check_model_for(ctx, plan);
  if (rc) return rc;
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  const size_t ts = plan->dtype == SUGG_F32 ? 4 : 8;
  const int n = ctx->params.n_suggest;
  void *table = nullptr, *idx = nullptr, *score = nullptr, *count = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&table, ts * plan->N);
  if (e == hipSuccess) e = hipMalloc(&idx, sizeof(int32_t) * plan->K * n);
  if (e == hipSuccess) e = hipMalloc(&score, ts * plan->K * n);
  if (e == hipSuccess) e = hipMalloc(&count, sizeof(int32_t) * plan->K);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const PathLaunch keep = plan->cfg;
  const int keep_items = plan->item_rows;
  PathLaunch best = keep;
  int best_items = keep_items;
  float best_ms = 1e30f;
  int ci = 0;
  struct Cand {
    int ci, items;
    PathLaunch cfg;
    float ms;
  };
  std::vector<Cand> cands;   // every candidate that ran
  // mean time of `passes` passes of the current shape (after one warm-up)
  auto time_shape = [&](int passes, float& ms) {
    ms = 0.f;
    for (int rep = -1; rep < passes && e == hipSuccess; ++rep) {   // rep -1 warms up
      if (rep == 0) e = hipEventRecord(e0, stream);
      if (e != hipSuccess) break;
      rc = plan->dtype == SUGG_F32
               ? run_path<float>(ctx, plan, (const float*)counters, (const float*)cycles, nullptr, (float*)table,
                                 (int32_t*)idx, (float*)score, (int32_t*)count, n, stream)
               : run_path<double>(ctx, plan, (const double*)counters, (const double*)cycles, nullptr,
                                  (double*)table, (int32_t*)idx, (double*)score, (int32_t*)count, n, stream);
      if (rc) e = hipErrorUnknown;
    }
    if (e == hipSuccess) e = hipEventRecord(e1, stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    ms /= passes;
  };
  std::vector<std::pair<int, int>> shapes;   // (waves, unroll): fused shapes, then the streaming form
  for (int w : kTuneWaves)
    for (int u : kTuneUnroll) shapes.push_back({w, u});
  for (int u : {-1, -2, -4}) shapes.push_back({4, u});
  for (int ir : kTuneItems)
    for (const auto& wu : shapes) {
      if (e != hipSuccess) break;
      if (plan->item_rows != ir) e = plan_items(plan, ir);
      if (e != hipSuccess) break;
      const int u = wu.second;
      plan->cfg = PathLaunch{wu.first, u, 0};
      const size_t lds = u > 0 ? path_lds_bound(ts, ctx->D, plan->E, plan->max_item_rows, plan->max_item_kernels,
                                                plan->Bmax)
                               : path_chunk_lds(ts, ctx->D, plan->E, plan->chunk_max_rows, plan->chunk_max_nk);
      if (lds > kLdsPerWorkgroup) {   // this item size does not fit
        if (times_ms) times_ms[ci] = -1.f;
        ++ci;
        continue;
      }
      float ms = 0.f;
      time_shape(reps, ms);
      if (times_ms) times_ms[ci] = ms;
      if (e == hipSuccess) cands.push_back({ci, plan->item_rows, plan->cfg, ms});
      ++ci;
    }
  // the split form (equal kernels of at most 64 versions): one more candidate
  if (times_ms) times_ms[ci] = -1.f;
  if (e == hipSuccess && plan->item_rows != keep_items) e = plan_items(plan, keep_items);
  if (e == hipSuccess && plan->split_ok()) {
    plan->cfg = PathLaunch{4, 0, 0};
    float ms = 0.f;
    time_shape(reps, ms);
    if (times_ms) times_ms[ci] = ms;
    if (e == hipSuccess) cands.push_back({ci, plan->item_rows, plan->cfg, ms});
  }
  // the fastest few are timed again, in two rounds of 2 reps passes each (a
  // round visits each finalist once), and the best mean wins: one short
  // sweep over all candidates cannot separate shapes a percent apart
  std::stable_sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
  const size_t n_fin = std::min<size_t>(cands.size(), kTuneFinalists);
  std::vector<float> fin_ms(n_fin, 0.f);
  for (int round = 0; round < 2 && e == hipSuccess; ++round)
    for (size_t f = 0; f < n_fin && e == hipSuccess; ++f) {
      if (plan->item_rows != cands[f].items) e = plan_items(plan, cands[f].items);
      if (e != hipSuccess) break;
      plan->cfg = cands[f].cfg;
      float ms = 0.f;
      time_shape(2 * reps, ms);
      fin_ms[f] += ms / 2;
    }
  for (size_t f = 0; f < n_fin && e == hipSuccess; ++f) {
    if (times_ms) times_ms[cands[f].ci] = fin_ms[f];
    if (fin_ms[f] < best_ms) {
      best_ms = fin_ms[f];
      best = cands[f].cfg;
      best_items = cands[f].items;
    }
  }
  plan->cfg = e == hipSuccess ? best : keep;
  const int want_items = e == hipSuccess ? best_items : keep_items;
  if (plan->item_rows != want_items) {
    const hipError_t e2 = plan_items(plan, want_items);
    if (e == hipSuccess) e = e2;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(table);
  (void)hipFree(idx);
  (void)hipFree(score);
  (void)hipFree(count);
  if (rc) return rc;
  return ctx->hip(e, "autotune");
}

int32_t sugg_capture_begin(sugg_ctx* ctx, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (!stream) return ctx->fail(SUGG_E_ARG, "capture needs a non-default stream");
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  return ctx->hip(hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed), "begin capture");
}

int32_t sugg_capture_end(sugg_ctx* ctx, hipStream_t stream, sugg_graph** out) {
  if (!ctx || !out) return SUGG_E_ARG;
  *out = nullptr;
  sugg_graph* g = new (std::nothrow) sugg_graph();
  if (!g) return ctx->fail(SUGG_E_BUDGET, "out of host memory");
  g->device = ctx->device;
  int rc = ctx->hip(hipStreamEndCapture(stream, &g->graph), "end capture");
  if (!rc) rc = ctx->hip(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0), "instantiate graph");
  if (rc) {
    delete g;
    return rc;
  }
  *out = g;
  return SUGG_OK;
}

int32_t sugg_graph_launch(sugg_ctx* ctx, sugg_graph* graph, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (!graph || graph->device != ctx->device) return ctx->fail(SUGG_E_ARG, "graph missing or from another device");
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  return ctx->hip(hipGraphLaunch(graph->exec, stream), "graph launch");
}

void sugg_graph_destroy(sugg_graph* graph) { delete graph; }

int32_t sugg_model_shape(const sugg_ctx* ctx, int32_t* E, int32_t* D) {
  if (!ctx || !E || !D) return SUGG_E_ARG;
  *E = ctx->has_stats ? ctx->E : 0;
  *D = ctx->has_model ? ctx->D : 0;
  return SUGG_OK;
}

int32_t sugg_model_get(sugg_ctx* ctx, double* mu, double* sigma, double* W, int64_t* counts) {
  if (!ctx) return SUGG_E_ARG;
  if (!ctx->has_stats) return ctx->fail(SUGG_E_STATE, "no model");
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  int rc = ctx->hip(hipDeviceSynchronize(), "synchronize");
  if (rc) return rc;
  if (mu && (rc = ctx->hip(hipMemcpy(mu, ctx->mu64, sizeof(double) * ctx->E, hipMemcpyDeviceToHost), "copy")))
    return rc;
  if (sigma && (rc = ctx->hip(hipMemcpy(sigma, ctx->sig64, sizeof(double) * ctx->E, hipMemcpyDeviceToHost), "copy")))
    return rc;
  if (ctx->has_model) {
    if (W && (rc = ctx->hip(hipMemcpy(W, ctx->W64, sizeof(double) * ctx->D * (ctx->E + 1), hipMemcpyDeviceToHost),
                            "copy")))
      return rc;
    if (counts) std::copy(ctx->counts.begin(), ctx->counts.end(), counts);
  }
  return SUGG_OK;
}

int32_t sugg_model_set(sugg_ctx* ctx, int32_t E, int32_t D, const double* mu, const double* sigma, const double* W,
                       const int64_t* counts) {
  if (!ctx) return SUGG_E_ARG;
  if (E < 1 || E > SUGG_MAX_EVENTS || D < 0 || D > SUGG_MAX_GLOBAL_OPTS) return ctx->fail(SUGG_E_SHAPE, "bad E or D");
  if (!mu || !sigma || (D > 0 && (!W || !counts))) return ctx->fail(SUGG_E_ARG, "null argument");
  for (int j = 0; j < E; ++j)
    if (!(sigma[j] > 0.0) || !std::isfinite(mu[j])) return ctx->fail(SUGG_E_ARG, "bad statistics at column %d", j);
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  int rc = ctx->ensure_model(E, D);
  if (rc) return rc;
  std::vector<double> isg(E), w64(W ? W : mu, W ? W + (size_t)D * (E + 1) : mu);
  const int ldw = w32_ld(E);
  std::vector<float> mu32(E), isg32(E), w32((size_t)D * ldw, 0.0f);
  for (int j = 0; j < E; ++j) {
    isg[j] = 1.0 / sigma[j];
    mu32[j] = (float)mu[j];
    isg32[j] = (float)isg[j];
  }
  for (int o = 0; o < D; ++o)
    for (int j = 0; j <= E; ++j) {
      const double v = W[(size_t)o * (E + 1) + j];
      w32[(size_t)o * ldw + j] = counts[o] > 0 ? (float)v : 0.0f;
    }
  hipError_t e = hipMemcpy(ctx->mu64, mu, sizeof(double) * E, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ctx->sig64, sigma, sizeof(double) * E, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ctx->isg64, isg.data(), sizeof(double) * E, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ctx->mu32, mu32.data(), sizeof(float) * E, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ctx->isg32, isg32.data(), sizeof(float) * E, hipMemcpyHostToDevice);
  if (e == hipSuccess && D > 0) e = hipMemcpy(ctx->W64, W, sizeof(double) * D * (E + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess && D > 0) e = hipMemcpy(ctx->W32, w32.data(), sizeof(float) * D * ldw, hipMemcpyHostToDevice);
  if (e != hipSuccess) return ctx->hip(e, "model upload");
  for (int o = 0; o < D; ++o) ctx->counts[o] = counts[o];
  ctx->has_stats = true;
  ctx->has_model = D > 0;
  return SUGG_OK;
}

}  // extern "C"
