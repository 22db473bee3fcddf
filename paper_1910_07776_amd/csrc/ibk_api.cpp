// Host side of the instance-based (IBK) scoring path: the sample database of
// a fit, per-plan query lists and the launches of a prediction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "ibk.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "sugg.h"

using namespace sugg;

void ibk_model_free(IbkModel*& m) {
  if (!m) return;
  dfree(m->Z); dfree(m->Z64); dfree(m->srow); dfree(m->norm); dfree(m->y); dfree(m->d_off);
  dfree(m->mu64); dfree(m->sig64); dfree(m->mu_t); dfree(m->isg_t);
  delete m;
  m = nullptr;
}

void ibk_plan_free(IbkPlan*& p) {
  if (!p) return;
  dfree(p->zq);
  dfree(p->edges);
  dfree(p->part_d);
  dfree(p->part_i);
  dfree(p->exact_q);
  dfree(p->exact_n);
  for (auto& q : p->q) {
    dfree(q.src); dfree(q.dst); dfree(q.tiles);
  }
  delete p;
  p = nullptr;
}

namespace {

int ibk_epad(int E) {
  for (int e : {32, 64, 128, 256})
    if (E <= e) return e;
  return -1;
}

template <typename V>
hipError_t upload_vec(V*& dst, const std::vector<V>& src) {
  const size_t bytes = std::max<size_t>(sizeof(V) * src.size(), 16);
  hipError_t e = hipMalloc((void**)&dst, bytes);
  if (e == hipSuccess && !src.empty()) e = hipMemcpy(dst, src.data(), sizeof(V) * src.size(), hipMemcpyHostToDevice);
  return e;
}

template <typename T>
int fit_t(sugg_ctx* ctx, sugg_plan* p, const T* c, const T* cyc, int k, hipStream_t s) {
  IbkModel* m = new (std::nothrow) IbkModel();
  if (!m) return ctx->fail(SUGG_E_BUDGET, "out of host memory");
  m->E = p->E;
  m->Epad = ibk_epad(p->E);
  m->D = p->D;
  m->k = k;
  m->Ntr = p->N;
  const int E = p->E;
  // samples of each global id: kernels in batch order, versions S ascending
  std::vector<std::vector<int32_t>> bef(p->D), aft(p->D);
  for (int kk = 0; kk < p->K; ++kk) {
    const int B = p->nopts[kk];
    for (int b = 0; b < B; ++b) {
      const int o = p->opt_ids[p->opt_off[kk] + b];
      for (int S = 0; S < (1 << B); ++S)
        if (!((S >> b) & 1)) {
          bef[o].push_back((int32_t)(p->row_off[kk] + S));
          aft[o].push_back((int32_t)(p->row_off[kk] + (S | (1 << b))));
        }
    }
  }
  m->off.assign(p->D + 1, 0);
  for (int o = 0; o < p->D; ++o) m->off[o + 1] = m->off[o] + (int64_t)bef[o].size();
  m->Ns = m->off[p->D];
  std::vector<int32_t> hb, ha;
  hb.reserve(m->Ns);
  ha.reserve(m->Ns);
  for (int o = 0; o < p->D; ++o) {
    hb.insert(hb.end(), bef[o].begin(), bef[o].end());
    ha.insert(ha.end(), aft[o].begin(), aft[o].end());
  }
  int32_t* d_after = nullptr;
  double* partial = nullptr;
  float* zrows = nullptr;
  const int chunks = colstats_chunks(std::max<int64_t>(p->N, 1));
  const int64_t ns1 = std::max<int64_t>(m->Ns, 1);
  hipError_t e = hipMalloc((void**)&m->mu64, sizeof(double) * E);
  if (e == hipSuccess) e = hipMalloc((void**)&m->sig64, sizeof(double) * E);
  if (e == hipSuccess) e = hipMalloc((void**)&m->mu_t, sizeof(T) * E);
  if (e == hipSuccess) e = hipMalloc((void**)&m->isg_t, sizeof(T) * E);
  if (e == hipSuccess) e = hipMalloc((void**)&partial, sizeof(double) * 2 * E * chunks);
  if (e == hipSuccess) e = hipMalloc((void**)&zrows, sizeof(float) * (size_t)p->N * m->Epad);
  if (e == hipSuccess) e = hipMalloc((void**)&m->Z, sizeof(float) * (size_t)ns1 * m->Epad);
  if (e == hipSuccess) e = hipMalloc((void**)&m->norm, sizeof(float) * (size_t)ns1);
  if (e == hipSuccess) e = upload_vec(m->srow, hb);
  if (e == hipSuccess) e = hipMalloc((void**)&m->Z64, sizeof(double) * (size_t)std::max<int64_t>(p->N, 1) * E);
  if (e == hipSuccess) e = upload_vec(d_after, ha);
  if (e == hipSuccess) e = hipMalloc((void**)&m->y, sizeof(double) * ns1);
  if (e == hipSuccess) e = upload_vec(m->d_off, m->off);
  // Tier 1 statistics, standardised rows, sample vectors in database order,
  // their norms, labels
  if (e == hipSuccess)
    e = launch_colstats<T>(c, cyc, p->N, E, partial, chunks, m->mu64, m->sig64, (T*)m->mu_t, (T*)m->isg_t,
                           ctx->d_status, s);
  if (e == hipSuccess) e = launch_ibk_z<T>(c, cyc, p->N, E, m->Epad, m->mu64, m->sig64, zrows, ctx->d_status, s);
  if (e == hipSuccess) e = launch_ibk_gather(zrows, m->srow, m->Ns, m->Epad, m->Z, s);
  if (e == hipSuccess) e = launch_ibk_norm(m->Z, m->Ns, m->Epad, m->norm, s);
  if (e == hipSuccess) e = launch_ibk_labels<T>(cyc, m->srow, d_after, m->Ns, m->y, s);
  // FP64 standardised training rows for exact distances
  double* lcyc = nullptr;
  if (e == hipSuccess) e = hipMalloc((void**)&lcyc, sizeof(double) * (size_t)std::max<int64_t>(p->N, 1));
  if (e == hipSuccess) e = launch_zfeat64<T>(c, cyc, p->N, E, m->mu64, m->sig64, m->Z64, lcyc, s);
  // the largest FP32 rounding of each column of the stored vectors
  uint32_t* dz = nullptr;
  if (e == hipSuccess) e = hipMalloc((void**)&dz, sizeof(uint32_t) * E);
  if (e == hipSuccess) e = hipMemsetAsync(dz, 0, sizeof(uint32_t) * E, s);
  if (e == hipSuccess) e = launch_ibk_dz(zrows, m->Epad, m->Z64, p->N, E, dz, s);
  std::vector<uint32_t> hdz(E, 0);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemcpy(hdz.data(), dz, sizeof(uint32_t) * E, hipMemcpyDeviceToHost);
  if (e == hipSuccess) {
    double acc = 0.0;
    for (int j = 0; j < E; ++j) {
      float f;
      std::memcpy(&f, &hdz[j], sizeof f);
      acc += (double)f * (double)f;
    }
    m->dt_norm = std::sqrt(acc) * (1.0 + 1e-12);
  }
  dfree(dz);
  dfree(lcyc);
  dfree(d_after);
  dfree(partial);
  dfree(zrows);
  if (e != hipSuccess) {
    ibk_model_free(m);
    return ctx->hip(e, "IBK fit");
  }
  ibk_model_free(ctx->ibk);
  ctx->ibk = m;
  return SUGG_OK;
}

// Query lists of a plan for one mode (see IbkQueries), tiles ordered by the
// size of their optimisation's database (largest first).
int build_queries(sugg_ctx* ctx, sugg_plan* p, const IbkModel* m, int mode) {
  IbkQueries& q = p->ibk->q[mode];
  if (q.built) return SUGG_OK;
  const int D = p->D;
  std::vector<std::vector<int32_t>> src(D);
  std::vector<std::vector<int64_t>> dst(D);
  for (int kk = 0; kk < p->K; ++kk) {
    const int B = p->nopts[kk];
    const int64_t r0 = p->row_off[kk];
    const int32_t* ids = p->opt_ids.data() + p->opt_off[kk];
    if (mode == 0) {
      for (int S = 1; S < (1 << B); ++S) {
        int b = 31 - __builtin_clz((unsigned)S);
        src[ids[b]].push_back((int32_t)(r0 + S - (1 << b)));
        dst[ids[b]].push_back(r0 + S);
      }
    } else {
      for (int S = 0; S < (1 << B); ++S)
        for (int b = 0; b < B; ++b)
          if (!((S >> b) & 1)) {
            src[ids[b]].push_back((int32_t)(r0 + S));
            dst[ids[b]].push_back((r0 + S) * p->Bmax + b);
          }
    }
  }
  std::vector<int32_t> hs;
  std::vector<int64_t> hd;
  std::vector<int32_t> tiles;
  q.per_opt.assign(D, 0);
  std::vector<int> order(D);
  for (int o = 0; o < D; ++o) order[o] = o;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return m->off[x + 1] - m->off[x] > m->off[y + 1] - m->off[y];
  });
  for (int o : order) {
    const int64_t base = (int64_t)hs.size();
    q.per_opt[o] = (int64_t)src[o].size();
    hs.insert(hs.end(), src[o].begin(), src[o].end());
    hd.insert(hd.end(), dst[o].begin(), dst[o].end());
    for (int64_t t = 0; t < (int64_t)src[o].size(); t += kIbkQueries) {
      tiles.push_back(o);
      tiles.push_back((int32_t)(base + t));
      tiles.push_back((int32_t)std::min<int64_t>(kIbkQueries, (int64_t)src[o].size() - t));
      tiles.push_back(0);
    }
  }
  if ((int64_t)hs.size() >= ((int64_t)1 << 31)) return ctx->fail(SUGG_E_BUDGET, "too many IBK queries in one plan");
  q.n = (int64_t)hs.size();
  q.n_tiles = (int)(tiles.size() / 4);
  hipError_t e = upload_vec(q.src, hs);
  if (e == hipSuccess) e = upload_vec(q.dst, hd);
  if (e == hipSuccess) e = upload_vec(q.tiles, tiles);
  if (e != hipSuccess) {
    dfree(q.src); dfree(q.dst); dfree(q.tiles);
    return ctx->hip(e, "IBK query lists");
  }
  q.built = true;
  return SUGG_OK;
}

int check_ibk_for(sugg_ctx* ctx, const sugg_plan* p) {
  const IbkModel* m = ctx->ibk;
  if (!m) return ctx->fail(SUGG_E_STATE, "no IBK model (call sugg_ibk_fit)");
  if (m->E != p->E) return ctx->fail(SUGG_E_SHAPE, "plan E=%d, IBK model E=%d", p->E, m->E);
  for (size_t i = 0; i < p->opt_ids.size(); ++i) {
    const int o = p->opt_ids[i];
    if (o >= m->D || m->off[o + 1] == m->off[o])
      return ctx->fail(SUGG_E_UNTRAINED_OPT, "optimisation %d has no IBK samples", o);
  }
  return SUGG_OK;
}

template <typename T>
int score_t(sugg_ctx* ctx, sugg_plan* p, const T* c, const T* cyc, T* grid, T* table, int32_t* idx, T* score,
            int32_t* count, hipStream_t s) {
  const IbkModel* m = ctx->ibk;
  if (!p->ibk) {
    p->ibk = new (std::nothrow) IbkPlan();
    if (!p->ibk) return ctx->fail(SUGG_E_BUDGET, "out of host memory");
  }
  IbkPlan* w = p->ibk;
  if (w->Epad != m->Epad) {
    dfree(w->zq);
    w->Epad = m->Epad;
  }
  hipError_t e = hipSuccess;
  if (!w->zq) e = hipMalloc((void**)&w->zq, sizeof(float) * std::max<int64_t>(p->N, 1) * w->Epad);
  if (e == hipSuccess && !w->edges) e = hipMalloc(&w->edges, sizeof(T) * std::max<int64_t>(p->N, 1));
  if (e != hipSuccess) return ctx->hip(e, "IBK workspace");
  const int mode = grid ? 1 : 0;
  int rc = build_queries(ctx, p, m, mode);
  if (rc) return rc;
  const IbkQueries& q = w->q[mode];
  e = launch_ibk_z<T>(c, cyc, p->N, p->E, w->Epad, m->mu64, m->sig64, w->zq, ctx->d_status, s);
  if (e == hipSuccess && grid) e = launch_ibk_nan<T>(grid, p->N * p->Bmax, s);
  IbkKnnArgs a;
  a.zq = w->zq;
  a.Z = m->Z;
  a.norm = m->norm;
  a.y = m->y;
  a.off = m->d_off;
  a.q_src = q.src;
  a.q_dst = q.dst;
  a.tiles = q.tiles;
  a.Epad = w->Epad;
  a.k = m->k;
  a.kt = ibk_kt(m->k);
  a.counters = c;
  a.cycles = cyc;
  a.E = p->E;
  a.mu64 = m->mu64;
  a.sig64 = m->sig64;
  a.Z64 = m->Z64;
  a.srow = m->srow;
  a.dt_norm = m->dt_norm;
  a.out = grid ? (void*)grid : w->edges;
  a.n_queries = q.n;
  a.n_tiles = q.n_tiles;
  // enough workgroups for one round of resident ones: each query tile's
  // samples are split into shares whose neighbour lists are merged after
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus <= 0)
    cus = 256;
  a.split = ibk_split(w->Epad, m->k, q.n_tiles, cus);
  const int64_t need = std::max<int64_t>(q.n, 1) * a.split * kIbkList;
  if (w->part_cap < need) {
    dfree(w->part_d);
    dfree(w->part_i);
    w->part_cap = 0;
    if (e == hipSuccess) e = hipMalloc((void**)&w->part_d, sizeof(float) * need);
    if (e == hipSuccess) e = hipMalloc((void**)&w->part_i, sizeof(int32_t) * need);
    if (e == hipSuccess) w->part_cap = need;
  }
  if (w->exact_cap < std::max<int64_t>(q.n, 1)) {
    dfree(w->exact_q);
    dfree(w->exact_n);
    w->exact_cap = 0;
    if (e == hipSuccess) e = hipMalloc((void**)&w->exact_q, sizeof(int32_t) * std::max<int64_t>(q.n, 1));
    if (e == hipSuccess) e = hipMalloc((void**)&w->exact_n, sizeof(int32_t));
    if (e == hipSuccess) e = hipMemset(w->exact_n, 0, sizeof(int32_t));
    if (e == hipSuccess) w->exact_cap = std::max<int64_t>(q.n, 1);
  }
  a.part_d = w->part_d;
  a.part_i = w->part_i;
  a.exact_q = w->exact_q;
  a.exact_n = w->exact_n;
  w->exact_mode = mode;
  if (e == hipSuccess) e = launch_ibk_knn<T>(a, q.n_tiles, s);
  if (e == hipSuccess)
    e = launch_ibk_compose<T, T>(grid ? nullptr : (const T*)w->edges, grid, p->Bmax, p->d_row_off, p->d_nopts, p->K,
                              p->Bmax, table, idx, score, count, ctx->params.n_suggest, (T)ctx->params.tau, s);
  return ctx->hip(e, "IBK scoring");
}

int common_checks(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles) {
  if (!plan || plan->ctx != ctx) return ctx->fail(SUGG_E_ARG, "plan missing or from another context");
  if (plan->N > 0 && (!counters || !cycles)) return ctx->fail(SUGG_E_ARG, "null counters or cycles");
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  return SUGG_OK;
}

}  // namespace

extern "C" {

int32_t sugg_ibk_fit(sugg_ctx* ctx, const sugg_plan* train, const void* counters, const void* cycles, int32_t k,
                     hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  int rc = common_checks(ctx, train, counters, cycles);
  if (rc) return rc;
  if (k < 1 || k > kIbkMaxK) return ctx->fail(SUGG_E_ARG, "k must be in [1, %d]", kIbkMaxK);
  if (ibk_epad(train->E) < 0) return ctx->fail(SUGG_E_SHAPE, "IBK supports at most 256 events (E=%d)", train->E);
  if (train->N == 0) return ctx->fail(SUGG_E_SHAPE, "IBK needs at least one training row");
  if (train->N >= ((int64_t)1 << 31)) return ctx->fail(SUGG_E_BUDGET, "too many training rows for IBK");
  sugg_plan* p = const_cast<sugg_plan*>(train);
  if (p->dtype == SUGG_F32) return fit_t<float>(ctx, p, (const float*)counters, (const float*)cycles, k, stream);
  return fit_t<double>(ctx, p, (const double*)counters, (const double*)cycles, k, stream);
}

int32_t sugg_ibk_counts(sugg_ctx* ctx, int64_t* counts, int32_t D) {
  if (!ctx || !counts) return SUGG_E_ARG;
  if (!ctx->ibk) return ctx->fail(SUGG_E_STATE, "no IBK model");
  for (int o = 0; o < D; ++o) counts[o] = o < ctx->ibk->D ? ctx->ibk->off[o + 1] - ctx->ibk->off[o] : 0;
  return SUGG_OK;
}

int32_t sugg_ibk_exact_count(sugg_ctx* ctx, const sugg_plan* plan, int64_t* n) {
  if (!ctx || !n) return SUGG_E_ARG;
  if (!plan || plan->ctx != ctx) return ctx->fail(SUGG_E_ARG, "plan missing or from another context");
  *n = 0;
  if (!plan->ibk || !plan->ibk->exact_n) return SUGG_OK;
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  int32_t v = 0;
  const int rc = ctx->hip(hipDeviceSynchronize(), "synchronize");
  if (rc) return rc;
  const hipError_t e = hipMemcpy(&v, plan->ibk->exact_n, sizeof(int32_t), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return ctx->hip(e, "copy");
  *n = v;
  return SUGG_OK;
}

int32_t sugg_ibk_predict(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles,
                         void* grid_out, void* table_out, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  int rc = common_checks(ctx, plan, counters, cycles);
  if (rc) return rc;
  if (plan->K > 0 && !table_out) return ctx->fail(SUGG_E_ARG, "table_out is required");
  rc = check_ibk_for(ctx, plan);
  if (rc || plan->K == 0) return rc;
  sugg_plan* p = const_cast<sugg_plan*>(plan);
  if (p->dtype == SUGG_F32)
    return score_t<float>(ctx, p, (const float*)counters, (const float*)cycles, (float*)grid_out, (float*)table_out,
                          nullptr, nullptr, nullptr, stream);
  return score_t<double>(ctx, p, (const double*)counters, (const double*)cycles, (double*)grid_out,
                         (double*)table_out, nullptr, nullptr, nullptr, stream);
}

int32_t sugg_ibk_suggest(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles,
                         void* table_out, int32_t* idx_out, void* score_out, int32_t* count_out, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  int rc = common_checks(ctx, plan, counters, cycles);
  if (rc) return rc;
  if (plan->K > 0 && (!idx_out || !score_out || !count_out))
    return ctx->fail(SUGG_E_ARG, "idx_out, score_out and count_out are required");
  rc = check_ibk_for(ctx, plan);
  if (rc || plan->K == 0) return rc;
  sugg_plan* p = const_cast<sugg_plan*>(plan);
  if (p->dtype == SUGG_F32)
    return score_t<float>(ctx, p, (const float*)counters, (const float*)cycles, nullptr, (float*)table_out, idx_out,
                          (float*)score_out, count_out, stream);
  return score_t<double>(ctx, p, (const double*)counters, (const double*)cycles, nullptr, (double*)table_out,
                         idx_out, (double*)score_out, count_out, stream);
}

}  // extern "C"
