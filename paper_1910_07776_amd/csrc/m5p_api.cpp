// Host side of the model-tree (M5P) scoring path: the fit (FP64 features on
// the GPU, tree induction on the host, upload), the tree export and the
// launches of a prediction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "ibk.hpp"
#include "kernels.hpp"
#include "m5p.hpp"
#include "plan.hpp"
#include "sugg.h"

using namespace sugg;

void m5p_model_free(M5pModel*& m) {
  if (!m) return;
  dfree(m->d_root); dfree(m->blk64); dfree(m->lw64); dfree(m->lb64); dfree(m->mu64); dfree(m->isg64);
  delete m;
  m = nullptr;
}

void m5p_plan_free(M5pPlan*& p) {
  if (!p) return;
  dfree(p->tiles);
  dfree(p->edges);
  delete p;
  p = nullptr;
}

namespace {

constexpr int64_t kM5pMaxCases = (int64_t)1 << 20;    // training pairs per optimisation
constexpr int64_t kM5pHostBudget = (int64_t)16 << 30;  // bytes of host memory for the induction
constexpr int64_t kM5pMaxFeatureBytes = (int64_t)8 << 30;   // FP64 training features copied to the host

int m5p_ldl(int E) { return E <= 64 ? 64 : E <= 128 ? 128 : 256; }

template <typename V>
hipError_t put(V*& dst, const std::vector<V>& src) {
  hipError_t e = hipMalloc((void**)&dst, std::max<size_t>(sizeof(V) * src.size(), 16));
  if (e == hipSuccess && !src.empty()) e = hipMemcpy(dst, src.data(), sizeof(V) * src.size(), hipMemcpyHostToDevice);
  return e;
}

// Trees of every global id with training pairs, induced in parallel.
int induce_all(sugg_ctx* ctx, const sugg_plan* p, const std::vector<double>& z, const std::vector<double>& lcyc,
               M5pModel* m) {
  const int D = p->D;
  // cases of each id: kernel by kernel, then bit, then before-version S
  std::vector<std::vector<int32_t>> before(D);
  std::vector<std::vector<double>> label(D);
  for (int kk = 0; kk < p->K; ++kk) {
    const int B = p->nopts[kk];
    const int64_t r0 = p->row_off[kk];
    for (int b = 0; b < B; ++b) {
      const int o = p->opt_ids[p->opt_off[kk] + b];
      for (int S = 0; S < (1 << B); ++S)
        if (!((S >> b) & 1)) {
          before[o].push_back((int32_t)(r0 + S));
          label[o].push_back(lcyc[r0 + S] - lcyc[r0 + (S | (1 << b))]);
        }
    }
  }
  for (int o = 0; o < D; ++o)
    if ((int64_t)before[o].size() > kM5pMaxCases)
      return ctx->fail(SUGG_E_BUDGET, "optimisation %d has %lld training pairs (M5P limit %lld)", o,
                       (long long)before[o].size(), (long long)kM5pMaxCases);
  m->trees.assign(D, M5pHostTree());
  std::vector<int> work;
  for (int o = 0; o < D; ++o)
    if (!before[o].empty()) work.push_back(o);
  std::atomic<int> next{0};
  std::atomic<bool> oom{false};
  auto worker = [&]() {
    for (int i = next++; i < (int)work.size(); i = next++) {
      const int o = work[i];
      try {
        m->trees[o] = m5p_induce(z.data(), p->E, before[o].data(), label[o].data(), (int64_t)before[o].size(), p->E,
                                 m->prm);
      } catch (const std::bad_alloc&) {
        oom = true;
      }
    }
  };
  // each tree holds every feature's sorted case order and values (12 B per
  // case and feature): as many trees at once as the host budget allows
  int64_t biggest = 1;
  for (int o : work) biggest = std::max<int64_t>(biggest, (int64_t)before[o].size());
  const int64_t per_tree = biggest * p->E * 12 + ((int64_t)64 << 20);
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int by_mem = (int)std::max<int64_t>(1, kM5pHostBudget / per_tree);
  const int nt = (int)std::min<size_t>(std::min<unsigned>(std::min<unsigned>(hw, 16u), (unsigned)by_mem), work.size());
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(worker);
  worker();
  for (auto& t : pool) t.join();
  if (oom) return ctx->fail(SUGG_E_BUDGET, "out of host memory inducing M5P trees");
  return SUGG_OK;
}

// Leaf ordinal stored in a threshold slot's bits (read back the same way).
void put_leaf(double& slot, int32_t id) {
  const int64_t v = id;
  std::memcpy(&slot, &v, sizeof v);
}

// Pack one tree into three-level blocks (see M5pBlock), breadth first from
// the root; leaf ordinals offset by leaf_base, block indices by the blocks
// already present.  Returns the root block; *chain receives the longest run
// of blocks a walk loads.
int pack_tree(const M5pHostTree& t, int leaf_base, std::vector<M5pBlock<double>>& b64, int* chain) {
  struct Todo {
    int node, block, level;
  };
  auto fresh = [&]() {
    M5pBlock<double> d{};
    for (int p = 0; p < 8; ++p) {
      d.feat[p] = -1;
      d.exit[p] = -1;
      put_leaf(d.thr[p], leaf_base);   // unreachable slots name a valid leaf
    }
    b64.push_back(d);
    return (int)b64.size() - 1;
  };
  std::vector<Todo> todo{{0, fresh(), 1}};
  *chain = 1;
  for (size_t q = 0; q < todo.size(); ++q) {
    const Todo td = todo[q];
    *chain = std::max(*chain, td.level);
    int pos[7];
    std::fill(pos, pos + 7, -1);
    pos[0] = td.node;
    for (int p = 0; p < 7; ++p) {
      const int m = pos[p];
      if (m < 0) continue;
      M5pBlock<double>& d = b64[td.block];
      if (t.feat[m] < 0) {
        put_leaf(d.thr[p], leaf_base + t.leaf[m]);
        continue;
      }
      d.feat[p] = (int16_t)t.feat[m];
      d.thr[p] = t.thr[m];
      if (p < 3) {
        pos[2 * p + 1] = t.left[m];
        pos[2 * p + 2] = t.right[m];
        continue;
      }
      const int kids[2] = {t.left[m], t.right[m]};
      for (int side = 0; side < 2; ++side) {
        const int c = kids[side];
        int ref;
        if (t.feat[c] < 0) {
          ref = -1 - (leaf_base + t.leaf[c]);
        } else {
          ref = fresh();
          todo.push_back({c, ref, td.level + 1});
        }
        b64[td.block].exit[2 * (p - 3) + side] = ref;
      }
    }
  }
  return todo[0].block;
}

// Concatenate the trees into the device arrays.
int upload_model(sugg_ctx* ctx, M5pModel* m) {
  const int E = m->E, ldl = m->ldl;
  std::vector<M5pBlock<double>> b64;
  std::vector<double> lw64, lb64;
  m->root.assign(m->D, -1);
  m->max_blocks = 1;
  int leaf_base = 0;
  for (int o = 0; o < m->D; ++o) {
    const M5pHostTree& t = m->trees[o];
    if (t.feat.empty()) continue;
    int chain = 1;
    m->root[o] = pack_tree(t, leaf_base, b64, &chain);
    m->max_blocks = std::max(m->max_blocks, chain);
    for (int l = 0; l < t.leaves; ++l) {
      const double* w = t.lw.data() + (size_t)l * (E + 1);
      for (int j = 0; j < ldl; ++j) {
        const double v = j < E ? w[j] : 0.0;
        lw64.push_back(v);
      }
      lb64.push_back(w[E]);
    }
    leaf_base += t.leaves;
  }
  hipError_t e = put(m->d_root, m->root);
  if (e == hipSuccess) e = put(m->blk64, b64);
  if (e == hipSuccess) e = put(m->lw64, lw64);
  if (e == hipSuccess) e = put(m->lb64, lb64);
  return ctx->hip(e, "M5P model upload");
}

template <typename T>
int fit_t(sugg_ctx* ctx, sugg_plan* p, const T* c, const T* cyc, const M5pParams& prm, hipStream_t s) {
  const int E = p->E;
  const int64_t N = p->N;
  double *partial = nullptr, *mu64 = nullptr, *sig64 = nullptr, *z64 = nullptr, *lcyc64 = nullptr;
  T *mu_t = nullptr, *isg_t = nullptr;
  const int chunks = colstats_chunks(std::max<int64_t>(N, 1));
  hipError_t e = hipMalloc((void**)&partial, sizeof(double) * 2 * E * chunks);
  if (e == hipSuccess) e = hipMalloc((void**)&mu64, sizeof(double) * E);
  if (e == hipSuccess) e = hipMalloc((void**)&sig64, sizeof(double) * E);
  if (e == hipSuccess) e = hipMalloc((void**)&mu_t, sizeof(T) * E);
  if (e == hipSuccess) e = hipMalloc((void**)&isg_t, sizeof(T) * E);
  if (e == hipSuccess) e = hipMalloc((void**)&z64, sizeof(double) * (size_t)N * E);
  if (e == hipSuccess) e = hipMalloc((void**)&lcyc64, sizeof(double) * (size_t)N);
  // Tier 1 on the GPU in FP64: column statistics, standardised features, ln cycles
  if (e == hipSuccess)
    e = launch_colstats<T>(c, cyc, N, E, partial, chunks, mu64, sig64, mu_t, isg_t, ctx->d_status, s);
  if (e == hipSuccess) e = launch_zfeat64<T>(c, cyc, N, E, mu64, sig64, z64, lcyc64, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  std::vector<double> hz, hl, hmu(E), hsig(E);
  try {
    hz.resize((size_t)N * E);
    hl.resize((size_t)N);
  } catch (const std::bad_alloc&) {
    e = hipErrorOutOfMemory;
  }
  if (e == hipSuccess) e = hipMemcpy(hz.data(), z64, sizeof(double) * hz.size(), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(hl.data(), lcyc64, sizeof(double) * hl.size(), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(hmu.data(), mu64, sizeof(double) * E, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(hsig.data(), sig64, sizeof(double) * E, hipMemcpyDeviceToHost);
  dfree(partial); dfree(mu64); dfree(sig64); dfree(mu_t); dfree(isg_t); dfree(z64); dfree(lcyc64);
  if (e != hipSuccess) return ctx->hip(e, "M5P features");
  for (double v : hl)
    if (!std::isfinite(v)) return ctx->fail(SUGG_E_BAD_COUNTER, "a training cycle count is <= 0, NaN or Inf");
  for (double v : hz)
    if (!std::isfinite(v)) return ctx->fail(SUGG_E_BAD_COUNTER, "a training counter is <= 0, NaN or Inf");
  M5pModel* m = new (std::nothrow) M5pModel();
  if (!m) return ctx->fail(SUGG_E_BUDGET, "out of host memory");
  m->E = E;
  m->D = p->D;
  m->ldl = m5p_ldl(E);
  m->prm = prm;
  int rc = induce_all(ctx, p, hz, hl, m);
  if (!rc) rc = upload_model(ctx, m);
  if (!rc) {
    std::vector<double> isg64(E);
    for (int j = 0; j < E; ++j) isg64[j] = 1.0 / hsig[j];
    e = put(m->mu64, hmu);
    if (e == hipSuccess) e = put(m->isg64, isg64);
    rc = ctx->hip(e, "M5P statistics upload");
  }
  if (rc) {
    m5p_model_free(m);
    return rc;
  }
  m5p_model_free(ctx->m5p);
  ctx->m5p = m;
  return SUGG_OK;
}

int check_m5p_for(sugg_ctx* ctx, const sugg_plan* p) {
  const M5pModel* m = ctx->m5p;
  if (!m) return ctx->fail(SUGG_E_STATE, "no M5P model (call sugg_m5p_fit)");
  if (m->E != p->E) return ctx->fail(SUGG_E_SHAPE, "plan E=%d, M5P model E=%d", p->E, m->E);
  for (size_t i = 0; i < p->opt_ids.size(); ++i) {
    const int o = p->opt_ids[i];
    if (o >= m->D || m->root[o] < 0) return ctx->fail(SUGG_E_UNTRAINED_OPT, "optimisation %d has no M5P tree", o);
  }
  return SUGG_OK;
}

template <typename T>
int score_t(sugg_ctx* ctx, sugg_plan* p, const T* c, const T* cyc, T* grid, T* table, int32_t* idx, T* score,
            int32_t* count, hipStream_t s) {
  const M5pModel* m = ctx->m5p;
  if (!p->m5p) {
    M5pPlan* w = new (std::nothrow) M5pPlan();
    if (!w) return ctx->fail(SUGG_E_BUDGET, "out of host memory");
    std::vector<int32_t> tiles;
    for (int kk = 0; kk < p->K; ++kk)
      for (int S0 = 0; S0 < (1 << p->nopts[kk]); S0 += kM5pRows) {
        tiles.push_back(kk);
        tiles.push_back(S0);
      }
    if (tiles.size() / 2 >= (size_t)1 << 31) {
      delete w;
      return ctx->fail(SUGG_E_BUDGET, "too many row tiles for M5P");
    }
    w->n_tiles = (int)(tiles.size() / 2);
    hipError_t e = put(w->tiles, tiles);
    if (e == hipSuccess) e = hipMalloc(&w->edges, sizeof(double) * std::max<int64_t>(p->N, 1));
    if (e != hipSuccess) {
      m5p_plan_free(w);
      return ctx->hip(e, "M5P plan workspace");
    }
    p->m5p = w;
  }
  M5pArgs<T> a;
  a.counters = c;
  a.cycles = cyc;
  a.row_off = p->d_row_off;
  a.nopts = p->d_nopts;
  a.opt_off = p->d_opt_off;
  a.opt_ids = p->d_opt_ids;
  a.tiles = p->m5p->tiles;
  a.mu = m->mu64;
  a.isg = m->isg64;
  a.root = m->d_root;
  a.blocks = m->blk64;
  a.lw = m->lw64;
  a.lb = m->lb64;
  a.ldl = m->ldl;
  a.max_blocks = m->max_blocks;
  a.E = p->E;
  a.Bmax = p->Bmax;
  a.grid = grid;
  a.edges = (double*)p->m5p->edges;
  a.status = ctx->d_status;
  hipError_t e = hipSuccess;
  if (!grid && p->Bmax <= kM5pSmallB) {
    e = launch_m5p_small<T>(a, p->K, table, idx, score, count, ctx->params.n_suggest, ctx->params.tau, s);
    return ctx->hip(e, "M5P scoring");
  }
  if (grid) e = launch_ibk_nan<T>(grid, p->N * p->Bmax, s);
  if (e == hipSuccess) e = launch_m5p<T>(a, p->m5p->n_tiles, s);
  if (e == hipSuccess)
    e = launch_ibk_compose<double, T>(a.edges, grid, p->Bmax, p->d_row_off, p->d_nopts, p->K,
                                      p->Bmax, table, idx, score, count, ctx->params.n_suggest, ctx->params.tau, s);
  return ctx->hip(e, "M5P scoring");
}

int common_checks(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles) {
  if (!plan || plan->ctx != ctx) return ctx->fail(SUGG_E_ARG, "plan missing or from another context");
  if (plan->N > 0 && (!counters || !cycles)) return ctx->fail(SUGG_E_ARG, "null counters or cycles");
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  return SUGG_OK;
}

}  // namespace

extern "C" {

int32_t sugg_m5p_fit(sugg_ctx* ctx, const sugg_plan* train, const void* counters, const void* cycles,
                     int32_t min_leaf, double smooth_k, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  int rc = common_checks(ctx, train, counters, cycles);
  if (rc) return rc;
  if (min_leaf < 1) return ctx->fail(SUGG_E_ARG, "min_leaf must be at least 1");
  if (!(smooth_k >= 0.0) || !std::isfinite(smooth_k)) return ctx->fail(SUGG_E_ARG, "smooth_k must be finite and >= 0");
  if (train->E > 256) return ctx->fail(SUGG_E_SHAPE, "M5P supports at most 256 events (E=%d)", train->E);
  if (train->N == 0) return ctx->fail(SUGG_E_SHAPE, "M5P needs at least one training row");
  if (train->N >= ((int64_t)1 << 31)) return ctx->fail(SUGG_E_BUDGET, "too many training rows for M5P");
  if (train->N * (int64_t)train->E * 8 > kM5pMaxFeatureBytes)
    return ctx->fail(SUGG_E_BUDGET, "M5P training features exceed %lld bytes", (long long)kM5pMaxFeatureBytes);
  M5pParams prm;
  prm.min_leaf = min_leaf;
  prm.smooth_k = smooth_k;
  sugg_plan* p = const_cast<sugg_plan*>(train);
  if (p->dtype == SUGG_F32) return fit_t<float>(ctx, p, (const float*)counters, (const float*)cycles, prm, stream);
  return fit_t<double>(ctx, p, (const double*)counters, (const double*)cycles, prm, stream);
}

int32_t sugg_m5p_tree(sugg_ctx* ctx, int32_t opt, int32_t cap, int32_t* feat, double* thr, int32_t* left,
                      int32_t* right, int64_t* count, int32_t* n_nodes) {
  if (!ctx || !n_nodes || cap < 0) return SUGG_E_ARG;
  const M5pModel* m = ctx->m5p;
  if (!m) return ctx->fail(SUGG_E_STATE, "no M5P model");
  if (opt < 0 || opt >= m->D || m->root[opt] < 0)
    return ctx->fail(SUGG_E_UNTRAINED_OPT, "optimisation %d has no M5P tree", opt);
  const M5pHostTree& t = m->trees[opt];
  const int n = (int)t.feat.size();
  *n_nodes = n;
  if (cap > 0 && (!feat || !thr || !left || !right || !count)) return ctx->fail(SUGG_E_ARG, "null output array");
  for (int i = 0; i < std::min(cap, n); ++i) {
    feat[i] = t.feat[i];
    thr[i] = t.feat[i] >= 0 ? t.thr[i] : std::nan("");
    left[i] = t.left[i];
    right[i] = t.right[i];
    count[i] = t.count[i];
  }
  return SUGG_OK;
}

int32_t sugg_m5p_predict(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles,
                         void* grid_out, void* table_out, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  int rc = common_checks(ctx, plan, counters, cycles);
  if (rc) return rc;
  if (plan->K > 0 && !table_out) return ctx->fail(SUGG_E_ARG, "table_out is required");
  rc = check_m5p_for(ctx, plan);
  if (rc || plan->K == 0) return rc;
  sugg_plan* p = const_cast<sugg_plan*>(plan);
  if (p->dtype == SUGG_F32)
    return score_t<float>(ctx, p, (const float*)counters, (const float*)cycles, (float*)grid_out, (float*)table_out,
                          nullptr, nullptr, nullptr, stream);
  return score_t<double>(ctx, p, (const double*)counters, (const double*)cycles, (double*)grid_out,
                         (double*)table_out, nullptr, nullptr, nullptr, stream);
}

int32_t sugg_m5p_suggest(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles,
                         void* table_out, int32_t* idx_out, void* score_out, int32_t* count_out, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  int rc = common_checks(ctx, plan, counters, cycles);
  if (rc) return rc;
  if (plan->K > 0 && (!idx_out || !score_out || !count_out))
    return ctx->fail(SUGG_E_ARG, "idx_out, score_out and count_out are required");
  rc = check_m5p_for(ctx, plan);
  if (rc || plan->K == 0) return rc;
  sugg_plan* p = const_cast<sugg_plan*>(plan);
  if (p->dtype == SUGG_F32)
    return score_t<float>(ctx, p, (const float*)counters, (const float*)cycles, nullptr, (float*)table_out, idx_out,
                          (float*)score_out, count_out, stream);
  return score_t<double>(ctx, p, (const double*)counters, (const double*)cycles, nullptr, (double*)table_out,
                         idx_out, (double*)score_out, count_out, stream);
}

int32_t sugg_m5p_shape(const sugg_ctx* ctx, int32_t* E, int32_t* D) {
  if (!ctx || !E || !D) return SUGG_E_ARG;
  if (!ctx->m5p) return const_cast<sugg_ctx*>(ctx)->fail(SUGG_E_STATE, "no M5P model");
  *E = ctx->m5p->E;
  *D = ctx->m5p->D;
  return SUGG_OK;
}

int32_t sugg_m5p_export(sugg_ctx* ctx, int64_t nodes_cap, int64_t leaves_cap, int64_t* node_off, int64_t* leaf_off,
                        int32_t* feat, double* thr, int32_t* left, int32_t* right, int32_t* leaf, int64_t* count,
                        double* lw, double* mu, double* isg) {
  if (!ctx || !node_off || !leaf_off || nodes_cap < 0 || leaves_cap < 0) return SUGG_E_ARG;
  const M5pModel* m = ctx->m5p;
  if (!m) return ctx->fail(SUGG_E_STATE, "no M5P model");
  const int E = m->E, D = m->D;
  node_off[0] = leaf_off[0] = 0;
  for (int o = 0; o < D; ++o) {
    node_off[o + 1] = node_off[o] + (int64_t)m->trees[o].feat.size();
    leaf_off[o + 1] = leaf_off[o] + (m->trees[o].feat.empty() ? 0 : m->trees[o].leaves);
  }
  if (nodes_cap == 0 && leaves_cap == 0) return SUGG_OK;   // sizes only
  if (nodes_cap < node_off[D] || leaves_cap < leaf_off[D])
    return ctx->fail(SUGG_E_ARG, "export needs %lld nodes and %lld leaves", (long long)node_off[D],
                     (long long)leaf_off[D]);
  if (!feat || !thr || !left || !right || !leaf || !count || !lw || !mu || !isg)
    return ctx->fail(SUGG_E_ARG, "null output array");
  for (int o = 0; o < D; ++o) {
    const M5pHostTree& t = m->trees[o];
    if (t.feat.empty()) continue;
    for (size_t i = 0; i < t.feat.size(); ++i) {
      const int64_t j = node_off[o] + (int64_t)i;
      feat[j] = t.feat[i];
      thr[j] = t.feat[i] >= 0 ? t.thr[i] : std::nan("");
      left[j] = t.left[i];
      right[j] = t.right[i];
      leaf[j] = t.leaf[i];
      count[j] = t.count[i];
    }
    std::copy(t.lw.begin(), t.lw.begin() + (size_t)t.leaves * (E + 1), lw + leaf_off[o] * (E + 1));
  }
  hipError_t e = hipMemcpy(mu, m->mu64, sizeof(double) * E, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(isg, m->isg64, sizeof(double) * E, hipMemcpyDeviceToHost);
  return ctx->hip(e, "M5P export");
}

int32_t sugg_m5p_import(sugg_ctx* ctx, int32_t E, int32_t D, const int64_t* node_off, const int64_t* leaf_off,
                        const int32_t* feat, const double* thr, const int32_t* left, const int32_t* right,
                        const int32_t* leaf, const int64_t* count, const double* lw, const double* mu,
                        const double* isg) {
  if (!ctx) return SUGG_E_ARG;
  if (E < 1 || E > 256 || D < 1 || D > SUGG_MAX_GLOBAL_OPTS) return ctx->fail(SUGG_E_SHAPE, "bad E or D");
  if (!node_off || !leaf_off || !mu || !isg) return ctx->fail(SUGG_E_ARG, "null argument");
  if (node_off[0] != 0 || leaf_off[0] != 0) return ctx->fail(SUGG_E_ARG, "offsets must start at 0");
  if (node_off[D] > 0 && (!feat || !thr || !left || !right || !leaf || !count || !lw))
    return ctx->fail(SUGG_E_ARG, "null tree array");
  for (int j = 0; j < E; ++j)
    if (!std::isfinite(mu[j]) || !std::isfinite(isg[j]) || !(isg[j] > 0.0))
      return ctx->fail(SUGG_E_ARG, "column statistic %d not finite (or 1/sd not positive)", j);
  if (!device_ok(ctx)) return ctx->fail(SUGG_E_HIP, "cannot select device");
  M5pModel* m = new (std::nothrow) M5pModel();
  if (!m) return ctx->fail(SUGG_E_BUDGET, "out of host memory");
  m->E = E;
  m->D = D;
  m->ldl = m5p_ldl(E);
  m->trees.resize(D);
  int rc = SUGG_OK;
  for (int o = 0; o < D && !rc; ++o) {
    const int64_t n = node_off[o + 1] - node_off[o], nl = leaf_off[o + 1] - leaf_off[o];
    if (n < 0 || nl < 0 || (n == 0) != (nl == 0) || n > (1 << 24)) {
      rc = ctx->fail(SUGG_E_ARG, "id %d: bad node or leaf offsets", o);
      break;
    }
    if (n == 0) continue;
    M5pHostTree& t = m->trees[o];
    t.leaves = (int)nl;
    t.feat.assign(feat + node_off[o], feat + node_off[o + 1]);
    t.thr.assign(thr + node_off[o], thr + node_off[o + 1]);
    t.left.assign(left + node_off[o], left + node_off[o + 1]);
    t.right.assign(right + node_off[o], right + node_off[o + 1]);
    t.leaf.assign(leaf + node_off[o], leaf + node_off[o + 1]);
    t.count.assign(count + node_off[o], count + node_off[o + 1]);
    t.lw.assign(lw + leaf_off[o] * (E + 1), lw + leaf_off[o + 1] * (E + 1));
    // a tree rooted at node 0: every other node the child of exactly one
    // earlier node, internal nodes test a real feature at a finite
    // threshold, leaves name each leaf model exactly once
    std::vector<int> parents(n, 0), depth(n, 0), seen(nl, 0);
    for (int64_t i = 0; i < n && !rc; ++i) {
      if (t.feat[i] >= 0) {
        if (t.feat[i] >= E || !std::isfinite(t.thr[i]) || t.leaf[i] != -1 || t.left[i] <= i || t.right[i] <= i ||
            t.left[i] >= n || t.right[i] >= n || t.left[i] == t.right[i]) {
          rc = ctx->fail(SUGG_E_ARG, "id %d node %lld: bad split", o, (long long)i);
          break;
        }
        ++parents[t.left[i]];
        ++parents[t.right[i]];
        depth[t.left[i]] = depth[t.right[i]] = depth[i] + 1;
      } else {
        if (t.feat[i] != -1 || t.left[i] != -1 || t.right[i] != -1 || t.leaf[i] < 0 || t.leaf[i] >= nl ||
            seen[t.leaf[i]]++) {
          rc = ctx->fail(SUGG_E_ARG, "id %d node %lld: bad leaf", o, (long long)i);
          break;
        }
        t.depth = std::max(t.depth, depth[i]);
      }
    }
    for (int64_t i = 0; i < n && !rc; ++i)
      if (parents[i] != (i == 0 ? 0 : 1)) rc = ctx->fail(SUGG_E_ARG, "id %d: node %lld is not a tree node", o, (long long)i);
    if (!rc && std::count(seen.begin(), seen.end(), 1) != nl) rc = ctx->fail(SUGG_E_ARG, "id %d: unused leaf model", o);
    for (double v : t.lw)
      if (!rc && !std::isfinite(v)) rc = ctx->fail(SUGG_E_ARG, "id %d: leaf model not finite", o);
  }
  if (!rc) rc = upload_model(ctx, m);
  if (!rc) {
    hipError_t e = put(m->mu64, std::vector<double>(mu, mu + E));
    if (e == hipSuccess) e = put(m->isg64, std::vector<double>(isg, isg + E));
    rc = ctx->hip(e, "M5P statistics upload");
  }
  if (rc) {
    m5p_model_free(m);
    return rc;
  }
  m5p_model_free(ctx->m5p);
  ctx->m5p = m;
  return SUGG_OK;
}

}  // extern "C"
