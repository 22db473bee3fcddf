// Internal: graphs and plans (the host-built structure of a batch), shared by
// the C entry points of the linear and the instance-based scoring paths.
#pragma once

#include <cstdint>
#include <vector>

#include "ctx.hpp"
#include "ibk.hpp"

struct sugg_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = 0;
  ~sugg_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

// Workspace of a plan's serving queries (sugg_serve_query), built on first use.
struct ServeWs {
  int cap = 0;
  float *ys = nullptr, *sc = nullptr, *br = nullptr, *bout = nullptr;
  int32_t* bc = nullptr;
  int64_t* seg = nullptr;
  ~ServeWs() {
    dfree(ys); dfree(sc); dfree(br); dfree(bout); dfree(bc); dfree(seg);
  }
};

int mlp_infer(sugg_ctx* ctx, sugg_mlp* m, const float* x, int B, float* y, hipStream_t s);
struct sugg_plan;
// sugg_load_features with the column-statistics partials in `partial` (null:
// the plan's workspace, allocated on first use) (api.cpp)
int load_features_core(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles, int32_t mode,
                       void* z_out, hipStream_t stream, double* partial);
// looks up, once per device, the address of the library's static scratch
// array on the current device (noalloc.hip); SUGG_OK or SUGG_E_HIP
int noalloc_scratch_setup(int device);
void mlp_dims(const sugg_mlp* m, int* in, int* out, int* max_batch);
// the BF16 input buffer of the mlp ([max_batch x in], row stride in), and
// frozen inference with ranking (as sugg_mlp_infer_rank) from what it holds
__bf16* mlp_input(sugg_mlp* m);
int mlp_infer_rank_input(sugg_ctx* ctx, sugg_mlp* m, int B, int skip, int n, float tau, float* y, int32_t* idx,
                         float* score, int32_t* count, hipStream_t s);

struct sugg_plan {
  sugg_ctx* ctx = nullptr;   // identity only: never dereferenced after creation
  int device = 0;
  int K = 0, E = 0, D = 0, dtype = SUGG_F32, Bmax = 0;
  int64_t N = 0;
  std::vector<int32_t> nopts, opt_ids;
  std::vector<int64_t> row_off, opt_off;
  std::vector<int64_t> opt_pairs;   // per global id: number of before/after pairs
  // device structure
  sugg::Item* d_items = nullptr;
  sugg::KRec* d_recs = nullptr;
  int64_t* d_row_off = nullptr;
  int64_t* d_opt_off = nullptr;
  int32_t* d_opt_ids = nullptr;
  int32_t* d_nopts = nullptr;
  int32_t* d_queue = nullptr;
  // split form of the scoring pass (equal kernels, B <= 6): per-kernel arrival
  // counters (zero between launches) and the chain-edge buffer [N]
  int32_t* d_arrivals = nullptr;
  void* d_split_edges = nullptr;
  // streaming form: chunks of consecutive whole kernels (about item_rows rows)
  sugg::Chunk* d_chunks = nullptr;
  sugg::CRec* d_crec = nullptr;   // [K] each kernel's record within its chunk
  int n_chunks = 0, chunk_max_rows = 1, chunk_max_nk = 1;
  bool split_ok() const { return uni_B >= 0 && uni_B <= 6 && uni_ops && d_arrivals; }
  int n_items = 0, max_item_rows = 1, max_item_kernels = 1;
  int uni_B = -1, uni_nk = 0;
  int uni_ops = 0;
  uint64_t uni_opt_lo = 0, uni_opt_hi = 0;
  sugg::PathLaunch cfg{4, 2, 0};   // launch shape of the scoring kernel (autotuned)
  int item_rows = 256;             // target rows of a work item (autotuned)
  // statistics workspace
  double* d_stat_partial = nullptr;
  int stat_chunks = 1;
  // fit workspace (allocated on the first fit)
  bool fit_ready = false;
  double* d_z64 = nullptr;
  double* d_lcyc64 = nullptr;
  double* d_gram_partial = nullptr;
  double* d_solveA = nullptr;
  double* d_reduced = nullptr;
  sugg::GramWork* d_gwork = nullptr;
  int64_t* d_pair_base = nullptr;
  int64_t* d_pair_row0 = nullptr;
  int32_t* d_pair_bit = nullptr;
  int32_t* d_opt_work_begin = nullptr;
  int n_gwork = 0;
  // instance-based (IBK) scoring workspace, built on its first use
  IbkPlan* ibk = nullptr;
  M5pPlan* m5p = nullptr;
  ServeWs* serve = nullptr;

  ~sugg_plan() {
    delete serve;
    ibk_plan_free(ibk);
    m5p_plan_free(m5p);
    dfree(d_items); dfree(d_recs); dfree(d_row_off); dfree(d_opt_off); dfree(d_opt_ids); dfree(d_nopts);
    dfree(d_queue); dfree(d_arrivals); dfree(d_split_edges); dfree(d_chunks); dfree(d_crec); dfree(d_stat_partial); dfree(d_z64); dfree(d_lcyc64); dfree(d_gram_partial);
    dfree(d_solveA); dfree(d_reduced); dfree(d_gwork); dfree(d_pair_base); dfree(d_pair_row0); dfree(d_pair_bit);
    dfree(d_opt_work_begin);
  }
};
