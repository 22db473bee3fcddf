// Internal: the instance-based Tier 2 model (IBK, k nearest neighbours by
// Euclidean distance between standardised feature vectors, Section 3.4), its
// device database and the per-plan query workspace.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace sugg {

constexpr int kIbkMaxK = 16;       // largest k
constexpr int kIbkList = 24;       // FP32 candidates kept per query (k plus a margin, at most 24)
constexpr int kIbkQueries = 128;   // queries per workgroup (4 waves x 32)
constexpr int kIbkTile = 32;       // database samples per staged tile
constexpr int kIbkQueue = 30;      // queued candidates per lane (at least 16, one tile's)

// Database of one fitted IBK model.  Samples of global optimisation o are
// [off[o], off[o+1]), stored kernel by kernel, then by before-version S; each
// is the standardised vector of its before version (a row of Z) and a label.
struct IbkModel {
  int E = 0, Epad = 0, D = 0, k = 10;
  int64_t Ntr = 0, Ns = 0;
  float* Z = nullptr;          // [Ns, Epad] FP32 sample vectors, columns >= E zero
  double* Z64 = nullptr;       // [Ntr, E] FP64 standardised training rows (exact distances)
  int32_t* srow = nullptr;     // [Ns] training row of each sample (its before version)
  double dt_norm = 0.0;        // Euclidean norm over columns of max_rows |Z32 - Z64|: the
                               //   FP32 rounding of any stored vector is at most this
  float* norm = nullptr;       // [Ns] their squared norms
  double* y = nullptr;         // [Ns] ln cyc(before) - ln cyc(after)
  int64_t* d_off = nullptr;    // [D+1]
  double* mu64 = nullptr;      // [E] training column means of ln(c / cyc)
  double* sig64 = nullptr;     // [E] and population standard deviations
  void* mu_t = nullptr;        // [E] the statistics in the training dtype (written by
  void* isg_t = nullptr;       //     the shared column-statistics kernel, unused here)
  std::vector<int64_t> off;    // host copy of d_off
};

// Query lists of one plan for one output mode.  Mode 0 (edges): one query per
// version S >= 1 of every kernel, the prediction of adding its highest bit to
// S without it (the last step of its ascending chain), written to row(k, S).
// Mode 1 (grid): one query per (version S, local bit b not in S), written to
// grid[row(k, S) * Bmax + b].  Queries are grouped by global id; a tile is
// (id, first query, count <= kIbkQueries).
struct IbkQueries {
  bool built = false;
  int64_t n = 0;
  int n_tiles = 0;
  int32_t* src = nullptr;      // [n] row whose feature vector is the query
  int64_t* dst = nullptr;      // [n] output index
  int32_t* tiles = nullptr;    // [n_tiles * 4]
  std::vector<int64_t> per_opt;
};

struct IbkPlan {
  int Epad = 0;
  float* zq = nullptr;         // [N, Epad] standardised rows of the batch
  void* edges = nullptr;       // [N] plan dtype: chain-edge predictions
  float* part_d = nullptr;     // candidate lists of every query (per sample share when split)
  int32_t* part_i = nullptr;
  int64_t part_cap = 0;        // entries allocated
  int32_t* exact_q = nullptr;  // queries whose FP32 candidates could not be certified, and
  int32_t* exact_n = nullptr;  //   their count (device), searched again in FP64
  int64_t exact_cap = 0;
  int exact_mode = -1;         // output form of the last call (0 edges, 1 grid)
  IbkQueries q[2];
};

struct IbkKnnArgs {
  const float* zq;
  const float* Z;
  const float* norm;
  const double* y;
  const int64_t* off;
  const int32_t* q_src;
  const int64_t* q_dst;
  const int32_t* tiles;
  int32_t Epad;
  int32_t k;
  int32_t kt;                  // FP32 candidates kept per query (k plus a margin)
  int32_t split;               // sample partitions per query tile (workgroups per tile)
  float* part_d;               // [queries, split, kIbkList] candidate lists
  int32_t* part_i;
  int64_t n_queries;
  int32_t n_tiles;
  void* out;                   // plan dtype
  // exact re-ranking: FP64 features of the queries (from the plan's counters)
  // and of the samples (training rows), and the queue of uncertified queries
  const void* counters;        // plan dtype [N, E]
  const void* cycles;          // plan dtype [N]
  int32_t E;
  const double* mu64;
  const double* sig64;
  const double* Z64;           // [Ntr, E]
  const int32_t* srow;         // [Ns]
  double dt_norm;              // IbkModel::dt_norm
  int32_t* exact_q;
  int32_t* exact_n;
};

template <typename T>
hipError_t launch_ibk_z(const T* counters, const T* cycles, int64_t N, int32_t E, int32_t Epad,
                        const double* mu, const double* sig, float* z, int32_t* status, hipStream_t s);
template <typename T>
hipError_t launch_ibk_nan(T* p, int64_t n, hipStream_t s);
hipError_t launch_ibk_norm(const float* z, int64_t N, int32_t Epad, float* norm, hipStream_t s);
hipError_t launch_ibk_gather(const float* Z, const int32_t* srow, int64_t Ns, int32_t Epad, float* Zs,
                             hipStream_t s);
template <typename T>
hipError_t launch_ibk_labels(const T* cycles, const int32_t* before, const int32_t* after, int64_t Ns,
                             double* y, hipStream_t s);
// per column, the largest |z32 - z64| over the rows (as float bits, maxed into out[E])
hipError_t launch_ibk_dz(const float* z32, int32_t Epad, const double* z64, int64_t N, int32_t E, uint32_t* out,
                         hipStream_t s);
// FP32 candidate search, re-ranking of the candidates by FP64 distance with a
// certificate, and an FP64 search over every sample for the queries the
// certificate does not cover; writes the mean label of the k nearest
template <typename T>
hipError_t launch_ibk_knn(const IbkKnnArgs& a, int n_tiles, hipStream_t s);
// candidates kept per query for a given k
inline int ibk_kt(int k) { return k <= 4 ? 8 : k <= 10 ? 16 : 24; }
int ibk_split(int Epad, int k, int n_tiles, int cus);
// Composition and top-n from chain edges (dtype TE, the composition's
// arithmetic) or from a grid (dtype TO); outputs of dtype TO.
template <typename TE, typename TO>
hipError_t launch_ibk_compose(const TE* edges, const TO* grid, int32_t grid_ld, const int64_t* row_off,
                              const int32_t* nopts, int32_t K, int32_t Bmax, TO* table, int32_t* idx_out,
                              TO* score_out, int32_t* count_out, int32_t n, TE tau, hipStream_t s);

}  // namespace sugg

using sugg::IbkModel;
using sugg::IbkPlan;

void ibk_model_free(IbkModel*& m);
void ibk_plan_free(IbkPlan*& p);
