// Host-side launch interface of the HIP kernels (internal to libsugg).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace sugg {

// One kernel of a work item: where its rows start, its index in the batch and
// its global optimisation ids (ascending; bit b of a version <-> opt[b]).
struct alignas(16) KRec {
  int64_t row_off;
  int32_t kid;
  int32_t pad;
  uint8_t opt[16];
};

// Row stride of the FP32 weight copy: E weights and the intercept, padded to
// a multiple of 4 so every row starts 16-byte aligned.
__host__ __device__ inline int w32_ld(int E) { return (E + 4) & ~3; }

// Arguments of the judge: plain composed log-speedups of given subsets.
template <typename T>
struct JudgeArgs {
  const T* counters;
  const T* cycles;
  int32_t E;
  int32_t D;
  const T* W;              // [D, ldw]: E weights then the intercept
  int32_t ldw;             // row stride of W
  const T* mu;
  const T* isg;
  const int64_t* row_off;  // [K+1]
  const int32_t* nopts;    // [K]
  const int64_t* opt_off;  // [K+1]
  const int32_t* opt_ids;
  int32_t K;
  int32_t C;               // candidates per kernel
  const int32_t* cand;     // [K, C] subset bitmasks, < 0 = none
  T* out;                  // [K, C]; 0 for S = 0, NaN for none
  const T* ref;            // [K, C] reference values (with flag)
  double tol;
  int32_t* flag;           // [K] or null: 1 where some candidate differs from ref by > tol
  int32_t accumulate;      // nonzero: keep flags already set (no clearing)
  int32_t* status;
  // a second candidate set judged in the same launch (C2 = 0: none), with
  // its own cand2 [K, C2], out2 and ref2, and the same flags
  int32_t C2;
  const int32_t* cand2;
  T* out2;
  const T* ref2;
};

// Arguments of the fused scoring kernel (predict / suggest).
template <typename T>
struct PathArgs {
  const JudgeArgs<T>* judge;   // non-null: run the judge instead (same dispatch)
  const int32_t* kmask;        // [K] or null: only kernels with kmask != 0 are scored and written
  const T* counters;       // [N, E]
  const T* cycles;         // [N]
  int32_t E;
  int32_t D;
  const Item* items;       // work list
  const KRec* recs;        // kernels of the items, item after item
  int32_t n_items;
  int32_t K;
  int32_t uni_B;           // >= 0: all kernels have uni_B optimisations and item i
  int32_t uni_nk;          //       holds kernels [i*uni_nk, (i+1)*uni_nk) (items unused)
  int32_t uni_ops;         // nonzero (with uni_B >= 0): every kernel has the same global
  uint64_t uni_opt_lo;     //   optimisation ids, byte b of (lo, hi) = id of local bit b;
  uint64_t uni_opt_hi;     //   the kernel records are then not read
  int32_t* queue;          // [2] next item, finished workgroups; zero at launch, re-armed by the kernel
  const T* mu;             // [E]
  const T* isg;            // [E] 1 / sigma
  const T* W;              // [D, ldw]: E weights then the intercept
  int32_t ldw;             // row stride of W
  T* grid;                 // [N, grid_ld] or null
  int32_t grid_ld;
  T* table;                // [N] or null
  int32_t* idx_out;        // [K, n] or null (no ranking)
  T* score_out;
  int32_t* count_out;
  int32_t n;
  T tau;
  int32_t* status;
};

struct PathLaunch {
  int waves;       // waves per workgroup (1..8)
  int unroll;      // rows per lane group per iteration (1, 2, 4)
  int grid;        // workgroups (persistent); 0 = occupancy-derived
};

// Fused normalise -> candidate predict -> compose [-> rank]; VPL = columns
// per lane (E <= 16 * VPL), instantiated for VPL 4, 8, 16.
template <typename T, int VPL>
hipError_t launch_path_vpl(const PathArgs<T>& a, int max_item_rows, int max_item_kernels, int max_B,
                           const PathLaunch& cfg, hipStream_t s);
// Split form for batches of equal kernels (same B <= 6, same ids, rows kernel
// after kernel): 16-version workgroups write chain edges to edges[N]; the
// last of a kernel's workgroups (arrivals[k], zero between launches, re-armed
// by that workgroup) composes and ranks.  Same results as the fused kernel.
template <typename T>
hipError_t launch_path_split(const PathArgs<T>& a, int32_t* arrivals, T* edges, hipStream_t s);

// The streaming form of the scoring pass: workgroups take chunks of
// consecutive whole kernels in memory order (mixed B), one chunk each.
struct alignas(16) Chunk {
  int64_t row0;   // first row
  int32_t k0;     // first kernel
  int32_t nk;     // kernels
  int32_t R;      // rows
  int32_t pad[3];
};
// One kernel of a chunk (kernel order, one record per kernel of the batch):
// its first row relative to its chunk's, its B and global ids (bit b <-> op[b]).
struct alignas(16) CRec {
  int16_t rel;
  int8_t B;
  int8_t pad;
  uint8_t op[12];
};
static_assert(sizeof(CRec) == 16 && SUGG_MAX_OPTS <= 12, "chunk kernel record");
template <typename T>
struct ChunkArgs {
  const T* counters;
  const T* cycles;
  int32_t E;
  int32_t D;
  const T* W;
  int32_t ldw;
  const T* mu;
  const T* isg;
  const CRec* recs;          // [K]
  const Chunk* chunks;
  int32_t n_chunks;
  int32_t max_rows;          // largest chunk
  int32_t max_nk;            // most kernels in a chunk
  T* table;                  // nullable
  int32_t* idx_out;          // nullable (then no ranking)
  T* score_out;
  int32_t* count_out;
  int32_t n;
  T tau;
  int32_t* status;
};
// unroll: rows per lane group per stage (1, 2, 4); one workgroup per chunk
template <typename T>
hipError_t launch_path_chunks(const ChunkArgs<T>& a, int unroll, hipStream_t s);
// dynamic LDS of the streaming form
size_t path_chunk_lds(size_t tsize, int D, int E, int max_rows, int max_nk);

template <typename T>
hipError_t launch_path(const PathArgs<T>& a, int max_item_rows, int max_item_kernels,
                       int max_B, const PathLaunch& cfg, hipStream_t s);

// Generic segmented top-n.
template <typename T>
hipError_t launch_rank(const T* scores, const int64_t* seg_off, int32_t nseg, int32_t skip_head,
                       int32_t n, T tau, int32_t* idx_out, T* score_out, int32_t* count_out,
                       hipStream_t s, int64_t seg_len = 0);   // seg_off null: segments of seg_len

// Threshold band of short suggestion lists (entries outside the list with
// score >= lo, ascending, at most C per segment; flag 1 on overflow).
template <typename T>
hipError_t launch_band(const T* scores, const int64_t* seg_off, int32_t nseg, int32_t skip_head,
                       const int32_t* top_idx, const int32_t* top_count, int32_t n, double lo, int32_t C,
                       int32_t* cand_out, T* ref_out, int32_t* flag_out, hipStream_t s);
// serving: flag kernels whose kept answer breaks Tier 3's threshold by the
// plain values, sort the others' lists by them
hipError_t launch_confirm(int32_t K, int32_t n, int32_t* idx, float* plain, const int32_t* count,
                          const int32_t* band_idx, const float* band_plain, int32_t C, float tau, int32_t* flag,
                          hipStream_t s);

// FP64 column statistics of x = ln(c / cyc) over all N rows.
template <typename T>
hipError_t launch_colstats(const T* counters, const T* cycles, int64_t N, int32_t E,
                           double* partial, int32_t nchunks, double* mu64, double* sig64,
                           T* mu_t, T* isg_t, int32_t* status, hipStream_t s);
int colstats_chunks(int64_t N);

// z = (x - mu) / sigma in the plan dtype.
template <typename T>
hipError_t launch_standardize(const T* counters, const T* cycles, int64_t N, int32_t E, const T* mu,
                              const T* isg, T* z, int32_t* status, hipStream_t s);

// z of the rows listed in rows[nrows] (e.g. each kernel's baseline version).
template <typename T>
hipError_t launch_standardize_rows(const T* counters, const T* cycles, const int64_t* rows, int64_t nrows, int32_t E,
                                   const T* mu, const T* isg, T* z, int32_t* status, hipStream_t s);
// the same values rounded to BF16, row i at z + i * ldz (the surrogate's input)
hipError_t launch_standardize_rows_bf16(const float* counters, const float* cycles, const int64_t* rows, int64_t nrows,
                                        int32_t E, const float* mu, const float* isg, __bf16* z, int32_t ldz,
                                        int32_t* status, hipStream_t s);

// FP64 z and ln(cycles) for the regression.
template <typename T>
hipError_t launch_zfeat64(const T* counters, const T* cycles, int64_t N, int32_t E,
                          const double* mu64, const double* sig64, double* z64, double* lcyc64,
                          hipStream_t s);

// One chunk of one optimisation's training pairs.
struct GramWork {
  int32_t opt;
  int32_t list_begin;   // into the per-optimisation (kernel, bit) list
  int32_t list_end;
  int32_t pad;
  int64_t s_begin;      // sample range within the optimisation's pair space
  int64_t s_end;
};

struct GramArgs {
  const double* z64;        // [N, E]
  const double* lcyc64;     // [N]
  int32_t E;
  const GramWork* work;
  int32_t n_work;
  const int64_t* pair_base; // [list] first pair index of each (kernel, bit) entry
  const int64_t* pair_row0; // [list] row_off of the kernel
  const int32_t* pair_bit;  // [list] local bit
  double* partial;          // [n_work, E*E + 2E + 2]
};

hipError_t launch_gram(const GramArgs& a, hipStream_t s);

// Sum the chunks of every optimisation (work items sorted by opt) and solve.
struct SolveArgs {
  const double* partial;
  const int32_t* opt_work_begin;  // [D+1] range of work items per optimisation
  int32_t E;
  int32_t D;
  double lambda;
  double* reduced;    // [D, E*E + 2E + 2] workspace: summed partials
  double* A;          // [D, (E+1)^2] workspace when the system does not fit in LDS
  double* W64;        // [D, E+1]
  float* W32;         // [D, w32_ld(E)]
  int32_t* status;
};

hipError_t launch_solve(const SolveArgs& a, hipStream_t s);

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);

// Arguments of the all-paths composition and greedy re-profiling kernels.
template <typename T>
struct PathsArgs {
  const T* counters;
  const T* cycles;
  int32_t E, D, ldw;
  const T* W;
  const T* mu;
  const T* isg;
  const int64_t* row_off;
  const int32_t* nopts;
  const int64_t* opt_off;
  const int32_t* opt_ids;
  int32_t K, Bmax, n;
  T tau;
  T* table;          // allpaths: [N]
  int32_t* idx_out;  // allpaths (nullable): [K, n]
  T* score_out;
  int32_t* count_out;
  int32_t* path_out;  // greedy: [K, Bmax + 1]
  int32_t* steps_out; // greedy: [K]
  T* gain_out;        // greedy: [K]
  int32_t* status;
};

template <typename T>
hipError_t launch_paths(const PathsArgs<T>& a, bool greedy, hipStream_t s);
template <typename T>
size_t paths_lds_bytes(int D, int E, int Bmax);

// ---- surrogate MLP --------------------------------------------------------
enum GemmEpilogue : int {
  kEpiWgrad = 0,       // FP32 split-K partial of a weight gradient
  kEpiFwdHidden = 1,   // + bias, keep pre-activation, GELU, BF16 row-major and transposed
  kEpiFwdOut = 2,      // + bias -> Y; with targets: squared error partials and dY
  kEpiBwdHidden = 3,   // * GELU'(pre-activation) -> BF16 row-major and transposed
  kEpiFwdRank = 4      // + bias -> Y (optional) and each row's top n above tau (the tile spans N)
};

// C[M x N] = A[M x K] . Bt[N x K]^T, BF16 operands, FP32 accumulation.
struct GemmArgs {
  const __bf16* A;
  int lda;
  const __bf16* Bt;
  int ldb;
  int M, N, K;
  int k_per_split;       // K range of one split (grid z), multiple of 32
  const float* bias;     // [N]
  float* Cf;             // FP32 output (pre-activation, Y or split partials)
  int ldcf;
  __bf16* Cb;            // BF16 row-major output
  int ldcb;
  __bf16* Ct;            // BF16 transposed output [N x M]
  int ldct;
  const float* gact;     // pre-activation for GELU'
  int ldg;
  const float* target;   // [M x N] targets
  int ldt;
  const int32_t* trow;   // nullable: output row r's target is row trow[r] of target
  int32_t* idx_out;      // kEpiFwdRank: [M x n] columns of each row's top n (-1 padded),
  float* score_out;      //   their values (NaN padded) and the count; columns >= skip
  int32_t* count_out;    //   with value > tau, by value descending then column ascending
  int n, skip;
  float tau;
  float* loss_part;      // one partial per output tile
  float scale;           // dY = scale * (Y - T)
};

// info (nullable, 4 ints): the launched instance as (tile rows, tile columns,
// K splits, 1 if the variant without bounds checks ran)
hipError_t launch_gemm(const GemmArgs& g, int epi, int splits, hipStream_t s, int32_t* info = nullptr);
// the output layer with the ranking epilogue: N must be 64 or 128, n <= 8
hipError_t launch_gemm_rank(const GemmArgs& g, hipStream_t s, int32_t* info = nullptr);
hipError_t launch_pack(const float* src, int rows, int cols, __bf16* dst, int ldd, __bf16* dst_t, int ldt,
                       hipStream_t s);
hipError_t launch_loss_sum(const float* part, int n, float scale, float* loss, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s);
// Rows idx[0..rows) of the FP32 matrix src [src_rows x cols] to BF16
// row-major dst and transposed dst_t (as launch_pack); an index outside
// [0, src_rows) reads row 0 and sets kStatusBadIndex in status.  The rows
// read are written to rows_out [rows].
struct GatherArgs {
  const float* src;
  int64_t src_rows;
  int cols;
  const int32_t* idx;
  int rows;
  __bf16* dst;
  int ldd;
  __bf16* dst_t;
  int ldt;
  int32_t* rows_out;
  int32_t* status;
};
hipError_t launch_gather_pack(const GatherArgs& g, hipStream_t s);
// A weight gradient dW[M x N] = A[M x K] . Bt[N x K]^T split over K and a
// hidden-layer backward (kEpiBwdHidden, one split) that do not depend on each
// other, in one launch where their instances allow (else two launches; the
// results are the same either way).
hipError_t launch_gemm_pair(const GemmArgs& gw, int splits, const GemmArgs& gb, hipStream_t s,
                            int32_t* info_w = nullptr, int32_t* info_b = nullptr);
// The end of up to three weight gradients in one launch: split-K sums (in
// split order) of the partials part [splits x n] into out [n], and row sums
// of the transposed BF16 activation gradient x [rows x cols] (leading
// dimension ld; its bias gradient) into bias_out [rows]; with loss non-null
// also the loss as launch_loss_sum.
struct WgradJob {
  const float* part;
  int64_t n;
  int splits;
  float* out;
  const __bf16* x;
  int rows, cols, ld;
  float* bias_out;
};
struct FinishArgs {
  WgradJob job[3];
  int njobs;
  const float* loss_part;   // nullable
  int loss_n;
  float loss_scale;
  float* loss;
};
hipError_t launch_wgrad_finish(const FinishArgs& a, hipStream_t s);
// Adam (as launch_adam) over the surrogate's flat parameters, writing the
// updated weights of its three layers to their BF16 working copies
// (row-major w[l]; transposed wt[l] where non-null, leading dimension = rows)
struct AdamPackArgs {
  float* p;
  const float* g;
  float* m;
  float* v;
  int64_t n;
  float lr, b1, b2, eps, c1, c2;
  int64_t off[3];     // first parameter of each weight matrix
  int rows[3], cols[3];
  __bf16* w[3];
  __bf16* wt[3];
};
hipError_t launch_adam_pack(const AdamPackArgs& a, int step, hipStream_t s);
// launch_adam_pack of one step and launch_gather_pack of the next mini-batch
// in one launch (the gather does not depend on the update)
hipError_t launch_adam_gather(const AdamPackArgs& a, int step, const GatherArgs& g, hipStream_t s);

}  // namespace sugg
