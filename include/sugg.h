/*
 * sugg.h - C ABI of the optimisation-suggestion scoring library (gfx950).
 *
 * The library implements the data-parallel path of the suggestion tool of
 * Taheri, Qasem and Burtscher, "A Tool for Automatically Suggesting
 * Source-Code Optimizations for Complex GPU Kernels": profiled counter vectors
 * are normalised by the cycle count (Section 2, Tier 1), one regression model
 * per optimisation is trained on before/after version pairs and predicts the
 * speedup of adding it (Section 2, Tier 2; Sections 3.3-3.4), and the
 * candidates are sorted by expected benefit and kept above a threshold
 * (Section 2, Tier 3).
 *
 * Data model
 *   A batch ("plan") holds K kernels.  Kernel k has B_k binary optimisations
 *   (0 <= B_k <= SUGG_MAX_OPTS) with global ids O_k[0..B_k), strictly
 *   ascending, each < D.  Every version S in [0, 2^B_k) (bit b of S set means
 *   optimisation O_k[b] is applied) has one profiled row.  Rows are stored
 *   kernel after kernel: row(k, S) = row_off[k] + S with
 *   row_off[k] = sum_{i<k} 2^B_i, N = row_off[K] rows in total.
 *   counters: N x E row-major, cycles: N, both of the plan's dtype, device
 *   memory owned by the caller.  Every value must be finite and > 0.
 *
 * Conventions
 *   - Every call returns SUGG_OK (0) or a negative SUGG_E_* code; the message
 *     is available from sugg_last_error().  No exception crosses the ABI.
 *   - Argument and shape errors are detected on the host, synchronously.
 *     Data errors (non-finite or non-positive counters, a singular system)
 *     are detected on the device and returned by the next sugg_sync().
 *   - Work is enqueued on the caller's HIP stream and is asynchronous unless
 *     stated otherwise; a context must not be used from two streams at once
 *     (calls that overlap on one context race on its model and status word).
 *   - Device pointers are caller-owned; the library allocates its own
 *     workspace at plan creation (and on the first fit with a plan), never in
 *     sugg_predict, sugg_suggest or sugg_rank_suggest.
 */
#ifndef SUGG_H
#define SUGG_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SUGG_API __attribute__((visibility("default")))

enum {
  SUGG_OK = 0,
  SUGG_E_ARG = -1,           /* bad argument (null pointer, bad enum, bad n) */
  SUGG_E_SHAPE = -2,         /* inconsistent sizes or layout */
  SUGG_E_BAD_COUNTER = -3,   /* a counter or cycle count that is <= 0, NaN or Inf */
  SUGG_E_UNTRAINED_OPT = -4, /* an optimisation id with no fitted model */
  SUGG_E_SINGULAR = -5,      /* a regression system is not positive definite */
  SUGG_E_BUDGET = -6,        /* request exceeds a size limit of the library */
  SUGG_E_HIP = -7,           /* HIP runtime error */
  SUGG_E_STATE = -8          /* call out of order (e.g. predict before fit) */
};

enum { SUGG_F32 = 0, SUGG_F64 = 1 };          /* dtype of counters and results */
enum { SUGG_FIT_STATS = 1, SUGG_APPLY = 2, SUGG_BASELINE = 4 };  /* sugg_load_features modes */

#define SUGG_MAX_OPTS 12      /* max optimisations per kernel (4096 versions) */
#define SUGG_MAX_EVENTS 256   /* max counter events per row */
#define SUGG_MAX_GLOBAL_OPTS 64
#define SUGG_MAX_SUGGEST 8    /* max suggestions per segment */

typedef struct sugg_ctx sugg_ctx;
typedef struct sugg_plan sugg_plan;
typedef struct sugg_graph sugg_graph;
typedef struct sugg_mlp sugg_mlp;

typedef struct {
  double lambda;      /* ridge penalty on the feature weights (intercept unpenalised) */
  double tau;         /* threshold on the predicted log-speedup; strict ">" */
  int32_t n_suggest;  /* suggestions kept per kernel, 1..SUGG_MAX_SUGGEST */
  int32_t reserved;
} sugg_params;

/* Context: owns the fitted model (column statistics and one regression per
 * global optimisation id), the device status word and its error message.
 * device: HIP device ordinal; params may be NULL (lambda 1e-2, tau ln 1.05,
 * n_suggest 3). */
SUGG_API int32_t sugg_create(sugg_ctx** out, int32_t device, const sugg_params* params);
SUGG_API void sugg_destroy(sugg_ctx* ctx);
SUGG_API const char* sugg_last_error(const sugg_ctx* ctx);
SUGG_API int32_t sugg_set_params(sugg_ctx* ctx, const sugg_params* params);
SUGG_API int32_t sugg_get_params(const sugg_ctx* ctx, sugg_params* out);

/* Plan: the structure of a batch (Section 3.3's version lattice per kernel).
 * nopts[K] and opt_ids[sum B_k] are HOST arrays, copied.  D is the number of
 * global optimisation ids, dtype SUGG_F32 or SUGG_F64.  Validates the layout,
 * builds the ragged work list (kernels grouped by B, largest first) and
 * uploads it.  Synchronous. */
SUGG_API int32_t sugg_plan_create(sugg_ctx* ctx, int32_t K, int32_t E, int32_t D, int32_t dtype,
                                  const int32_t* nopts, const int32_t* opt_ids, sugg_plan** out);
SUGG_API void sugg_plan_destroy(sugg_plan* plan);
SUGG_API int64_t sugg_plan_rows(const sugg_plan* plan);     /* N, or -1 */
SUGG_API int32_t sugg_plan_max_opts(const sugg_plan* plan); /* max B_k, or -1 */

/* Launch shape of the plan's scoring kernel: waves per workgroup (1-8),
 * rows per lane group and pipeline stage (1, 2 or 4), workgroups (0 = as
 * many as fit on the device at once).  unroll = 0 selects the split form for
 * plans whose kernels all have the same B <= 6 and the same ids: 16 versions
 * per workgroup, the last of a kernel's workgroups composing and ranking it
 * (per-plan counters, re-armed by each launch).  unroll = -1, -2 or -4
 * selects the streaming form (1, 2 or 4 rows per lane group and stage):
 * workgroups of 4 waves each take a chunk of consecutive whole kernels in
 * memory order (about sugg_plan_get_items rows, any mix of B) and stream,
 * compose and rank it.  The split and streaming forms serve sugg_suggest and
 * sugg_predict without a grid; other calls take the fused form with unroll
 * 1.  Results do not depend on the shape. */
SUGG_API int32_t sugg_plan_set_launch(sugg_plan* plan, int32_t waves, int32_t unroll, int32_t grid);
SUGG_API int32_t sugg_plan_get_launch(const sugg_plan* plan, int32_t* waves, int32_t* unroll, int32_t* grid);

/* Work-item size of the plan's scoring pass: kernels of equal B are packed
 * into items of about `rows` versions for the fused form, and consecutive
 * kernels into chunks of at most `rows` versions for the streaming form (a
 * kernel with more versions is an item or chunk alone); 16 <= rows <= 4096.  Rebuilds and uploads the work list
 * (synchronous; not inside a graph capture).  Results do not depend on it.
 * sugg_plan_get_items returns the current size (-1 for a null plan). */
SUGG_API int32_t sugg_plan_set_items(sugg_ctx* ctx, sugg_plan* plan, int32_t rows);
SUGG_API int32_t sugg_plan_get_items(const sugg_plan* plan);

/* Autotuner: times the fused scoring pass (sugg_suggest) of this plan on the
 * given inputs for every candidate: for item sizes 64, 128, 256, 512 and
 * 1024 rows, waves 2, 4, 8 x unroll 1, 2, 4, then the streaming form with
 * unroll -1, -2, -4 (12 shapes per size, in that order), then the split form
 * where the plan has one (with the plan's item size); reps timed passes each
 * after one warm-up; the four fastest are then timed again in two rounds of
 * 2 reps passes each, and the best of those is kept in the plan.  times_ms
 * (nullable, at least SUGG_TUNE_CANDIDATES floats, times_cap its length)
 * receives the mean pass time of each candidate, the second timing for the
 * four finalists (-1 for one the plan cannot run: an item size whose
 * workspace exceeds LDS, a split form it does not have).  Needs a fitted
 * model; allocates and frees temporary outputs; synchronises the stream. */
#define SUGG_TUNE_CANDIDATES 61
SUGG_API int32_t sugg_autotune(sugg_ctx* ctx, sugg_plan* plan, const void* counters, const void* cycles,
                               int32_t reps, float* times_ms, int32_t times_cap, hipStream_t stream);

/* Tier 1 (Section 2): features are ln(counter / cycles).
 * mode SUGG_FIT_STATS: set the context's column statistics (mean, population
 *   standard deviation; sigma < 1e-12 is replaced by 1) from all N rows,
 *   computed in FP64 whatever the dtype.
 * mode SUGG_APPLY: requires statistics; z_out (nullable) receives the
 *   standardised features z = (x - mu) / sigma, N x E, plan dtype.
 * SUGG_APPLY | SUGG_BASELINE: z_out is K x E and holds only each kernel's
 *   baseline version (S = 0): the learned surrogate's input.
 * FIT_STATS | APPLY does both. */
SUGG_API int32_t sugg_load_features(sugg_ctx* ctx, const sugg_plan* plan, const void* counters,
                                    const void* cycles, int32_t mode, void* z_out, hipStream_t stream);

/* sugg_load_features for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, modes, results (bit-identical) and errors,
 * but the call allocates nothing.  The FP64 column-statistics partials of
 * SUGG_FIT_STATS (2 x E x min(1024, ceil(N / 256)) doubles) live in a static
 * device array of SUGG_NOALLOC_SCRATCH_BYTES that the library holds on every
 * GPU it runs on until the process ends (its address is looked up by
 * sugg_create); a plan whose partials would not fit is rejected with
 * SUGG_E_BUDGET (never the case within SUGG_MAX_EVENTS).  With
 * SUGG_FIT_STATS the context's model storage must already hold the plan's E
 * columns (one earlier sugg_load_features, sugg_fit or sugg_model_set of
 * that E), else SUGG_E_STATE.  Every call on one GPU shares that GPU's
 * array and the array keeps the last call's partials: calls that overlap in
 * time on one GPU (from any context or stream) race. */
#define SUGG_NOALLOC_SCRATCH_BYTES (4 << 20)
SUGG_API int32_t sugg_load_features_noalloc(sugg_ctx* ctx, const sugg_plan* plan, const void* counters,
                                            const void* cycles, int32_t mode, void* z_out, hipStream_t stream);

/* Tier 2 training (Section 2; Sections 3.3-3.4): column statistics from the
 * training rows, then for every global optimisation o with at least one
 * before/after pair (version S without o, the same kernel's version S with o)
 * a ridge regression of ln cyc(before) - ln cyc(after) on [z(before), 1]:
 *   (X^T X + lambda diag(1,..,1,0)) w_o = X^T y,
 * accumulated and solved by Cholesky in FP64.  Replaces the model. */
SUGG_API int32_t sugg_fit(sugg_ctx* ctx, const sugg_plan* train, const void* counters,
                          const void* cycles, hipStream_t stream);

/* Tier 2 prediction.  Every global id used by the plan must be trained
 * (else SUGG_E_UNTRAINED_OPT).
 * grid_out (nullable): N x Bmax (Bmax = sugg_plan_max_opts), plan dtype;
 *   grid[row(k,S)][b] = w_{O_k[b]} . [z, 1] for b < B_k not in S, NaN for
 *   b in S or b >= B_k: the predicted log-speedup of adding optimisation b.
 * table_out (required): N, plan dtype; table[row(k,S)] = sum over the bits b
 *   of S, ascending, of the prediction for adding b to version S & (2^b - 1)
 *   (the composed log-speedup of applying subset S; table[row(k,0)] = 0). */
SUGG_API int32_t sugg_predict(sugg_ctx* ctx, const sugg_plan* plan, const void* counters,
                              const void* cycles, void* grid_out, void* table_out, hipStream_t stream);

/* Tier 3 (Section 2) over arbitrary segments: segment i is
 * scores[seg_off[i] .. seg_off[i+1]) (device int64 offsets, non-decreasing);
 * its first skip_head entries are never candidates.  Keeps entries with
 * score > tau (NaN never), sorts by score descending then index ascending,
 * writes the first n: idx_out[i*n + j] = index within the segment (-1 pad),
 * score_out[i*n + j] (NaN pad), count_out[i] = number kept (<= n).
 * 1 <= n <= SUGG_MAX_SUGGEST.  scores and score_out are of dtype. */
SUGG_API int32_t sugg_rank_suggest(sugg_ctx* ctx, int32_t dtype, const void* scores,
                                   const int64_t* seg_off, int32_t nseg, int32_t skip_head,
                                   int32_t n, double tau, int32_t* idx_out, void* score_out,
                                   int32_t* count_out, hipStream_t stream);

/* The fused scoring path: sugg_predict's table plus, per kernel k, the top
 * n_suggest subsets S >= 1 with table > tau (context parameters), in one
 * persistent kernel.  table_out (nullable) as in sugg_predict; idx_out[K*n]
 * holds subset bitmasks S, score_out[K*n] their composed log-speedups,
 * count_out[K]; padding as in sugg_rank_suggest. */
SUGG_API int32_t sugg_suggest(sugg_ctx* ctx, const sugg_plan* plan, const void* counters,
                              const void* cycles, void* table_out, int32_t* idx_out,
                              void* score_out, int32_t* count_out, hipStream_t stream);

/* sugg_suggest restricted to the kernels with kmask[k] != 0 (device int32
 * [K]): only their rows are read and only their table entries and
 * suggestion lists are written; the other kernels' outputs are left as they
 * are.  Used to re-score kernels whose learned-surrogate answer was rejected. */
SUGG_API int32_t sugg_suggest_subset(sugg_ctx* ctx, const sugg_plan* plan, const void* counters,
                                     const void* cycles, const int32_t* kmask, void* table_out,
                                     int32_t* idx_out, void* score_out, int32_t* count_out, hipStream_t stream);

/* Judge: the plain composed log-speedup (sugg_predict's table value) of C
 * given subsets per kernel, reading only the versions on each subset's
 * ascending chain (popcount(S) rows).  cand [K x C] device int32 subset
 * bitmasks (< 0: none); out [K x C] plan dtype: the table value, bit-identical
 * to sugg_predict's; 0 for S = 0; NaN for none or S >= 2^B_k.  1 <= C <= 64.
 * With ref [K x C] (e.g. a learned surrogate's values of the same subsets)
 * and flag_out [K] (both device, or both null): flag_out[k] = 1 when some
 * candidate S >= 1 of kernel k has |ref - out| > tol (or a non-finite
 * difference), else 0; with accumulate != 0 a flag already set stays set
 * (flag_out is not cleared first), so several calls can judge one kernel. */
SUGG_API int32_t sugg_judge(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles,
                            const int32_t* cand, int32_t C, void* out, const void* ref, double tol,
                            int32_t* flag_out, int32_t accumulate, hipStream_t stream);

/* Threshold band of short suggestion lists, for judging a learned
 * surrogate's decisions at the Tier 3 threshold (Section 2: candidates are
 * kept only above a preset threshold).  Per segment i (scores[seg_off[i] ..
 * seg_off[i+1]), entries below skip_head excluded) whose list from
 * sugg_rank_suggest (top_idx [nseg x n], top_count [nseg]) holds fewer than n
 * entries: the other entries p with scores[p] >= tau - band (compared in
 * FP64), ascending, into cand_out [nseg x C] (int32, -1 padding) with their
 * scores in ref_out [nseg x C] (dtype, NaN padding); flag_out[i] = 1 when
 * more than C qualified, else 0.  A full list (n entries) has an empty band.
 * All pointers device; 1 <= n <= SUGG_MAX_SUGGEST, 1 <= C <= 64, band >= 0. */
SUGG_API int32_t sugg_band_select(sugg_ctx* ctx, int32_t dtype, const void* scores, const int64_t* seg_off,
                                  int32_t nseg, int32_t skip_head, const int32_t* top_idx,
                                  const int32_t* top_count, int32_t n, double tau, double band, int32_t C,
                                  int32_t* cand_out, void* ref_out, int32_t* flag_out, hipStream_t stream);

/* All-paths composition (an estimator of a subset's speedup that does not
 * depend on the order of adding its optimisations; the paper predicts one
 * optimisation at a time, Section 2, and leaves subsets open):
 *   L(0) = 0,  L(S) = (sum over b in S, ascending, of [L(S-b) + P(S-b, b)]) / |S|,
 * the mean over every order of S of the linear model's predictions added
 * along it.  table_out [N] (required) and, with idx_out, the top
 * n_suggest subsets above tau per kernel as in sugg_suggest.  B_k <= 10
 * (SUGG_E_SHAPE otherwise). */
SUGG_API int32_t sugg_predict_allpaths(sugg_ctx* ctx, const sugg_plan* plan, const void* counters,
                                       const void* cycles, void* table_out, int32_t* idx_out, void* score_out,
                                       int32_t* count_out, hipStream_t stream);

/* Greedy re-profiling (the tool used iteratively, Section 2: apply the best
 * suggestion, profile the new version, ask again), on kernels whose every
 * version is profiled: from S = 0, while some b not in S has a predicted
 * benefit P(S, b) > tau, take the largest (ties: the smaller b) and continue
 * from row(k, S + b).  path_out [K x (Bmax+1)] int32: the visited versions
 * starting with 0, -1 after the last; steps_out [K]: optimisations applied;
 * gain_out [K] (plan dtype): sum of the predicted benefits of the steps. */
SUGG_API int32_t sugg_greedy(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles,
                             int32_t* path_out, int32_t* steps_out, void* gain_out, hipStream_t stream);

/* The surrogate's suggestions for a batch whose kernels all have one B
 * (FP32 plan; mlp frozen, in = E, out = 2^B, max batch >= K): Tier 1 of each
 * kernel's baseline version (version 0) with the fitted model's column
 * statistics, rounded to BF16 as the network's input, the network, and
 * Tier 3 over each kernel's subsets S >= 1 (n and tau of the context) as in
 * sugg_mlp_infer_rank; table_out (nullable) [K x 2^B] receives the
 * network's whole table.  idx_out [K x n] holds subsets S (bitmasks of the
 * kernel's local optimisation bits), as sugg_suggest.  Same lists as
 * sugg_load_features (baseline rows) + sugg_mlp_infer_rank (skip 1).  A bad
 * baseline counter is reported by the next sugg_sync. */
SUGG_API int32_t sugg_surrogate_suggest(sugg_ctx* ctx, const sugg_plan* plan, sugg_mlp* mlp, const void* counters,
                                        const void* cycles, void* table_out, int32_t* idx_out, void* score_out,
                                        int32_t* count_out, hipStream_t stream);

/* One serving query, every step enqueued on the stream (no host wait): for
 * a plan whose K kernels all have B optimisations (FP32), a frozen surrogate
 * mapping E features to 2^B log-speedups (K <= its max batch):
 *   1. each kernel's standardised baseline row (Tier 1, as sugg_load_features
 *      with SUGG_BASELINE, rounded to BF16 into the network's input), 2. the
 *      surrogate's table, 3. its top n_suggest above tau (in the output
 *      layer's epilogue where 2^B is 64 or 128), 4. the threshold band of short lists (sugg_band_select, at
 *      most cap subsets), 5. the judge of the listed and band subsets
 *      against the plain composed values, 6. Tier 3's threshold checked on
 *      the plain values (every listed subset above tau, no band subset
 *      above tau), 7. the plain fused path for the kernels flagged
 *      (difference above tol, band overflow, or a threshold breach).
 * idx_out [K x n] / score_out [K x n] / count_out [K]: the answer (subsets of
 * the surrogate's list with their plain values, sorted by them: descending,
 * equal values by smaller subset - Tier 3's ranking of the plain values over
 * the judged subsets - or the plain answer where flagged); flag_out [K]: 1
 * where the plain path answered.  A learned
 * surrogate is an extension of the paper's Tier 2, which stays the judge.
 * The plan keeps a workspace for its queries (allocated on its first call,
 * not inside a graph capture). */
SUGG_API int32_t sugg_serve_query(sugg_ctx* ctx, const sugg_plan* plan, sugg_mlp* mlp, const void* counters,
                                  const void* cycles, double tol, double band, int32_t cap, int32_t* idx_out,
                                  void* score_out, int32_t* count_out, int32_t* flag_out, hipStream_t stream);

/* Waits for the stream, then returns and clears the device status word:
 * SUGG_E_BAD_COUNTER or SUGG_E_SINGULAR if a kernel flagged one since the
 * last sync, else SUGG_OK. */
SUGG_API int32_t sugg_sync(sugg_ctx* ctx, hipStream_t stream);

/* Graph capture of scoring passes (Tiers 1-3 of Section 2 replayed without
 * per-launch host work).  Between sugg_capture_begin and sugg_capture_end on
 * a non-default stream, sugg_predict / sugg_suggest / sugg_rank_suggest calls
 * on that stream are recorded instead of run; the graph then replays them
 * with sugg_graph_launch on any stream of the device.  The recorded calls
 * keep their pointers: inputs are read and outputs written in place at every
 * replay.  The scoring kernels re-arm their work counters themselves, so a
 * graph holds kernel nodes only.  A plan must not run in two launches that
 * overlap in time (they share its work counter). */
SUGG_API int32_t sugg_capture_begin(sugg_ctx* ctx, hipStream_t stream);
SUGG_API int32_t sugg_capture_end(sugg_ctx* ctx, hipStream_t stream, sugg_graph** out);
SUGG_API int32_t sugg_graph_launch(sugg_ctx* ctx, sugg_graph* graph, hipStream_t stream);
SUGG_API void sugg_graph_destroy(sugg_graph* graph);

/* ---- Instance-based Tier 2 model (IBK) ---------------------------------------
 * Section 3.4's instance-based learner, the one the paper adopts (Section 6;
 * its results use k = 10): every before/after pair of an optimisation in the
 * training kernels is stored (the before version's standardised feature
 * vector and the measured log-speedup of adding it), and a prediction is
 * the mean label of the k stored vectors nearest in Euclidean distance (the
 * paper's "mode" of real-valued labels read as their mean; equal distances:
 * the earlier stored sample, samples stored kernel by kernel, then by
 * version).  The IBK model lives beside the linear one in the context.
 * E <= 256.  Candidate distances are evaluated in FP32, the final ones in
 * FP64, labels averaged in FP64.
 *
 * sugg_ibk_fit: column statistics of the training rows (as sugg_load_features
 *   FIT_STATS, kept with the IBK model), their standardised vectors, and the
 *   sample database of every global id; 1 <= k <= 16.  Synchronous (the
 *   database is built on the host from the plan and uploaded); replaces a
 *   previous IBK model.
 * sugg_ibk_counts: samples stored per global id into counts[0..D) (host).
 * sugg_ibk_predict / sugg_ibk_suggest: as sugg_predict / sugg_suggest with
 *   the IBK model for Tier 2 (table_out, grid_out, idx_out, score_out,
 *   count_out with the same layouts); every id of the plan needs samples
 *   (else SUGG_E_UNTRAINED_OPT).  A plan's first IBK call per output form
 *   (with or without the grid) builds and uploads its query lists and
 *   allocates its workspace (not inside a graph capture); later calls only
 *   enqueue kernels.
 *   The neighbours are exact: the FP32 search keeps k plus a margin of
 *   candidates (at least 6), which are re-ranked by FP64 distance between
 *   FP64 standardised features; where a bound on the FP32 error cannot
 *   certify that the k nearest are among them, the query is searched again
 *   over all its samples in FP64 (sugg_ibk_exact_count reports how many were,
 *   in the plan's last IBK call; synchronous). */
SUGG_API int32_t sugg_ibk_fit(sugg_ctx* ctx, const sugg_plan* train, const void* counters, const void* cycles,
                              int32_t k, hipStream_t stream);
SUGG_API int32_t sugg_ibk_counts(sugg_ctx* ctx, int64_t* counts, int32_t D);
SUGG_API int32_t sugg_ibk_exact_count(sugg_ctx* ctx, const sugg_plan* plan, int64_t* n);
SUGG_API int32_t sugg_ibk_predict(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles,
                                  void* grid_out, void* table_out, hipStream_t stream);
SUGG_API int32_t sugg_ibk_suggest(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles,
                                  void* table_out, int32_t* idx_out, void* score_out, int32_t* count_out,
                                  hipStream_t stream);

/* ---- Model-tree Tier 2 model (M5P) ------------------------------------------
 * Section 3.4's model tree, after Quinlan's M5: per global id a regression
 * tree over the standardised Tier 1 features of the before versions, grown
 * by standard-deviation reduction (binary splits z_j <= t, t halfway between
 * adjacent distinct training values; no split of a node with fewer than
 * 2 * min_leaf pairs or with label sd at most 5 % of the root's; each side
 * keeps min_leaf pairs); least-squares linear models with an intercept at
 * every node on the features tested in its subtree (in feature order, a
 * feature whose centred column lies within 1e-9 of the span of those kept
 * before it is left out, so collinear counters give a unique model);
 * bottom-up pruning by the M5 error estimate (mean |residual| * (n + v) /
 * (n - v), v kept parameters); smoothing from
 * the leaf up, p <- (n_c p + smooth_k q) / (n_c + smooth_k), folded into one
 * linear model per leaf.  Ties: split gains within 1e-9 of the root's label
 * sd are equal (first feature, then lowest threshold wins); a pruning
 * comparison within the same margin prunes.  The M5P model lives beside the
 * linear and IBK models in the context.  E <= 256.
 *
 * sugg_m5p_fit: FP64 column statistics and standardised features of the
 *   training rows on the GPU, then the trees on the host (one thread per id,
 *   up to 16), uploaded.  Synchronous; replaces a previous M5P model.
 *   min_leaf >= 1 (the paper's tool, Weka's M5P, uses 4), smooth_k >= 0 (15;
 *   0 disables smoothing).  SUGG_E_BAD_COUNTER if a training counter or
 *   cycle count is not positive and finite; SUGG_E_BUDGET above 2^20 pairs
 *   per id or 8 GiB of FP64 training features (N x E x 8 bytes).  Trees are
 *   induced in as many host threads as 16 GiB of sort buffers allow.
 * sugg_m5p_tree: the pruned tree of global id opt, preorder (a node, its left
 *   subtree, its right subtree), into host arrays of cap entries: feat (-1 at
 *   a leaf), thr (go left when z[feat] <= thr; NaN at a leaf), left and right
 *   child (-1 at a leaf), count (training pairs reaching the node);
 *   *n_nodes receives the node count (call with cap = 0 to size the arrays).
 * sugg_m5p_predict / sugg_m5p_suggest: as sugg_predict / sugg_suggest with
 *   the M5P model for Tier 2 (same layouts); every id of the plan needs a
 *   tree (else SUGG_E_UNTRAINED_OPT).  Tests compare in the plan dtype: FP32
 *   plans walk the trees on FP32 features.  A plan's first M5P call builds
 *   its row tiles and workspace (not inside a graph capture). */
SUGG_API int32_t sugg_m5p_fit(sugg_ctx* ctx, const sugg_plan* train, const void* counters, const void* cycles,
                              int32_t min_leaf, double smooth_k, hipStream_t stream);
SUGG_API int32_t sugg_m5p_tree(sugg_ctx* ctx, int32_t opt, int32_t cap, int32_t* feat, double* thr, int32_t* left,
                               int32_t* right, int64_t* count, int32_t* n_nodes);
SUGG_API int32_t sugg_m5p_predict(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles,
                                  void* grid_out, void* table_out, hipStream_t stream);
SUGG_API int32_t sugg_m5p_suggest(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles,
                                  void* table_out, int32_t* idx_out, void* score_out, int32_t* count_out,
                                  hipStream_t stream);

/* M5P model checkpoint (host arrays, synchronous).
 * sugg_m5p_shape: E and D of the context's M5P model (SUGG_E_STATE if none).
 * sugg_m5p_export: node_off and leaf_off [D+1] always (id o's nodes are
 *   [node_off[o], node_off[o+1]) of the concatenated arrays, its leaf models
 *   [leaf_off[o], leaf_off[o+1]); no nodes = untrained); with
 *   nodes_cap = leaves_cap = 0 nothing else (sizing), otherwise, for caps of
 *   at least node_off[D] and leaf_off[D]: each id's preorder tree as in
 *   sugg_m5p_tree (child indices within the id's tree) plus leaf (the node's
 *   leaf model ordinal within the id, -1 inside), lw [leaves x (E+1)] (the
 *   smoothed leaf models, intercept last), and mu, isg [E] (the FP64 mean and
 *   reciprocal standard deviation of ln(c / cyc) that standardise features).
 * sugg_m5p_import: replaces the context's M5P model with such arrays, which
 *   predict exactly as the exported model did.  Checked: every tree rooted at
 *   node 0 with each other node the child of exactly one earlier node, splits
 *   on features < E at finite thresholds, each leaf model used by exactly one
 *   leaf, finite leaf models and statistics (SUGG_E_ARG otherwise; the
 *   previous model is kept). */
SUGG_API int32_t sugg_m5p_shape(const sugg_ctx* ctx, int32_t* E, int32_t* D);
SUGG_API int32_t sugg_m5p_export(sugg_ctx* ctx, int64_t nodes_cap, int64_t leaves_cap, int64_t* node_off,
                                 int64_t* leaf_off, int32_t* feat, double* thr, int32_t* left, int32_t* right,
                                 int32_t* leaf, int64_t* count, double* lw, double* mu, double* isg);
SUGG_API int32_t sugg_m5p_import(sugg_ctx* ctx, int32_t E, int32_t D, const int64_t* node_off,
                                 const int64_t* leaf_off, const int32_t* feat, const double* thr,
                                 const int32_t* left, const int32_t* right, const int32_t* leaf,
                                 const int64_t* count, const double* lw, const double* mu, const double* isg);

/* ---- Learned surrogate ------------------------------------------------------
 * An extension of the paper's Tier 2 (which predicts one optimisation at a
 * time): an MLP in -> hidden -> hidden -> out with exact-erf GELU after both
 * hidden layers, mapping a kernel's standardised baseline counter vector to
 * the composed log-speedups of all its 2^B optimisation subsets, trained on
 * tables from sugg_predict.  BF16 weights and activations, FP32 accumulation
 * on the matrix cores, FP32 master weights.
 *
 * Parameters live in one caller-owned FP32 device buffer of
 * sugg_mlp_param_count() floats: W1 [hidden x in], b1 [hidden],
 * W2 [hidden x hidden], b2 [hidden], W3 [out x hidden], b3 [out] (row-major,
 * weight rows are output units).  Gradients and Adam moments use the same
 * layout.  x is [batch x in], y and targets [batch x out], FP32 row-major,
 * device memory.  Widths must be multiples of 8 in [8, 4096]; batch <=
 * max_batch.  The object owns the BF16 working copies and the activations
 * kept for the backward; calls on one object must not overlap. */
SUGG_API int32_t sugg_mlp_create(sugg_ctx* ctx, int32_t in, int32_t hidden, int32_t out, int32_t max_batch,
                                 sugg_mlp** out_mlp);
SUGG_API void sugg_mlp_destroy(sugg_mlp* mlp);
SUGG_API int64_t sugg_mlp_param_count(const sugg_mlp* mlp);
/* The matrix-core kernel instances the object's last forward and backward
 * launched, host array info [8 x 4]: rows are the forward's layers 1-3, then
 * the backward's dW3, dA2, dW2, dA1, dW1 products; columns are workgroup tile
 * rows, tile columns, K splits, and the K stage (32, 64 or 128) of the
 * variant without bounds checks where that ran, 0 where the variant with
 * bounds checks ran (all zeros for a product not launched yet).  Lets a
 * caller (a test) see which instances a given batch size exercises. */
SUGG_API int32_t sugg_mlp_launch_info(const sugg_mlp* mlp, int32_t* info);
/* Keeps a copy of params for inference (sugg_serve_query): the BF16 working
 * weights are packed from it once, and again only after another call
 * packed other parameters. */
SUGG_API int32_t sugg_mlp_freeze(sugg_ctx* ctx, sugg_mlp* mlp, const float* params, hipStream_t stream);
/* y = MLP(x); keep != 0 saves what sugg_mlp_backward needs. */
SUGG_API int32_t sugg_mlp_forward(sugg_ctx* ctx, sugg_mlp* mlp, const float* params, const float* x, int32_t batch,
                                  float* y, int32_t keep, hipStream_t stream);
/* Forward with targets: loss (device scalar) = mean over batch and outputs of
 * (y - target)^2; keeps activations and dY = 2 (y - target) / (batch * out).
 * y is nullable. */
SUGG_API int32_t sugg_mlp_loss(sugg_ctx* ctx, sugg_mlp* mlp, const float* params, const float* x,
                               const float* target, int32_t batch, float* y, float* loss, hipStream_t stream);
/* Hand-written backward of the last keeping forward of this batch: grads of
 * every parameter for the output gradient dy [batch x out] (nullable: the dY
 * left by sugg_mlp_loss).  Errors with SUGG_E_STATE without such a forward. */
SUGG_API int32_t sugg_mlp_backward(sugg_ctx* ctx, sugg_mlp* mlp, const float* params, const float* dy, int32_t batch,
                                   float* grads, hipStream_t stream);
/* Adam (Kingma and Ba) with bias correction at step >= 1, in place on params,
 * m and v. */
SUGG_API int32_t sugg_mlp_adam(sugg_ctx* ctx, sugg_mlp* mlp, float* params, const float* grads, float* m, float* v,
                               int32_t step, float lr, float beta1, float beta2, float eps, hipStream_t stream);
/* sugg_mlp_loss + sugg_mlp_backward + sugg_mlp_adam (beta 0.9 / 0.999,
 * eps 1e-8); grads is the caller's gradient buffer. */
SUGG_API int32_t sugg_mlp_train_step(sugg_ctx* ctx, sugg_mlp* mlp, float* params, float* grads, float* m, float* v,
                                     int32_t step, float lr, const float* x, const float* target, int32_t batch,
                                     float* loss, hipStream_t stream);

/* A training epoch in one call: for s in [0, steps), the mini-batch of rows
 * perm[s*batch .. (s+1)*batch) of X [n_rows x in] with targets the same rows
 * of Y [n_rows x out] (gathered by the first kernel, no copies), then what
 * sugg_mlp_train_step does with Adam step step0 + s + 1; loss of step s into
 * losses[s] (device).  Seven launches a step: three forward GEMMs, two
 * launches that each pair a weight gradient with the backward through that
 * layer, the first layer's weight gradient, one launch that finishes all
 * three weight and bias gradients and the loss, and Adam (which also
 * rewrites the BF16 working weights) together with the gather of the next
 * mini-batch (the first gather is a launch of its own).  Bit-identical to
 * train_step on the gathered batches.  perm is a
 * device int32 array of steps*batch entries; an entry outside [0, n_rows)
 * reads row 0 and the next sugg_sync reports SUGG_E_ARG.  Asynchronous. */
/* Inference with the frozen parameters (sugg_mlp_freeze; SUGG_E_STATE
 * without): y [batch x out] for x [batch x in], as sugg_mlp_forward without
 * kept activations; the working weights are packed once per freeze. */
SUGG_API int32_t sugg_mlp_infer(sugg_ctx* ctx, sugg_mlp* mlp, const float* x, int32_t batch, float* y,
                                hipStream_t stream);
/* Inference with the frozen parameters and Tier 3 on every row of the
 * output (Section 2: the best n choices above the threshold, by expected
 * benefit): idx [batch x n] the output columns >= skip whose value exceeds
 * tau, by value descending then column ascending, -1 padded; score the
 * values (NaN padded); count [batch] how many.  Identical to sugg_mlp_infer
 * then sugg_rank_suggest over rows of out values (skip_head = skip).  For
 * out = 64 or 128 the output layer ranks in its epilogue (the outputs never
 * leave the chip unless y, nullable, asks for them).  1 <= n <= 8,
 * 0 <= skip < out. */
SUGG_API int32_t sugg_mlp_infer_rank(sugg_ctx* ctx, sugg_mlp* mlp, const float* x, int32_t batch, int32_t skip,
                                     int32_t n, float tau, float* y, int32_t* idx, float* score, int32_t* count,
                                     hipStream_t stream);

SUGG_API int32_t sugg_mlp_train_epoch(sugg_ctx* ctx, sugg_mlp* mlp, float* params, float* grads, float* m,
                                      float* v, int32_t step0, float lr, const float* X, const float* Y,
                                      int64_t n_rows, const int32_t* perm, int32_t batch, int32_t steps,
                                      float* losses, hipStream_t stream);

/* Model checkpoint (host arrays, synchronous).  W is D x (E+1), row o =
 * feature weights of optimisation o followed by its intercept; counts[o] is
 * its number of training pairs (0 = untrained). */
SUGG_API int32_t sugg_model_shape(const sugg_ctx* ctx, int32_t* E, int32_t* D);
SUGG_API int32_t sugg_model_get(sugg_ctx* ctx, double* mu, double* sigma, double* W, int64_t* counts);
SUGG_API int32_t sugg_model_set(sugg_ctx* ctx, int32_t E, int32_t D, const double* mu,
                                const double* sigma, const double* W, const int64_t* counts);

#ifdef __cplusplus
}
#endif
#endif /* SUGG_H */
