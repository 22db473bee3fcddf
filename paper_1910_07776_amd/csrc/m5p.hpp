// Internal: the model-tree Tier 2 learner (M5P, Section 3.4, after Quinlan's
// M5): per optimisation a regression tree grown by standard-deviation
// reduction, linear models at the nodes on the features tested below them,
// pruned bottom-up by the M5 error estimate and smoothed towards the root.
//
// The tree is induced on the host from FP64 features computed on the GPU; a
// prediction walks it on the GPU and evaluates one linear model per leaf,
// into which the smoothing along the leaf's path has been folded (a chain of
// convex combinations of linear models is a linear model).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace sugg {

// One optimisation's pruned tree on the host, in preorder (a node, then its
// left subtree, then its right subtree).
struct M5pHostTree {
  std::vector<int32_t> feat;    // tested feature; -1 at a leaf
  std::vector<double> thr;      // go left when z[feat] <= thr
  std::vector<int32_t> left, right;   // child nodes; -1 at a leaf
  std::vector<int32_t> leaf;    // leaf ordinal at a leaf, -1 inside
  std::vector<int64_t> count;   // training cases reaching the node
  std::vector<double> lw;       // [leaves, E + 1]: smoothed leaf models, intercept last
  int leaves = 0;
  int depth = 0;                // longest root-to-leaf path (edges)
};

struct M5pParams {
  int min_leaf = 4;             // fewest training cases on each side of a split
  double sd_frac = 0.05;        // no split below this fraction of the root's label sd
  double smooth_k = 15.0;       // smoothing constant
  double tie = 1e-9;            // ties, relative to the root's label sd
};

// Induce one tree.  Z: FP64 standardised rows with row stride ldz; rows[i]:
// the row of training case i; y[i]: its label.  Cases are numbered in the
// order given (ties between equal feature values follow it).
M5pHostTree m5p_induce(const double* Z, int64_t ldz, const int32_t* rows, const double* y, int64_t n, int E,
                       const M5pParams& prm);

// Device form of a tree: blocks of three levels in one 128-byte line, so one
// load decides three tests of a walk.  Positions 0..6 hold a node and its
// descendants down two levels (children of position p at 2p+1, 2p+2); a
// leaf position has feat = -1 and its leaf ordinal in thr's bits.  The eight
// exits below positions 3..6 name the next block (>= 0) or a leaf (-1 - id).
template <typename T>
struct alignas(128) M5pBlock {
  int16_t feat[8];
  int32_t exit[8];
  T thr[8];
};

// Device form of a fitted model: every optimisation's tree concatenated.
// Predictions are formed in FP64 whatever the plan's dtype (features from the
// counters, the walk's tests, the leaf models), so a walk takes the branch
// the FP64 reference takes.
struct M5pModel {
  int E = 0, D = 0, ldl = 0;
  M5pParams prm;
  std::vector<M5pHostTree> trees;     // per global id (empty when untrained)
  std::vector<int32_t> root;          // per global id: first block, -1 when untrained
  int32_t* d_root = nullptr;
  M5pBlock<double>* blk64 = nullptr;
  int max_blocks = 0;                 // longest chain of blocks of a walk
  double* lw64 = nullptr;             // [leaves, ldl], columns >= E zero
  double* lb64 = nullptr;             // [leaves] intercepts
  double *mu64 = nullptr, *isg64 = nullptr;   // column constants for the features
};

struct M5pPlan {
  int32_t* tiles = nullptr;           // [n_tiles, 2]: kernel, first version
  int n_tiles = 0;
  void* edges = nullptr;              // [N] plan dtype
};

// TI: the plan's dtype (counters, cycles, outputs); arithmetic in FP64.
template <typename TI>
struct M5pArgs {
  const TI* counters;
  const TI* cycles;
  const int64_t* row_off;
  const int32_t* nopts;
  const int64_t* opt_off;
  const int32_t* opt_ids;
  const int32_t* tiles;
  const double* mu;
  const double* isg;
  const int32_t* root;
  const M5pBlock<double>* blocks;
  const double* lw;
  const double* lb;
  int32_t ldl;
  int32_t max_blocks;
  int32_t E;
  int32_t Bmax;
  TI* grid;       // grid mode when non-null: every b not in S
  double* edges;  // else chain edges: e[row(k, S | 2^b)] for b above the top bit of S
  int32_t* status;
};

constexpr int kM5pRows = 16;          // versions per workgroup (16 lanes each)

template <typename TI>
hipError_t launch_m5p(const M5pArgs<TI>& a, int n_tiles, hipStream_t s);
// Kernels of at most 64 versions, chain edges only: the whole pass (edges,
// composition, top-n) in one launch, one workgroup per kernel.
constexpr int kM5pSmallB = 6;
template <typename TI>
hipError_t launch_m5p_small(const M5pArgs<TI>& a, int K, TI* table, int32_t* idx, TI* score, int32_t* count, int n,
                            double tau, hipStream_t s);

}  // namespace sugg

using sugg::M5pModel;
using sugg::M5pPlan;

void m5p_model_free(M5pModel*& m);
void m5p_plan_free(M5pPlan*& p);
