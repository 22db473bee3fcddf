// Prediction with M5P model trees (Section 3.4): per version row, Tier 1's
// standardised features, then for every optimisation the row needs a walk
// down that optimisation's tree and the leaf's smoothed linear model.
//
// A workgroup takes 16 versions of one kernel.  Sixteen lanes share a row
// (16-byte loads, the row arithmetic of the fused scoring kernel) and leave
// its features in LDS.  The tile's predictions are then walked one per
// thread, all at once (a walk is a chain of dependent loads, so the tile's
// critical path is one walk, not a row's several), and the leaf models are
// evaluated sixteen lanes per prediction with a DPP reduction.  Edge mode
// forms the predictions of the ascending chain only (row S predicts adding
// each b above its top bit: the one edge into every version S | 2^b); grid
// mode every b not in S.  Counters are read in the plan's dtype TI and every
// step computes in FP64 (features, tests, leaf models), so each walk takes
// the branch of the FP64 reference and FP32 plans differ from it only by the
// rounding of their outputs.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "m5p.hpp"
#include "path_impl.hpp"

namespace sugg {

constexpr int kM5pThreads = kM5pRows * kRowLanes;

// Lane l16's chunks of a row, columns (l16 + 16 ch) * VW + [0, VW), read in
// the plan dtype and widened to FP64 (1 past E).
template <typename TI, int NCH, int VW>
__device__ __forceinline__ void m5p_load_row(const TI* rp, int E, int l16, double (&c)[NCH][VW]) {
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int c0 = (l16 + kRowLanes * ch) * VW;
    if (c0 + VW <= E) {
      const VecN<TI, VW> q = *reinterpret_cast<const VecN<TI, VW>*>(rp + c0);
#pragma unroll
      for (int v = 0; v < VW; ++v) c[ch][v] = (double)q.v[v];
    } else {
#pragma unroll
      for (int v = 0; v < VW; ++v) c[ch][v] = c0 + v < E ? (double)rp[c0 + v] : 1.0;
    }
  }
}

// Selections among a block's slots with constant indices (no dynamic
// indexing of register arrays).
template <typename V>
__device__ __forceinline__ V m5p_sel4(const V* v, int i) {
  const V lo = (i & 1) ? v[1] : v[0];
  const V hi = (i & 1) ? v[3] : v[2];
  return (i & 2) ? hi : lo;
}
template <typename V>
__device__ __forceinline__ V m5p_sel8(const V* v, int i) {
  const V lo = m5p_sel4(v, i & 3);
  const V hi = m5p_sel4(v + 4, i & 3);
  return (i & 4) ? hi : lo;
}
__device__ __forceinline__ int m5p_leaf_bits(float t) { return __float_as_int(t); }
__device__ __forceinline__ int m5p_leaf_bits(double t) { return (int)__double_as_longlong(t); }

// The leaf that a version with features zr (in LDS) reaches in the tree whose
// first block is blk.
template <typename T>
__device__ __forceinline__ int m5p_walk(const M5pBlock<T>* blocks, int blk, int max_blocks, const T* zr) {
  for (int it = 0; it < max_blocks; ++it) {   // a walk ends within max_blocks loads
    const M5pBlock<T> q = blocks[blk];         // three levels in one line
    int f = q.feat[0];
    T t = q.thr[0];
    if (f < 0) return m5p_leaf_bits(t);
    const int g0 = !(zr[f] <= t);
    f = g0 ? q.feat[2] : q.feat[1];
    t = g0 ? q.thr[2] : q.thr[1];
    if (f < 0) return m5p_leaf_bits(t);
    const int i2 = 2 * g0 + !(zr[f] <= t);
    f = m5p_sel4(q.feat + 3, i2);
    t = m5p_sel4(q.thr + 3, i2);
    if (f < 0) return m5p_leaf_bits(t);
    const int ex = m5p_sel8(q.exit, 2 * i2 + !(zr[f] <= t));
    if (ex < 0) return -1 - ex;
    blk = ex;
  }
  return 0;
}

// Predictions (edges) of the tile's row g = 0..15: edge mode every b above
// the top bit of S (all B bits for S = 0), grid mode every b not in S.
__device__ __forceinline__ int m5p_row_edges(int S, int B, bool grid) {
  if (S >= (1 << B)) return 0;
  return grid ? B - __popc((unsigned)S) : B - 1 - (S ? 31 - __clz(S) : -1);
}

template <typename TI, int VPL, int VW>
__global__ void __launch_bounds__(kM5pThreads) m5p_kernel(const M5pArgs<TI> a) {
  using T = double;
  constexpr int NCH = VPL / VW;
  constexpr int EP = kRowLanes * VPL;
  constexpr int kMaxEdges = kM5pRows * SUGG_MAX_OPTS;
  static_assert(kMaxEdges <= kM5pThreads, "one walk per thread");
  __shared__ __align__(32) T zl[kM5pRows][EP];
  __shared__ int32_t e_leaf[kMaxEdges];
  __shared__ int32_t e_gb[kMaxEdges];
  const int tid = threadIdx.x, g = tid / kRowLanes, l16 = tid % kRowLanes;
  const int k = a.tiles[2 * blockIdx.x];
  const int S0 = a.tiles[2 * blockIdx.x + 1];
  const int B = a.nopts[k];
  const int64_t r0 = a.row_off[k];
  const int32_t* ids = a.opt_ids + a.opt_off[k];
  const bool grid = a.grid != nullptr;
  // 1. rows: Tier 1 features of the 16 versions into LDS
  {
    const int S = S0 + g;
    const bool live = S < (1 << B);
    const int Sr = live ? S : S0;   // a dead row re-reads a live one and is not used
    T s_r[NCH][VW], m_r[NCH][VW];
    column_constants<T, NCH, VW, false>(a.mu, a.isg, a.E, l16, s_r, m_r);
    T c[NCH][VW];
    m5p_load_row<TI, NCH, VW>(a.counters + (r0 + Sr) * a.E, a.E, l16, c);
    T z[NCH][VW];
    const T chk = row_features<T, NCH, VW>(c, (T)a.cycles[r0 + Sr], s_r, m_r, z);
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      VecN<T, VW> q;
#pragma unroll
      for (int v = 0; v < VW; ++v) q.v[v] = z[ch][v];
      *reinterpret_cast<VecN<T, VW>*>(&zl[g][(l16 + kRowLanes * ch) * VW]) = q;
    }
    const bool bad = live && l16 == 0 && !__builtin_isfinite(chk);
    if (__ballot(bad) != 0 && (tid % kWave) == 0) atomicOr(a.status, (int)kStatusBadCounter);
  }
  __syncthreads();
  // 2. walks: one thread per prediction of the tile, down its tree to a leaf
  int n_e = 0;
#pragma unroll
  for (int r = 0; r < kM5pRows; ++r) n_e += m5p_row_edges(S0 + r, B, grid);
  if (tid < n_e) {
    int rem = tid, r = 0;
    for (; r < kM5pRows; ++r) {
      const int cnt = m5p_row_edges(S0 + r, B, grid);
      if (rem < cnt) break;
      rem -= cnt;
    }
    const int S = S0 + r;
    int b;
    if (grid) {
      b = 0;
      for (int seen = -1;; ++b)
        if (!((S >> b) & 1) && ++seen == rem) break;
    } else {
      b = (S ? 31 - __clz(S) : -1) + 1 + rem;
    }
    e_leaf[tid] = m5p_walk<T>(a.blocks, a.root[ids[b]], a.max_blocks, zl[r]);
    e_gb[tid] = (r << 8) | b;
  }
  __syncthreads();
  // 3. leaf models: sixteen lanes per prediction, the row's features from LDS
  for (int e = g; e < n_e; e += kM5pRows) {
    const int r = e_gb[e] >> 8, b = e_gb[e] & 255, leaf = e_leaf[e];
    const T* wrow = a.lw + (int64_t)leaf * a.ldl;
    T part = T(0);
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const int c0 = (l16 + kRowLanes * ch) * VW;
      const VecN<T, VW> zq = *reinterpret_cast<const VecN<T, VW>*>(&zl[r][c0]);
      const VecN<T, VW> w = *reinterpret_cast<const VecN<T, VW>*>(wrow + c0);
#pragma unroll
      for (int v = 0; v < VW; ++v) part = fma(zq.v[v], w.v[v], part);
    }
    const T p = row_sum16(part) + a.lb[leaf];
    if (l16 == 0) {
      const int S = S0 + r;
      if (grid) a.grid[(r0 + S) * a.Bmax + b] = (TI)p;
      // the chain edges in FP64 in both modes: the composition reads them
      if (!grid || b > (S ? 31 - __clz(S) : -1)) a.edges[r0 + (S | (1 << b))] = p;
    }
  }
}

// Small kernels (at most 64 versions), chain edges only: one workgroup per
// kernel.  Every row's features into LDS (four rows per 16-lane group, their
// loads in flight together), every chain edge walked at once (thread t takes
// version t + 1), the leaf models four per group with their weight rows in
// flight together, then Tier 3 in LDS: the composition level by level and
// the top-n of wave 0.  The arithmetic of an edge and of the composition is
// that of the tiled kernel and the separate composition, so both give the
// same bits.
template <typename TI, int VPL, int VW, int KT>
__global__ void __launch_bounds__(kM5pThreads) m5p_small_kernel(const M5pArgs<TI> a, TI* table, int32_t* idx_out,
                                                                TI* score_out, int32_t* count_out, int n, double tau) {
  using T = double;
  constexpr int NCH = VPL / VW;
  constexpr int EP = kRowLanes * VPL;
  constexpr int kRows = 64, kPer = kRows / kM5pRows;
  __shared__ __align__(32) T zl[kRows][EP];
  __shared__ T ev[kRows];
  __shared__ T L[kRows];
  __shared__ int32_t e_leaf[kRows];
  const int tid = threadIdx.x, g = tid / kRowLanes, l16 = tid % kRowLanes;
  const int k = blockIdx.x;
  const int B = a.nopts[k];
  const int V = 1 << B;
  const int64_t r0 = a.row_off[k];
  const int32_t* ids = a.opt_ids + a.opt_off[k];
  {
    T s_r[NCH][VW], m_r[NCH][VW];
    column_constants<T, NCH, VW, false>(a.mu, a.isg, a.E, l16, s_r, m_r);
    T c[kPer][NCH][VW], cy[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int S = g + kM5pRows * i;
      m5p_load_row<TI, NCH, VW>(a.counters + (r0 + (S < V ? S : 0)) * a.E, a.E, l16, c[i]);
      cy[i] = (T)a.cycles[r0 + (S < V ? S : 0)];
    }
    bool bad = false;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int S = g + kM5pRows * i;
      // rows past the kernel's versions are not read later; for V >= 4 the
      // test is uniform over a wave (its four groups hold rows 16 i + 4 w ..
      // 16 i + 4 w + 3), so those waves skip the logarithms
      if (S >= V) continue;
      T z[NCH][VW];
      const T chk = row_features<T, NCH, VW>(c[i], cy[i], s_r, m_r, z);
      bad |= l16 == 0 && !__builtin_isfinite(chk);
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        VecN<T, VW> q;
#pragma unroll
        for (int v = 0; v < VW; ++v) q.v[v] = z[ch][v];
        *reinterpret_cast<VecN<T, VW>*>(&zl[S][(l16 + kRowLanes * ch) * VW]) = q;
      }
    }
    if (__ballot(bad) != 0 && (tid % kWave) == 0) atomicOr(a.status, (int)kStatusBadCounter);
  }
  __syncthreads();
  if (tid + 1 < V) {
    const int Sp = tid + 1, top = 31 - __clz(Sp);
    const T* zr = zl[Sp - (1 << top)];
    e_leaf[tid] = m5p_walk<T>(a.blocks, a.root[ids[top]], a.max_blocks, zr);
  }
  __syncthreads();
  {
    const T* wrow[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e = g + kM5pRows * i;
      wrow[i] = a.lw + (int64_t)(e + 1 < V ? e_leaf[e] : 0) * a.ldl;
    }
    VecN<T, VW> w[kPer][NCH];
#pragma unroll
    for (int i = 0; i < kPer; ++i)
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
        w[i][ch] = *reinterpret_cast<const VecN<T, VW>*>(wrow[i] + (l16 + kRowLanes * ch) * VW);
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e = g + kM5pRows * i;
      if (e + 1 >= V) break;   // uniform per 16-lane group
      const int Sp = e + 1, top = 31 - __clz(Sp);
      const T* zr = zl[Sp - (1 << top)];
      T part = T(0);
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        const VecN<T, VW> zq = *reinterpret_cast<const VecN<T, VW>*>(zr + (l16 + kRowLanes * ch) * VW);
#pragma unroll
        for (int v = 0; v < VW; ++v) part = fma(zq.v[v], w[i][ch].v[v], part);
      }
      const T p = row_sum16(part) + a.lb[e_leaf[e]];
      if (l16 == 0) ev[Sp] = p;
    }
  }
  if (tid == 0) L[0] = T(0);
  __syncthreads();
  for (int b = 0; b < B; ++b) {
    const int lo = 1 << b;
    if (tid >= lo && tid < 2 * lo) L[tid] = L[tid - lo] + ev[tid];
    __syncthreads();
  }
  if (tid < kWave) {
    Entry<T> lst[KT];
#pragma unroll
    for (int i = 0; i < KT; ++i) lst[i] = empty_entry<T>();
    if (tid < V) {
      const T v = L[tid];
      if (table) table[r0 + tid] = (TI)v;
      if (tid != 0 && v > tau) {
        Entry<T> e;
        e.v = v;
        e.s = tid;
        list_insert<T, KT>(lst, e);
      }
    }
    if (idx_out) {
      group_merge<T, KT>(lst, kWave);
      if (tid == 0) {
        int cnt = 0;
#pragma unroll
        for (int i = 0; i < KT; ++i)
          if (i < n) {
            const bool ok = lst[i].s >= 0;
            idx_out[(int64_t)k * n + i] = ok ? lst[i].s : -1;
            score_out[(int64_t)k * n + i] = ok ? (TI)lst[i].v : qnan<TI>();
            cnt += ok ? 1 : 0;
          }
        count_out[k] = cnt;
      }
    }
  }
}

template <typename TI, int VPL>
hipError_t launch_m5p_vpl(const M5pArgs<TI>& a, int n_tiles, hipStream_t s) {
  constexpr int VEC = 16 / sizeof(TI);
  const bool vec = (a.E % VEC) == 0 && (reinterpret_cast<uintptr_t>(a.counters) % 16) == 0;
  (void)hipGetLastError();
  if (vec) hipLaunchKernelGGL((m5p_kernel<TI, VPL, VEC>), dim3(n_tiles), dim3(kM5pThreads), 0, s, a);
  else hipLaunchKernelGGL((m5p_kernel<TI, VPL, 1>), dim3(n_tiles), dim3(kM5pThreads), 0, s, a);
  return hipGetLastError();
}

template <typename TI, int VPL>
hipError_t launch_m5p_small_vpl(const M5pArgs<TI>& a, int K, TI* table, int32_t* idx, TI* score, int32_t* count,
                                int n, double tau, hipStream_t s) {
  constexpr int VEC = 16 / sizeof(TI);
  const bool vec = (a.E % VEC) == 0 && (reinterpret_cast<uintptr_t>(a.counters) % 16) == 0;
  (void)hipGetLastError();
  const dim3 grid(K), block(kM5pThreads);
  if (n <= 4) {
    if (vec) hipLaunchKernelGGL((m5p_small_kernel<TI, VPL, VEC, 4>), grid, block, 0, s, a, table, idx, score, count, n, tau);
    else hipLaunchKernelGGL((m5p_small_kernel<TI, VPL, 1, 4>), grid, block, 0, s, a, table, idx, score, count, n, tau);
  } else {
    if (vec) hipLaunchKernelGGL((m5p_small_kernel<TI, VPL, VEC, 8>), grid, block, 0, s, a, table, idx, score, count, n, tau);
    else hipLaunchKernelGGL((m5p_small_kernel<TI, VPL, 1, 8>), grid, block, 0, s, a, table, idx, score, count, n, tau);
  }
  return hipGetLastError();
}

template <typename TI>
hipError_t launch_m5p_small(const M5pArgs<TI>& a, int K, TI* table, int32_t* idx, TI* score, int32_t* count, int n,
                            double tau, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  if (a.E <= 16 * 4) return launch_m5p_small_vpl<TI, 4>(a, K, table, idx, score, count, n, tau, s);
  if (a.E <= 16 * 8) return launch_m5p_small_vpl<TI, 8>(a, K, table, idx, score, count, n, tau, s);
  return launch_m5p_small_vpl<TI, 16>(a, K, table, idx, score, count, n, tau, s);
}

template <typename TI>
hipError_t launch_m5p(const M5pArgs<TI>& a, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  if (a.E <= 16 * 4) return launch_m5p_vpl<TI, 4>(a, n_tiles, s);
  if (a.E <= 16 * 8) return launch_m5p_vpl<TI, 8>(a, n_tiles, s);
  return launch_m5p_vpl<TI, 16>(a, n_tiles, s);
}

template hipError_t launch_m5p<float>(const M5pArgs<float>&, int, hipStream_t);
template hipError_t launch_m5p<double>(const M5pArgs<double>&, int, hipStream_t);
template hipError_t launch_m5p_small<float>(const M5pArgs<float>&, int, float*, int32_t*, float*, int32_t*, int,
                                            double, hipStream_t);
template hipError_t launch_m5p_small<double>(const M5pArgs<double>&, int, double*, int32_t*, double*, int32_t*, int,
                                             double, hipStream_t);

}  // namespace sugg
