// Prediction with M5P model trees (Section 3.4): per version row, Tier 1's
// standardised features, then for every optimisation the row needs a walk
// down that optimisation's tree and the leaf's smoothed linear model.
//
// A workgroup takes 16 versions of one kernel; sixteen lanes share a row
// (16-byte loads, the row arithmetic of the fused scoring kernel), keep its
// features in registers for the leaf model's dot product and in LDS for the
// tree tests, which read one feature each.  Every lane of a row walks the
// tree (the same path), so the row's lanes stay converged for the dot
// product's DPP reduction.  Edge mode forms the predictions of the ascending
// chain only (row S predicts adding each b above its top bit: the one edge
// into every version S | 2^b); grid mode every b not in S.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "m5p.hpp"
#include "path_impl.hpp"

namespace sugg {

constexpr int kM5pThreads = kM5pRows * kRowLanes;

template <typename T, int NCH, int VW>
__device__ __forceinline__ void m5p_load_row(const T* rp, int E, int l16, T (&c)[NCH][VW]) {
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int c0 = (l16 + kRowLanes * ch) * VW;
    if (c0 + VW <= E) {
      const VecN<T, VW> q = *reinterpret_cast<const VecN<T, VW>*>(rp + c0);
#pragma unroll
      for (int v = 0; v < VW; ++v) c[ch][v] = q.v[v];
    } else {
#pragma unroll
      for (int v = 0; v < VW; ++v) c[ch][v] = c0 + v < E ? rp[c0 + v] : T(1);
    }
  }
}

template <typename T, int VPL, int VW>
__global__ void __launch_bounds__(kM5pThreads) m5p_kernel(const M5pArgs<T> a) {
  constexpr int NCH = VPL / VW;
  constexpr int EP = kRowLanes * VPL;
  __shared__ T zl[kM5pRows][EP];
  const int tid = threadIdx.x, g = tid / kRowLanes, l16 = tid % kRowLanes;
  const int k = a.tiles[2 * blockIdx.x];
  const int S0 = a.tiles[2 * blockIdx.x + 1];
  const int B = a.nopts[k];
  const int64_t r0 = a.row_off[k];
  const int32_t* ids = a.opt_ids + a.opt_off[k];
  const int S = S0 + g;
  const bool live = S < (1 << B);
  const int Sr = live ? S : S0;   // a dead row re-reads a live one and writes nothing
  T s_r[NCH][VW], m_r[NCH][VW];
  column_constants<T, NCH, VW, false>(a.mu, a.isg, a.E, l16, s_r, m_r);
  T c[NCH][VW];
  m5p_load_row<T, NCH, VW>(a.counters + (r0 + Sr) * a.E, a.E, l16, c);
  T z[NCH][VW];
  const T chk = row_features<T, NCH, VW>(c, a.cycles[r0 + Sr], s_r, m_r, z);
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
    for (int v = 0; v < VW; ++v) zl[g][(l16 + kRowLanes * ch) * VW + v] = z[ch][v];
  __syncthreads();
  if (live) {
    const int top = S ? 31 - __clz(S) : -1;
    for (int b = a.grid ? 0 : top + 1; b < B; ++b) {   // uniform per row
      if ((S >> b) & 1) continue;
      int node = a.root[ids[b]];
      M5pNode nd = a.nodes[node];
      for (int d = 0; d < a.max_depth && nd.feat >= 0; ++d) {
        node = zl[g][nd.feat] <= a.thr[node] ? nd.left : nd.right;
        nd = a.nodes[node];
      }
      const int leaf = nd.leaf >= 0 ? nd.leaf : 0;   // a walk always ends at a leaf (max_depth)
      const T p = row_dot<T, NCH, VW>(z, a.lw + (int64_t)leaf * a.ldl, l16) + a.lb[leaf];
      if (l16 == 0) {
        if (a.grid) a.grid[(r0 + S) * a.Bmax + b] = p;
        else a.edges[r0 + (S | (1 << b))] = p;
      }
    }
  }
  const bool bad = live && l16 == 0 && !__builtin_isfinite(chk);
  if (__ballot(bad) != 0 && (tid % kWave) == 0) atomicOr(a.status, (int)kStatusBadCounter);
}

template <typename T, int VPL>
hipError_t launch_m5p_vpl(const M5pArgs<T>& a, int n_tiles, hipStream_t s) {
  constexpr int VEC = 16 / sizeof(T);
  const bool vec = (a.E % VEC) == 0 && (reinterpret_cast<uintptr_t>(a.counters) % 16) == 0;
  (void)hipGetLastError();
  if (vec) hipLaunchKernelGGL((m5p_kernel<T, VPL, VEC>), dim3(n_tiles), dim3(kM5pThreads), 0, s, a);
  else hipLaunchKernelGGL((m5p_kernel<T, VPL, 1>), dim3(n_tiles), dim3(kM5pThreads), 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_m5p(const M5pArgs<T>& a, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  if (a.E <= 16 * 4) return launch_m5p_vpl<T, 4>(a, n_tiles, s);
  if (a.E <= 16 * 8) return launch_m5p_vpl<T, 8>(a, n_tiles, s);
  return launch_m5p_vpl<T, 16>(a, n_tiles, s);
}

template hipError_t launch_m5p<float>(const M5pArgs<float>&, int, hipStream_t);
template hipError_t launch_m5p<double>(const M5pArgs<double>&, int, hipStream_t);

}  // namespace sugg
