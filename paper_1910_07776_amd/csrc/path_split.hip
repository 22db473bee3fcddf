// The scoring pass (Section 2, Tiers 1-3) for batches of equal kernels (the
// same B <= 6 and the same optimisations everywhere, rows kernel after
// kernel), split over 16-version workgroups.
//
// The fused kernel gives each kernel to one workgroup, whose chain (row loads,
// features, chain edges, composition, ranking) is serial; with a few hundred
// kernels per batch that leaves two workgroups per compute unit and little to
// overlap.  Here a kernel's 2^B versions are spread over 2^B / 16 workgroups
// of one row per 16-lane group: each forms the features and the chain edges
// of its rows (the prediction of adding every b above the row's top bit) and
// hands them to the other workgroups through a per-plan edge buffer; the last
// of the kernel's workgroups
// to arrive (a per-kernel counter, which it re-arms for the next launch)
// composes the table and takes the top n, in one wave, exactly as the fused
// kernel does.  Row, edge, composition and ranking arithmetic are the fused
// kernel's, so both forms give the same bits.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "path_impl.hpp"

namespace sugg {

constexpr int kSplitRows = 16;
constexpr int kSplitThreads = kSplitRows * kRowLanes;

// Edges cross workgroups (and XCDs, whose L2 caches are not coherent with each
// other) through device-scope atomics rather than through fences, which would
// write back a whole L2 per workgroup.  An edge is written with an exchange
// whose old value is consumed, so the write has been performed device-wide
// before the workgroup barrier that precedes the arrival count; the last
// arrival reads edges back with an OR of zero.  Bit patterns pass unchanged.
__device__ __forceinline__ void edge_put(float* p, float v) {
  const unsigned old = atomicExch(reinterpret_cast<unsigned*>(p), __float_as_uint(v));
  asm volatile("" ::"v"(old));
}
__device__ __forceinline__ void edge_put(double* p, double v) {
  const unsigned long long old =
      atomicExch(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v));
  asm volatile("" ::"v"(old));
}
__device__ __forceinline__ float edge_get(float* p) {
  return __uint_as_float(atomicOr(reinterpret_cast<unsigned*>(p), 0u));
}
__device__ __forceinline__ double edge_get(double* p) {
  return __longlong_as_double((long long)atomicOr(reinterpret_cast<unsigned long long*>(p), 0ull));
}

template <typename T, int VPL, int VW, bool FULL>
__global__ void __launch_bounds__(kSplitThreads) path_split_kernel(const PathArgs<T> a, int32_t* arrivals,
                                                                   T* edges) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NCH = VPL / VW;
  constexpr int EP = kRowLanes * VPL;
  const int E = a.E, D = a.D, B = a.uni_B;
  const int tid = threadIdx.x, g = tid / kRowLanes, l16 = tid % kRowLanes, lane = tid % kWave;
  const int V = 1 << B;
  const int parts = V > kSplitRows ? V / kSplitRows : 1;
  const int k = blockIdx.x / parts, part = blockIdx.x - k * parts;
  const int64_t row0 = (int64_t)k << B;
  const int S = part * kSplitRows + g;
  const bool live = S < V;
  const int Sr = live ? S : 0;   // a dead row re-reads the baseline and writes nothing
  T* Wl = reinterpret_cast<T*>(smem);
  T* Wb = Wl + D * EP;
  __shared__ int s_last;
  // the row is requested first, so its latency overlaps the weight staging
  T c[NCH][VW];
  const T* rp = a.counters + (row0 + Sr) * E;
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int c0 = (l16 + kRowLanes * ch) * VW;
    if (FULL || c0 < E) {
      const VecN<T, VW> q = *reinterpret_cast<const VecN<T, VW>*>(rp + c0);
#pragma unroll
      for (int v = 0; v < VW; ++v) c[ch][v] = q.v[v];
    } else {
#pragma unroll
      for (int v = 0; v < VW; ++v) c[ch][v] = T(1);
    }
  }
  const T cy = a.cycles[row0 + Sr];
  stage_weights<T, FULL>(a.W, a.ldw, D, E, EP, Wl, Wb, tid, kSplitThreads);
  T s_r[NCH][VW], m_r[NCH][VW];
  column_constants<T, NCH, VW, FULL>(a.mu, a.isg, E, l16, s_r, m_r);
  __syncthreads();
  T z[NCH][VW];
  const T chk = row_features<T, NCH, VW>(c, cy, s_r, m_r, z);
  const bool bad = live && !__builtin_isfinite(chk);
  if (live) {
    for (int h = (S ? 31 - __clz(S) : -1) + 1; h < B; ++h) {   // uniform per 16-lane group
      const int o = (int)((a.uni_opt_lo >> (8 * h)) & 0xffu);
      const T p = row_dot<T, NCH, VW>(z, Wl + o * EP, l16) + Wb[o];
      if (l16 == 0) edge_put(edges + row0 + (S | (1 << h)), p);
    }
  }
  if (__ballot(bad) != 0 && lane == 0) atomicOr(a.status, (int)kStatusBadCounter);
  // the last workgroup of the kernel composes and ranks it
  __shared__ T ev[64];
  __syncthreads();   // this workgroup's edge exchanges have returned
  if (parts > 1) {
    if (tid == 0) s_last = atomicAdd(arrivals + k, 1) == parts - 1;
    __syncthreads();
    if (!s_last) return;   // uniform per workgroup
    if (tid == 0) atomicExch(arrivals + k, 0);   // re-armed for the next launch
  }
  if (tid > 0 && tid < V) ev[tid] = edge_get(edges + row0 + tid);
  __syncthreads();
  if (tid >= kWave) return;
  // L(S) = sum over the bits b of S, ascending, of the edge into S & (2^(b+1) - 1)
  T x = -__builtin_inf();
  if (lane < V) {
    T L = T(0);
    for (int b = 0; b < B; ++b)
      if ((lane >> b) & 1) L += ev[lane & ((2 << b) - 1)];
    if (a.table) a.table[row0 + lane] = L;
    if (lane != 0 && L > a.tau) x = L;
  }
  if (!a.idx_out) return;
  // top n: n rounds of a group maximum (ties: the smallest S)
  const int G = V;
  const int gbase = lane & ~(G - 1);
  const uint64_t gmask = G == kWave ? ~0ull : ((1ull << G) - 1ull);
  T v = x;
  int place = -1;
  for (int j = 0; j < a.n; ++j) {
    const T m = group_max(v, G, lane);
    const bool hit = v == m && m > -__builtin_inf();
    const uint64_t won = (__ballot(hit) >> gbase) & gmask;
    if (won && lane == gbase + __ffsll((long long)won) - 1) {
      place = j;
      v = -__builtin_inf();
    }
  }
  const int cnt = __popcll((__ballot(place >= 0) >> gbase) & gmask);
  if (lane < V && place >= 0) {
    a.idx_out[(int64_t)k * a.n + place] = lane;
    a.score_out[(int64_t)k * a.n + place] = x;
  }
  if (lane == 0) {
    for (int j = cnt; j < a.n; ++j) {
      a.idx_out[(int64_t)k * a.n + j] = -1;
      a.score_out[(int64_t)k * a.n + j] = qnan<T>();
    }
    a.count_out[k] = cnt;
  }
}

template <typename T, int VPL>
hipError_t launch_split_vpl(const PathArgs<T>& a, int32_t* arrivals, T* edges, hipStream_t s) {
  constexpr int VEC = 16 / sizeof(T);
  constexpr int EP = kRowLanes * VPL;
  const int V = 1 << a.uni_B;
  const int parts = V > kSplitRows ? V / kSplitRows : 1;
  const dim3 grid((unsigned)(a.K * parts)), block(kSplitThreads);
  const size_t smem = sizeof(T) * ((size_t)a.D * EP + a.D) + 16;
  const bool vec_ok = (a.E % VEC) == 0 && (reinterpret_cast<uintptr_t>(a.counters) % 16) == 0;
  if (smem > 64 * 1024) {
    for (const void* f : {reinterpret_cast<const void*>(path_split_kernel<T, VPL, VEC, true>),
                          reinterpret_cast<const void*>(path_split_kernel<T, VPL, VEC, false>),
                          reinterpret_cast<const void*>(path_split_kernel<T, VPL, 1, false>)}) {
      const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
      if (e != hipSuccess) return e;
    }
  }
  (void)hipGetLastError();  // report only this launch's status
  if (vec_ok && a.E == EP)
    hipLaunchKernelGGL((path_split_kernel<T, VPL, VEC, true>), grid, block, smem, s, a, arrivals, edges);
  else if (vec_ok)
    hipLaunchKernelGGL((path_split_kernel<T, VPL, VEC, false>), grid, block, smem, s, a, arrivals, edges);
  else
    hipLaunchKernelGGL((path_split_kernel<T, VPL, 1, false>), grid, block, smem, s, a, arrivals, edges);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_path_split(const PathArgs<T>& a, int32_t* arrivals, T* edges, hipStream_t s) {
  if (a.K <= 0) return hipSuccess;
  if (a.E <= 16 * 4) return launch_split_vpl<T, 4>(a, arrivals, edges, s);
  if (a.E <= 16 * 8) return launch_split_vpl<T, 8>(a, arrivals, edges, s);
  return launch_split_vpl<T, 16>(a, arrivals, edges, s);
}

template hipError_t launch_path_split<float>(const PathArgs<float>&, int32_t*, float*, hipStream_t);
template hipError_t launch_path_split<double>(const PathArgs<double>&, int32_t*, double*, hipStream_t);

}  // namespace sugg
