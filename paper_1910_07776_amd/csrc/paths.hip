// Two further uses of the single-optimisation predictions (Section 2, Tier 2):
//
//  allpaths  the composed log-speedup of a subset averaged over every order
//            of applying its optimisations:
//              L(0) = 0,  L(S) = (sum over b in S, ascending, of
//                                  [L(S - b) + P(S - b, b)]) / |S|
//            computed level by level in |S| from every prediction of the
//            kernel held in LDS, then Tier 3's top n.  One workgroup per
//            kernel.
//  greedy    the tool used iteratively on a kernel whose versions are all
//            profiled: from the baseline, apply the optimisation with the
//            largest predicted benefit above the threshold (ties: the smaller
//            bit), continue from the profiled version reached, until none
//            remains.  One wave per kernel; B steps at most.
//
// Both predict with the fused kernel's row arithmetic (row_features,
// row_dot), so their predictions equal the grid of sugg_predict bit for bit.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "path_impl.hpp"

namespace sugg {

constexpr int kPathsThreads = 256;

template <typename T, int NCH, int VW>
__device__ __forceinline__ void load_row(const T* rp, int E, int l16, T (&c)[NCH][VW]) {
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

// LDS: weights [D][EP], intercepts [D], grid [2^Bmax][Bmax], table [2^Bmax].
template <typename T>
__host__ __device__ inline size_t paths_smem(int D, int EP, int Bmax) {
  return sizeof(T) * ((size_t)D * EP + D + ((size_t)Bmax << Bmax) + ((size_t)1 << Bmax)) + 16;
}

template <typename T, int VPL, int VW, int KT>
__global__ void __launch_bounds__(kPathsThreads) allpaths_kernel(const PathsArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NCH = VPL / VW;
  const int EP = kRowLanes * VPL, E = a.E, D = a.D;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l16 = lane & 15, grp = lane >> 4;
  T* Wl = reinterpret_cast<T*>(smem);
  T* Wb = Wl + D * EP;
  T* G = Wb + D;
  T* L = G + ((size_t)a.Bmax << a.Bmax);
  stage_weights<T, false>(a.W, a.ldw, D, E, EP, Wl, Wb, tid, kPathsThreads);
  T s_r[NCH][VW], m_r[NCH][VW];
  column_constants<T, NCH, VW, false>(a.mu, a.isg, E, l16, s_r, m_r);
  const int k = blockIdx.x;
  const int B = a.nopts[k];
  const int64_t r0 = a.row_off[k];
  const int32_t* ids = a.opt_ids + a.opt_off[k];
  __syncthreads();
  // every prediction of the kernel: row S, bit b not in S
  bool bad = false;
  for (int S0 = wave * 4; S0 < (1 << B); S0 += (kPathsThreads / 64) * 4) {   // uniform per wave
    const int S = S0 + grp;
    const bool live = S < (1 << B);
    const int Sc = live ? S : (1 << B) - 1;
    T c[NCH][VW];
    load_row<T, NCH, VW>(a.counters + (r0 + Sc) * E, E, l16, c);
    T z[NCH][VW];
    const T chk = row_features<T, NCH, VW>(c, a.cycles[r0 + Sc], s_r, m_r, z);
    bad |= live && !__builtin_isfinite(chk);
    for (int b = 0; b < B; ++b) {
      const int o = ids[b];
      const T p = row_dot<T, NCH, VW>(z, Wl + o * EP, l16) + Wb[o];
      if (l16 == 0 && live) G[S * B + b] = ((S >> b) & 1) ? qnan<T>() : p;
    }
  }
  if (tid == 0) L[0] = T(0);
  __syncthreads();
  // composition by levels of |S|
  for (int lev = 1; lev <= B; ++lev) {
    for (int S = tid; S < (1 << B); S += kPathsThreads) {
      if (__popc((uint32_t)S) != (unsigned)lev) continue;
      T acc = T(0);
      for (int b = 0; b < B; ++b)
        if ((S >> b) & 1) {
          const int Sp = S & ~(1 << b);
          acc += L[Sp] + G[Sp * B + b];
        }
      L[S] = acc / (T)lev;
    }
    __syncthreads();
  }
  for (int S = tid; S < (1 << B); S += kPathsThreads) a.table[r0 + S] = L[S];
  if (a.idx_out && wave == 0) {
    Entry<T> lst[KT];
#pragma unroll
    for (int i = 0; i < KT; ++i) lst[i] = empty_entry<T>();
    for (int S = 1 + lane; S < (1 << B); S += 64) {
      const T v = L[S];
      if (v > a.tau) {
        Entry<T> e;
        e.v = v;
        e.s = S;
        list_insert<T, KT>(lst, e);
      }
    }
    group_merge<T, KT>(lst, kWave);
    if (lane == 0) write_list<T, KT>(lst, k, a.n, a.idx_out, a.score_out, a.count_out);
  }
  if (__ballot(bad) != 0 && lane == 0) atomicOr(a.status, (int)kStatusBadCounter);
}

// One wave per kernel; lanes 0..15 (one DPP row) read the current version's
// row, every lane of the row receives each prediction.
template <typename T, int VPL, int VW>
__global__ void __launch_bounds__(kPathsThreads) greedy_kernel(const PathsArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NCH = VPL / VW;
  const int EP = kRowLanes * VPL, E = a.E, D = a.D;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l16 = lane & 15;
  T* Wl = reinterpret_cast<T*>(smem);
  T* Wb = Wl + D * EP;
  stage_weights<T, false>(a.W, a.ldw, D, E, EP, Wl, Wb, tid, kPathsThreads);
  T s_r[NCH][VW], m_r[NCH][VW];
  column_constants<T, NCH, VW, false>(a.mu, a.isg, E, l16, s_r, m_r);
  __syncthreads();
  const int k = blockIdx.x * (kPathsThreads / 64) + wave;
  if (k >= a.K) return;   // no barrier follows
  const int B = a.nopts[k];
  const int64_t r0 = a.row_off[k];
  const int32_t* ids = a.opt_ids + a.opt_off[k];
  int S = 0, steps = 0;
  T gain = T(0);
  bool bad = false;
  int32_t* path = a.path_out + (int64_t)k * (a.Bmax + 1);
  if (lane == 0) path[0] = 0;
  while (true) {   // uniform per wave: every lane follows the same S
    T c[NCH][VW];
    load_row<T, NCH, VW>(a.counters + (r0 + S) * E, E, l16, c);
    T z[NCH][VW];
    const T chk = row_features<T, NCH, VW>(c, a.cycles[r0 + S], s_r, m_r, z);
    bad |= lane < kRowLanes && !__builtin_isfinite(chk);
    T best = T(0);
    int bb = -1;
    for (int b = 0; b < B; ++b) {
      if ((S >> b) & 1) continue;
      const int o = ids[b];
      const T p = row_dot<T, NCH, VW>(z, Wl + o * EP, l16) + Wb[o];
      const T pv = __shfl(p, 0, kWave);   // lane 0's value, the one every kernel uses
      if (pv > a.tau && (bb < 0 || pv > best)) {
        best = pv;
        bb = b;
      }
    }
    if (bb < 0) break;
    S |= 1 << bb;
    gain += best;
    ++steps;
    if (lane == 0) path[steps] = S;
  }
  if (lane == 0) {
    for (int i = steps + 1; i <= a.Bmax; ++i) path[i] = -1;
    a.steps_out[k] = steps;
    a.gain_out[k] = gain;
  }
  if (__ballot(bad) != 0 && lane == 0) atomicOr(a.status, (int)kStatusBadCounter);
}

template <typename T, int VPL>
hipError_t launch_paths_vpl(const PathsArgs<T>& a, bool greedy, hipStream_t s) {
  constexpr int VEC = 16 / sizeof(T);
  const int EP = kRowLanes * VPL;
  const bool vec = (a.E % VEC) == 0 && (reinterpret_cast<uintptr_t>(a.counters) % 16) == 0;
  (void)hipGetLastError();
  if (greedy) {
    const size_t smem = sizeof(T) * ((size_t)a.D * EP + a.D) + 16;
    const dim3 grid((unsigned)((a.K + 3) / 4));
    if (vec) hipLaunchKernelGGL((greedy_kernel<T, VPL, VEC>), grid, dim3(kPathsThreads), smem, s, a);
    else hipLaunchKernelGGL((greedy_kernel<T, VPL, 1>), grid, dim3(kPathsThreads), smem, s, a);
    return hipGetLastError();
  }
  const size_t smem = paths_smem<T>(a.D, EP, a.Bmax);
  auto pick = [&](auto kern) -> hipError_t {
    if (smem > 64 * 1024) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(a.K), dim3(kPathsThreads), smem, s, a);
    return hipGetLastError();
  };
  if (a.n <= 4) return vec ? pick(allpaths_kernel<T, VPL, VEC, 4>) : pick(allpaths_kernel<T, VPL, 1, 4>);
  return vec ? pick(allpaths_kernel<T, VPL, VEC, 8>) : pick(allpaths_kernel<T, VPL, 1, 8>);
}

template <typename T>
hipError_t launch_paths(const PathsArgs<T>& a, bool greedy, hipStream_t s) {
  if (a.K <= 0) return hipSuccess;
  if (a.E <= 16 * 4) return launch_paths_vpl<T, 4>(a, greedy, s);
  if (a.E <= 16 * 8) return launch_paths_vpl<T, 8>(a, greedy, s);
  return launch_paths_vpl<T, 16>(a, greedy, s);
}

template <typename T>
size_t paths_lds_bytes(int D, int E, int Bmax) {
  const int EP = E <= 64 ? 64 : E <= 128 ? 128 : 256;
  return paths_smem<T>(D, EP, Bmax);
}

template hipError_t launch_paths<float>(const PathsArgs<float>&, bool, hipStream_t);
template hipError_t launch_paths<double>(const PathsArgs<double>&, bool, hipStream_t);
template size_t paths_lds_bytes<float>(int, int, int);
template size_t paths_lds_bytes<double>(int, int, int);

}  // namespace sugg
