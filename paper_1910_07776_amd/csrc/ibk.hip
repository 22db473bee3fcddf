// Instance-based Tier 2 model (IBK, Section 3.4): k nearest neighbours of a
// standardised feature vector among the stored before/after samples of one
// optimisation, by Euclidean distance; the prediction is the mean of their
// labels.  Distances come from FP32 matrix-core products,
// |q - t|^2 = |q|^2 + |t|^2 - 2 q.t, one 32 x 32 block of (sample, query)
// pairs per v_mfma_f32_32x32x2_f32 sweep over the features.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <type_traits>
#include <cmath>

#include "common.hpp"
#include "ibk.hpp"
#include "path_impl.hpp"

namespace sugg {

typedef float floatx16 __attribute__((ext_vector_type(16)));

// ---- standardised rows, zero-padded to Epad columns -------------------------
template <typename T>
__global__ void __launch_bounds__(256) ibk_z_kernel(const T* __restrict__ c, const T* __restrict__ cyc, int64_t N,
                                                    int E, int Epad, const double* __restrict__ mu,
                                                    const double* __restrict__ sig, float* __restrict__ z,
                                                    int32_t* status) {
  const int64_t total = N * Epad;
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / Epad;
    const int j = (int)(i - r * Epad);
    float v = 0.0f;
    if (j < E) {
      const T x = dlog<T>(c[r * E + j]) - dlog<T>(cyc[r]);
      bad |= !__builtin_isfinite(x);
      v = (float)(((double)x - mu[j]) / sig[j]);
    }
    z[i] = v;
  }
  if (__ballot(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(status, (int)kStatusBadCounter);
}

template <typename T>
hipError_t launch_ibk_z(const T* counters, const T* cycles, int64_t N, int32_t E, int32_t Epad,
                        const double* mu, const double* sig, float* z, int32_t* status, hipStream_t s) {
  const int64_t total = N * Epad;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  (void)hipGetLastError();
  hipLaunchKernelGGL(ibk_z_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, counters, cycles, N, (int)E,
                     (int)Epad, mu, sig, z, status);
  return hipGetLastError();
}

// ---- squared row norms: 16 lanes per row, float4 columns, fixed order -------
__global__ void __launch_bounds__(256) ibk_norm_kernel(const float* __restrict__ z, int64_t N, int Epad,
                                                       float* __restrict__ norm) {
  const int l16 = threadIdx.x & 15;
  const int64_t r = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 4;
  float acc = 0.0f;
  if (r < N)
    for (int j = l16 * 4; j < Epad; j += 64) {
      const float4 v = *reinterpret_cast<const float4*>(z + r * Epad + j);
      acc = fmaf(v.x, v.x, acc);
      acc = fmaf(v.y, v.y, acc);
      acc = fmaf(v.z, v.z, acc);
      acc = fmaf(v.w, v.w, acc);
    }
  acc = row_sum16(acc);
  if (r < N && l16 == 0) norm[r] = acc;
}

hipError_t launch_ibk_norm(const float* z, int64_t N, int32_t Epad, float* norm, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  const int64_t blocks = (N * 16 + 255) / 256;
  (void)hipGetLastError();
  hipLaunchKernelGGL(ibk_norm_kernel, dim3((unsigned)blocks), dim3(256), 0, s, z, N, (int)Epad, norm);
  return hipGetLastError();
}

// ---- labels: measured log-speedup of every stored pair, in FP64 -------------
template <typename T>
__global__ void __launch_bounds__(256) ibk_label_kernel(const T* __restrict__ cyc, const int32_t* __restrict__ before,
                                                        const int32_t* __restrict__ after, int64_t Ns,
                                                        double* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < Ns; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = log((double)cyc[before[i]]) - log((double)cyc[after[i]]);
}

template <typename T>
hipError_t launch_ibk_labels(const T* cycles, const int32_t* before, const int32_t* after, int64_t Ns, double* y,
                             hipStream_t s) {
  if (Ns <= 0) return hipSuccess;
  int64_t blocks = (Ns + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  (void)hipGetLastError();
  hipLaunchKernelGGL(ibk_label_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, cycles, before, after, Ns, y);
  return hipGetLastError();
}

// ---- sample rows in database order ---------------------------------------------
__global__ void __launch_bounds__(256) ibk_gather_kernel(const float* __restrict__ Z, const int32_t* __restrict__ srow,
                                                         int64_t Ns, int Epad, float* __restrict__ Zs) {
  const int q = Epad / 4;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < Ns * q; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = i / q;
    const int c = (int)(i - s * q) * 4;
    *reinterpret_cast<float4*>(Zs + s * Epad + c) =
        *reinterpret_cast<const float4*>(Z + (int64_t)srow[s] * Epad + c);
  }
}

hipError_t launch_ibk_gather(const float* Z, const int32_t* srow, int64_t Ns, int32_t Epad, float* Zs,
                             hipStream_t s) {
  if (Ns <= 0) return hipSuccess;
  int64_t blocks = (Ns * (Epad / 4) + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  (void)hipGetLastError();
  hipLaunchKernelGGL(ibk_gather_kernel, dim3((unsigned)blocks), dim3(256), 0, s, Z, srow, Ns, (int)Epad, Zs);
  return hipGetLastError();
}

// ---- the k-nearest-neighbour search ------------------------------------------
// A lane's KT nearest samples so far, ascending by (distance, sample index),
// in registers.  Insertion is a fixed compare-exchange pass (no indexing by
// lane data); callers guard it with a wave-uniform test so that the common
// case (no lane of the wave improves its list) costs one comparison.
template <int KT>
__device__ __forceinline__ bool knn_better(float d, int s, float wd, int wi) {
  return d < wd || (d == wd && s < wi);
}

template <int KT>
__device__ __forceinline__ void knn_insert(float (&ld)[KT], int (&li)[KT], float d, int s) {
  // the new entry replaces the last, then sinks to its place
  ld[KT - 1] = d;
  li[KT - 1] = s;
#pragma unroll
  for (int j = KT - 1; j > 0; --j) {
    const bool sw = ld[j] < ld[j - 1] || (ld[j] == ld[j - 1] && li[j] < li[j - 1]);
    const float td = ld[j - 1];
    const int ti = li[j - 1];
    ld[j - 1] = sw ? ld[j] : td;
    li[j - 1] = sw ? li[j] : ti;
    ld[j] = sw ? td : ld[j];
    li[j] = sw ? ti : li[j];
  }
}

// One workgroup: one tile of up to 128 queries of one optimisation (wave w
// owns queries 32w .. 32w+31, one per lane column), sweeping the
// optimisation's samples (contiguous rows) in tiles of 32 staged in LDS; the
// next tile's loads are in flight while the current one is multiplied.  Lane
// l holds query (l mod 32)'s feature half h = l / 32: the matrix core's
// k-slot h of step j carries feature h*EH + j, for samples (A) and queries
// (B) alike, so the block product is the full dot product.
template <int EH, int KT, typename T>
__global__ void __launch_bounds__(256) ibk_knn_kernel(const IbkKnnArgs a) {
  constexpr int EP = 2 * EH;
  constexpr int LS = EP + 4;                           // padded LDS row (floats)
  constexpr int F4 = (kIbkTile * EP / 4) / 256;        // float4 per thread per tile
  static_assert(F4 >= 1 && (kIbkTile * EP / 4) % 256 == 0, "tile staging shape");
  __shared__ __align__(16) float tz[kIbkTile * LS];
  __shared__ __align__(16) float tn[kIbkTile];
  // per-lane queue of candidates that beat the list's last entry as of the
  // latest merge (entry j of thread t at [j * 256 + t])
  __shared__ float qd[kIbkQueue * 256];
  __shared__ int qi[kIbkQueue * 256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 31, h = lane >> 5;
  const int tile = blockIdx.x / a.split, part = blockIdx.x - tile * a.split;
  const int o = a.tiles[tile * 4 + 0];
  const int q0 = a.tiles[tile * 4 + 1];
  const int nq = a.tiles[tile * 4 + 2];
  const int64_t s0 = a.off[o];
  const int ns = (int)(a.off[o + 1] - s0);
  // this workgroup's share of the samples: whole 32-sample tiles
  const int ntl = (ns + kIbkTile - 1) / kIbkTile, per = (ntl + a.split - 1) / a.split;
  const int tb = part * per * kIbkTile;
  const int te = min(ns, (part + 1) * per * kIbkTile);
  const int qloc = wave * 32 + col;
  const bool qvalid = qloc < nq;
  const bool wave_live = wave * 32 < nq;
  const float* Zo = a.Z + s0 * EP;
  const float* No = a.norm + s0;

  float qv[EH];
  {
    const int32_t qrow = a.q_src[q0 + (qvalid ? qloc : 0)];
    const float* qp = a.zq + (int64_t)qrow * EP + h * EH;
#pragma unroll
    for (int j = 0; j < EH; j += 4) {
      const float4 v = *reinterpret_cast<const float4*>(qp + j);
      qv[j] = v.x;
      qv[j + 1] = v.y;
      qv[j + 2] = v.z;
      qv[j + 3] = v.w;
    }
  }
  float qn = 0.0f;
#pragma unroll
  for (int j = 0; j < EH; ++j) qn = fmaf(qv[j], qv[j], qn);
  qn += __shfl_xor(qn, 32, kWave);
  float ld[KT];
  int li[KT];
#pragma unroll
  for (int j = 0; j < KT; ++j) {
    ld[j] = INFINITY;
    li[j] = INT_MAX;
  }

  int qc = 0;
  auto flush = [&]() {
    for (int j = 0; j < qc; ++j) {
      const float d = qd[j * 256 + tid];
      const int sidx = qi[j * 256 + tid];
      if (knn_better<KT>(d, sidx, ld[KT - 1], li[KT - 1])) knn_insert<KT>(ld, li, d, sidx);
    }
    qc = 0;
  };

  float4 stg[F4];
  float stn = INFINITY;
  auto fetch = [&](int t0) {
#pragma unroll
    for (int f = 0; f < F4; ++f) {
      const int idx = tid + f * 256;
      const int row = idx / (EP / 4), c4 = idx - row * (EP / 4);
      stg[f] = t0 + row < te ? *reinterpret_cast<const float4*>(Zo + (int64_t)(t0 + row) * EP + c4 * 4)
                             : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    if (tid < kIbkTile) stn = t0 + tid < te ? No[t0 + tid] : INFINITY;
  };
  auto store = [&]() {
#pragma unroll
    for (int f = 0; f < F4; ++f) {
      const int idx = tid + f * 256;
      const int row = idx / (EP / 4), c4 = idx - row * (EP / 4);
      *reinterpret_cast<float4*>(&tz[row * LS + c4 * 4]) = stg[f];
    }
    if (tid < kIbkTile) tn[tid] = stn;
  };

  if (tb < te) fetch(tb);
  for (int t0 = tb; t0 < te; t0 += kIbkTile) {   // uniform over the workgroup
    store();
    __syncthreads();
    if (t0 + kIbkTile < te) fetch(t0 + kIbkTile);   // in flight during the products
    if (wave_live) {
      // two accumulation chains (alternate groups of four features) keep
      // the matrix core busy across the dependent-accumulate latency
      floatx16 acc0, acc1;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        acc0[r] = 0.0f;
        acc1[r] = 0.0f;
      }
      const float* ar = &tz[col * LS + h * EH];
#pragma unroll
      for (int j = 0; j < EH; j += 8) {
        const float4 av = *reinterpret_cast<const float4*>(ar + j);
        const float4 bv = *reinterpret_cast<const float4*>(ar + j + 4);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, qv[j], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(bv.x, qv[j + 4], acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, qv[j + 1], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(bv.y, qv[j + 5], acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(av.z, qv[j + 2], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(bv.z, qv[j + 6], acc1, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(av.w, qv[j + 3], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(bv.w, qv[j + 7], acc1, 0, 0, 0);
      }
      // block entry r of this lane: sample (r/4)*8 + h*4 + r%4, query col;
      // padded samples have an infinite norm and never enter a list
      float4 tq[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) tq[g] = *reinterpret_cast<const float4*>(&tn[g * 8 + h * 4]);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = (r >> 2) * 8 + h * 4 + (r & 3);
        const float4 t4 = tq[r >> 2];
        const float tnv = (r & 3) == 0 ? t4.x : (r & 3) == 1 ? t4.y : (r & 3) == 2 ? t4.z : t4.w;
        const float d = qn + tnv - 2.0f * (acc0[r] + acc1[r]);
        if (knn_better<KT>(d, t0 + i, ld[KT - 1], li[KT - 1])) {
          qd[qc * 256 + tid] = d;
          qi[qc * 256 + tid] = t0 + i;
          ++qc;
        }
      }
      // merge the queues before one of them could overflow on the next tile:
      // the wave pays for its fullest lane, once for all of them
      if (__ballot(qc > kIbkQueue - 16) != 0ull) flush();
    }
    __syncthreads();   // the tile is consumed before the next store
  }
  flush();
  // the two lanes of a query column saw disjoint samples: merge the partner's
  // list, then average the k nearest labels
  float od[KT];
  int oi[KT];
#pragma unroll
  for (int j = 0; j < KT; ++j) {   // the partner's list as it stands, before either lane merges
    od[j] = __shfl_xor(ld[j], 32, kWave);
    oi[j] = __shfl_xor(li[j], 32, kWave);
  }
#pragma unroll
  for (int j = 0; j < KT; ++j)
    if (knn_better<KT>(od[j], oi[j], ld[KT - 1], li[KT - 1])) knn_insert<KT>(ld, li, od[j], oi[j]);
  if (a.split > 1) {   // partial list of this share; merged by ibk_merge_kernel
    if (h == 0 && qvalid) {
      const int64_t base = ((int64_t)(q0 + qloc) * a.split + part) * kIbkList;
#pragma unroll
      for (int j = 0; j < kIbkList; ++j) {
        a.part_d[base + j] = j < KT ? ld[j] : INFINITY;
        a.part_i[base + j] = j < KT ? li[j] : INT_MAX;
      }
    }
    return;
  }
  if (h == 0 && qvalid) {
    // a non-finite query or sample (bad counters, reported through the status
    // word) leaves slots unfilled: the prediction is then NaN, and no label
    // is read outside the optimisation's samples
    const int kk = a.k < ns ? a.k : ns;
    double sum = 0.0;
    bool full = true;
#pragma unroll
    for (int j = 0; j < KT; ++j)
      if (j < kk) {
        const bool ok = li[j] >= 0 && li[j] < ns;
        full = full && ok;
        sum += ok ? a.y[s0 + li[j]] : 0.0;
      }
    reinterpret_cast<T*>(a.out)[a.q_dst[q0 + qloc]] = full ? (T)(sum / (double)kk) : qnan<T>();
  }
}

// Merge of the partial lists of one query (one thread per query): the KT
// nearest over all shares, then the mean of their labels.
template <int KT, typename T>
__global__ void __launch_bounds__(256) ibk_merge_kernel(const IbkKnnArgs a) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= a.n_queries) return;
  float ld[KT];
  int li[KT];
#pragma unroll
  for (int j = 0; j < KT; ++j) {
    ld[j] = INFINITY;
    li[j] = INT_MAX;
  }
  for (int p = 0; p < a.split; ++p) {
    const int64_t base = (q * a.split + p) * kIbkList;
    for (int j = 0; j < KT; ++j) {
      const float d = a.part_d[base + j];
      const int s = a.part_i[base + j];
      if (!knn_better<KT>(d, s, ld[KT - 1], li[KT - 1])) break;   // lists are ascending
      knn_insert<KT>(ld, li, d, s);
    }
  }
  // the query's optimisation: the tile that holds it (tiles ascend in q)
  int lo = 0, hi = a.n_tiles - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.tiles[mid * 4 + 1] <= q) lo = mid;
    else hi = mid - 1;
  }
  const int o = a.tiles[lo * 4 + 0];
  const int64_t s0 = a.off[o];
  const int ns = (int)(a.off[o + 1] - s0);
  const int kk = a.k < ns ? a.k : ns;
  double sum = 0.0;
  bool full = true;
#pragma unroll
  for (int j = 0; j < KT; ++j)
    if (j < kk) {
      const bool ok = li[j] >= 0 && li[j] < ns;
      full = full && ok;
      sum += ok ? a.y[s0 + li[j]] : 0.0;
    }
  reinterpret_cast<T*>(a.out)[a.q_dst[q]] = full ? (T)(sum / (double)kk) : qnan<T>();
}

template <int EH, int KT, typename T>
hipError_t launch_knn_kt(const IbkKnnArgs& a, int n_tiles, hipStream_t s) {
  hipLaunchKernelGGL((ibk_knn_kernel<EH, KT, T>), dim3(n_tiles * a.split), dim3(256), 0, s, a);
  if (a.split > 1) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((ibk_merge_kernel<KT, T>), dim3((unsigned)((a.n_queries + 255) / 256)), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

// Sample shares per query tile: enough workgroups for one full round of the
// resident ones (occupancy of this kernel instance x compute units).
template <int EH, int KT>
int split_kt(int n_tiles, int cus) {
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(ibk_knn_kernel<EH, KT, float>),
                                                   256, 0) != hipSuccess || per < 1)
    per = 2;
  return n_tiles > 0 ? std::min(8, std::max(1, (per * cus + n_tiles - 1) / n_tiles)) : 1;
}

int ibk_split(int Epad, int k, int n_tiles, int cus) {
  auto by_k = [&](auto eh) -> int {
    constexpr int EH = decltype(eh)::value;
    if (k <= 4) return split_kt<EH, 4>(n_tiles, cus);
    if (k <= 8) return split_kt<EH, 8>(n_tiles, cus);
    if (k <= 12) return split_kt<EH, 12>(n_tiles, cus);
    return split_kt<EH, 16>(n_tiles, cus);
  };
  if (Epad == 32) return by_k(std::integral_constant<int, 16>{});
  if (Epad == 64) return by_k(std::integral_constant<int, 32>{});
  return by_k(std::integral_constant<int, 64>{});
}

template <int EH, typename T>
hipError_t launch_knn_eh(const IbkKnnArgs& a, int n_tiles, hipStream_t s) {
  if (a.k <= 4) return launch_knn_kt<EH, 4, T>(a, n_tiles, s);
  if (a.k <= 8) return launch_knn_kt<EH, 8, T>(a, n_tiles, s);
  if (a.k <= 12) return launch_knn_kt<EH, 12, T>(a, n_tiles, s);
  return launch_knn_kt<EH, 16, T>(a, n_tiles, s);
}

template <typename T>
hipError_t launch_ibk_knn(const IbkKnnArgs& a, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  (void)hipGetLastError();
  switch (a.Epad) {
    case 32: return launch_knn_eh<16, T>(a, n_tiles, s);
    case 64: return launch_knn_eh<32, T>(a, n_tiles, s);
    case 128: return launch_knn_eh<64, T>(a, n_tiles, s);
    default: return hipErrorInvalidValue;
  }
}

// ---- composition along the ascending chain, then the top-n ------------------
// L(S) = L(S without its highest bit b) + step(S), step(S) = the prediction of
// adding b to S without it (the same sum, in the same order, as adding the
// steps of the chain from the baseline one by one).  One wave per kernel.
template <typename T, int KT>
__global__ void __launch_bounds__(64) ibk_compose_kernel(const T* __restrict__ edges, const T* __restrict__ grid,
                                                         int grid_ld, const int64_t* __restrict__ row_off,
                                                         const int32_t* __restrict__ nopts, int K, T* table,
                                                         int32_t* idx_out, T* score_out, int32_t* count_out, int n,
                                                         T tau) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* L = reinterpret_cast<T*>(smem);
  const int k = blockIdx.x, lane = threadIdx.x;
  if (k >= K) return;
  const int B = nopts[k];
  const int64_t r0 = row_off[k];
  if (lane == 0) L[0] = T(0);
  __syncthreads();
  for (int b = 0; b < B; ++b) {
    const int lo = 1 << b;
    for (int S = lo + lane; S < 2 * lo; S += kWave) {
      const T e = edges ? edges[r0 + S] : grid[(r0 + S - lo) * grid_ld + b];
      L[S] = L[S - lo] + e;
    }
    __syncthreads();
  }
  Entry<T> lst[KT];
#pragma unroll
  for (int i = 0; i < KT; ++i) lst[i] = empty_entry<T>();
  for (int S = lane; S < (1 << B); S += kWave) {
    const T v = L[S];
    if (table) table[r0 + S] = v;
    if (S != 0 && v > tau) {
      Entry<T> e;
      e.v = v;
      e.s = S;
      list_insert<T, KT>(lst, e);
    }
  }
  if (idx_out) {
    group_merge<T, KT>(lst, kWave);
    if (lane == 0) write_list<T, KT>(lst, k, n, idx_out, score_out, count_out);
  }
}

template <typename T>
hipError_t launch_ibk_compose(const T* edges, const T* grid, int32_t grid_ld, const int64_t* row_off,
                              const int32_t* nopts, int32_t K, int32_t Bmax, T* table, int32_t* idx_out,
                              T* score_out, int32_t* count_out, int32_t n, T tau, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  const size_t smem = sizeof(T) * ((size_t)1 << Bmax);
  (void)hipGetLastError();
  if (n <= 4)
    hipLaunchKernelGGL((ibk_compose_kernel<T, 4>), dim3(K), dim3(64), smem, s, edges, grid, grid_ld, row_off,
                       nopts, K, table, idx_out, score_out, count_out, n, tau);
  else
    hipLaunchKernelGGL((ibk_compose_kernel<T, 8>), dim3(K), dim3(64), smem, s, edges, grid, grid_ld, row_off,
                       nopts, K, table, idx_out, score_out, count_out, n, tau);
  return hipGetLastError();
}

// ---- NaN fill (grid entries that are not predictions) ----------------------
template <typename T>
__global__ void __launch_bounds__(256) ibk_nan_kernel(T* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = qnan<T>();
}

template <typename T>
hipError_t launch_ibk_nan(T* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  (void)hipGetLastError();
  hipLaunchKernelGGL(ibk_nan_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

#define SUGG_INST(T)                                                                                        \
  template hipError_t launch_ibk_z<T>(const T*, const T*, int64_t, int32_t, int32_t, const double*,          \
                                      const double*, float*, int32_t*, hipStream_t);                         \
  template hipError_t launch_ibk_labels<T>(const T*, const int32_t*, const int32_t*, int64_t, double*,       \
                                           hipStream_t);                                                     \
  template hipError_t launch_ibk_knn<T>(const IbkKnnArgs&, int, hipStream_t);                                \
  template hipError_t launch_ibk_compose<T>(const T*, const T*, int32_t, const int64_t*, const int32_t*,     \
                                            int32_t, int32_t, T*, int32_t*, T*, int32_t*, int32_t, T,        \
                                            hipStream_t);                                                    \
  template hipError_t launch_ibk_nan<T>(T*, int64_t, hipStream_t);
SUGG_INST(float)
SUGG_INST(double)
#undef SUGG_INST

}  // namespace sugg
