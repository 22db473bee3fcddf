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

// ---- the FP32 rounding of the stored vectors, per column ----------------------
// Non-negative floats order as their bit patterns, so a column maximum is an
// unsigned maximum; each workgroup reduces its rows in LDS first.
__global__ void __launch_bounds__(256) ibk_dz_kernel(const float* __restrict__ z32, int Epad,
                                                     const double* __restrict__ z64, int64_t N, int E,
                                                     uint32_t* __restrict__ out) {
  __shared__ uint32_t m[256];
  for (int j = threadIdx.x; j < E; j += blockDim.x) m[j] = 0u;
  __syncthreads();
  const int64_t total = N * E;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / E;
    const int j = (int)(i - r * E);
    const double d = fabs((double)z32[r * Epad + j] - z64[i]);
    const float f = __builtin_isfinite(d) ? (float)d : INFINITY;
    // round up so the float never understates the double
    const float fu = (double)f < d ? __uint_as_float(__float_as_uint(f) + 1u) : f;   // next float up
    atomicMax(&m[j], __float_as_uint(fu));
  }
  __syncthreads();
  for (int j = threadIdx.x; j < E; j += blockDim.x)
    if (m[j]) atomicMax(&out[j], m[j]);
}

hipError_t launch_ibk_dz(const float* z32, int32_t Epad, const double* z64, int64_t N, int32_t E, uint32_t* out,
                         hipStream_t s) {
  if (N <= 0) return hipSuccess;
  int64_t blocks = (N * E + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  (void)hipGetLastError();
  hipLaunchKernelGGL(ibk_dz_kernel, dim3((unsigned)blocks), dim3(256), 0, s, z32, (int)Epad, z64, N, (int)E, out);
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

// During the sweep a lane's candidates are 64-bit keys: the distance's bits
// mapped to an unsigned order in the high word, the sample index in the low
// word, so one unsigned comparison orders two candidates by (distance, index)
// exactly as knn_better does (-0 is taken as +0 first).  The KT keys are kept
// unordered, with the largest (the worst candidate) and its slot tracked: an
// insertion overwrites that slot and finds the new largest in one fixed
// pass.  The set kept is the same as an ordered list's; it is ordered once,
// at the end.
__device__ __forceinline__ uint64_t knn_key(float d, int s) {
  const uint32_t b = __float_as_uint(d + 0.0f);
  const uint32_t o = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  return ((uint64_t)o << 32) | (uint32_t)s;
}
__device__ __forceinline__ float knn_key_d(uint64_t k) {
  const uint32_t o = (uint32_t)(k >> 32);
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}
__device__ __forceinline__ int knn_key_s(uint64_t k) { return (int)(uint32_t)k; }

template <int KT>
__device__ __forceinline__ void knn_put(uint64_t (&lk)[KT], uint64_t& wk, int& wp, uint64_t key) {
#pragma unroll
  for (int j = 0; j < KT; ++j) lk[j] = j == wp ? key : lk[j];
  wk = lk[0];
  wp = 0;
#pragma unroll
  for (int j = 1; j < KT; ++j) {
    const bool w = lk[j] > wk;
    wk = w ? lk[j] : wk;
    wp = w ? j : wp;
  }
}

// Odd-even transposition sort of the keys into ascending order (KT rounds of
// fixed compare-exchanges).
template <int KT>
__device__ __forceinline__ void knn_sort(uint64_t (&lk)[KT]) {
#pragma unroll
  for (int r = 0; r < KT; ++r)
#pragma unroll
    for (int j = r & 1; j + 1 < KT; j += 2) {
      const uint64_t a = lk[j], b = lk[j + 1];
      lk[j] = a < b ? a : b;
      lk[j + 1] = a < b ? b : a;
    }
}

// One workgroup: one tile of up to 128 queries of one optimisation (wave w
// owns queries 32w .. 32w+31, one per lane column), sweeping the
// optimisation's samples (contiguous rows) in tiles of 32 staged in LDS; the
// next tile's loads are in flight while the current one is multiplied.  Lane
// l holds query (l mod 32)'s feature half h = l / 32: the matrix core's
// k-slot h of step j carries feature h*EH + j, for samples (A) and queries
// (B) alike, so the block product is the full dot product.
// two workgroups per compute unit where the registers allow it without
// spilling (up to 128 events with lists of at most 16), else one
template <int EH, int KT>
constexpr int ibk_knn_waves() { return EH <= 64 && KT <= 16 ? 2 : 1; }

template <int EH, int KT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ibk_knn_waves<EH, KT>())))
ibk_knn_kernel(const IbkKnnArgs a) {
  constexpr int EP = 2 * EH;
  constexpr int LS = EP + 4;                           // padded LDS row (floats)
  constexpr int F4 = (kIbkTile * EP / 4) / 256;        // float4 per thread per tile
  static_assert(F4 >= 1 && (kIbkTile * EP / 4) % 256 == 0, "tile staging shape");
  __shared__ __align__(16) float tz[kIbkTile * LS];
  __shared__ __align__(16) float tn[kIbkTile];
  // per-lane queue of candidates that beat the list's last entry as of the
  // latest merge (entry j of thread t at [j * 256 + t])
  __shared__ uint64_t qk[kIbkQueue * 256];
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
  uint64_t lk[KT];
  const uint64_t empty = knn_key(INFINITY, INT_MAX);
#pragma unroll
  for (int j = 0; j < KT; ++j) lk[j] = empty;
  uint64_t wk = empty;   // the worst kept candidate, at slot wp
  int wp = 0;

  int qc = 0;
  auto flush = [&]() {
    // four queue entries read at a time (slots past qc read as the largest
    // key, which never enters): one LDS wait per four insertions
    for (int j = 0; j < qc; j += 4) {
      uint64_t key[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = j + u < kIbkQueue ? j + u : kIbkQueue - 1;   // in bounds even if read unconditionally
        key[u] = j + u < qc ? qk[q * 256 + tid] : ~0ull;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (key[u] < wk) knn_put<KT>(lk, wk, wp, key[u]);
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

  // Queues are merged by every wave of the workgroup at the same tile, when
  // one of them could overflow: merges at different tiles would each hold
  // the other waves at the next barrier.  flag[t % 2] is tile t's decision;
  // the other slot is cleared for the next tile.
  __shared__ int flag[2];
  if (tid < 2) flag[tid] = 0;
  int it = 0;
  if (tb < te) fetch(tb);
  for (int t0 = tb; t0 < te; t0 += kIbkTile, ++it) {   // uniform over the workgroup
    store();
    __syncthreads();
    if (tid == 0) flag[(it + 1) & 1] = 0;
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
        const uint64_t key = knn_key(d, t0 + i);
        if (key < wk) {
          qk[qc * 256 + tid] = key;
          ++qc;
        }
      }
      // merge the queues before one of them could overflow on the next tile
      // (a wave pays for its fullest lane, once for all of them)
      if (__ballot(qc > kIbkQueue - 16) != 0ull && lane == 0) flag[it & 1] = 1;
    }
    __syncthreads();   // the tile is consumed before the next store
    if (flag[it & 1]) flush();
  }
  flush();
  knn_sort<KT>(lk);
  float ld[KT];
  int li[KT];
#pragma unroll
  for (int j = 0; j < KT; ++j) {
    ld[j] = knn_key_d(lk[j]);
    li[j] = knn_key_s(lk[j]);
  }
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
  // the candidate list of this share (the whole database when split = 1):
  // re-ranked in FP64 by ibk_refine_kernel after the shares are merged
  if (h == 0 && qvalid) {
    const int64_t base = ((int64_t)(q0 + qloc) * a.split + part) * kIbkList;
#pragma unroll
    for (int j = 0; j < kIbkList; ++j) {
      a.part_d[base + j] = j < KT ? ld[j] : INFINITY;
      a.part_i[base + j] = j < KT ? li[j] : INT_MAX;
    }
  }
}

// Merge of the shares' candidate lists of one query (one thread per query):
// the KT best by FP32 distance over all shares, written over share 0's list.
template <int KT>
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
  const int64_t base = q * a.split * kIbkList;
#pragma unroll
  for (int j = 0; j < KT; ++j) {
    a.part_d[base + j] = ld[j];
    a.part_i[base + j] = li[j];
  }
}

// The global optimisation of query q: the tile that holds it (tiles ascend in q).
__device__ __forceinline__ int ibk_query_opt(const IbkKnnArgs& a, int64_t q) {
  int lo = 0, hi = a.n_tiles - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.tiles[mid * 4 + 1] <= q) lo = mid;
    else hi = mid - 1;
  }
  return a.tiles[lo * 4 + 0];
}

constexpr int kIbkMaxCols = 16;   // FP64 feature columns per lane (16 lanes x 16 = 256 events)

// This lane's FP64 standardised features of plan row r, columns l16 + 16 i
// (zero past E): z = (ln c - ln cyc - mu) / sigma, as the training rows.
template <typename T>
__device__ __forceinline__ void ibk_query64(const IbkKnnArgs& a, int64_t r, int l16, double (&q)[kIbkMaxCols]) {
  const T* c = reinterpret_cast<const T*>(a.counters) + r * a.E;
  const double lc = log((double)reinterpret_cast<const T*>(a.cycles)[r]);
#pragma unroll
  for (int i = 0; i < kIbkMaxCols; ++i) {
    const int j = l16 + 16 * i;
    q[i] = j < a.E ? (log((double)c[j]) - lc - a.mu64[j]) / a.sig64[j] : 0.0;
  }
}

// FP64 squared distance between this lane group's query and training row
// `row`, summed over the 16 lanes of the group (every lane receives it).
__device__ __forceinline__ double ibk_dist64(const IbkKnnArgs& a, int32_t row, int l16,
                                             const double (&q)[kIbkMaxCols]) {
  const double* t = a.Z64 + (int64_t)row * a.E;
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < kIbkMaxCols; ++i) {
    const int j = l16 + 16 * i;
    if (j < a.E) {
      const double d = q[i] - t[j];
      acc = fma(d, d, acc);
    }
  }
  return row_sum16(acc);
}

// Re-ranking (16 lanes per query): the KT FP32 candidates' exact FP64
// distances, the k nearest of them by (distance, sample index), and the mean
// of their labels.  Every sample outside the candidates has an FP32 distance
// of at least the list's last, dlast; its FP64 distance then exceeds
// dlast - err(dlast), err bounding the FP32 error (the features' FP32
// rounding and the accumulation in |q|^2 + |t|^2 - 2 q.t), so when the k-th
// FP64 distance lies below that the k nearest are certain.  Otherwise the
// query goes to the queue of ibk_exact_kernel.
template <typename T, int KT>
__global__ void __launch_bounds__(256) ibk_refine_kernel(const IbkKnnArgs a) {
  const int lane = threadIdx.x & 63, l16 = lane & 15;
  const int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  if (q >= a.n_queries) return;   // whole 16-lane groups leave together
  const int o = ibk_query_opt(a, q);
  const int64_t s0 = a.off[o];
  const int ns = (int)(a.off[o + 1] - s0);
  const int kk = a.k < ns ? a.k : ns;
  double qv[kIbkMaxCols];
  ibk_query64<T>(a, a.q_src[q], l16, qv);
  const int64_t base = q * a.split * kIbkList;
  double dd[KT];
  int di[KT];
  float dlast = INFINITY;
  bool full = true;
#pragma unroll
  for (int j = 0; j < KT; ++j) {
    const float d32 = a.part_d[base + j];
    const int s = a.part_i[base + j];
    const bool ok = s >= 0 && s < ns;
    full = full && ok;
    dlast = d32;
    dd[j] = ok ? ibk_dist64(a, a.srow[s0 + s], l16, qv) : INFINITY;
    di[j] = ok ? s : INT_MAX;
  }
  // selection of the k nearest (insertion, ties by the smaller sample index)
#pragma unroll
  for (int j = 1; j < KT; ++j) {
#pragma unroll
    for (int i = j; i > 0; --i) {
      const bool sw = dd[i] < dd[i - 1] || (dd[i] == dd[i - 1] && di[i] < di[i - 1]);
      const double td = dd[i - 1];
      const int ti = di[i - 1];
      dd[i - 1] = sw ? dd[i] : td;
      di[i - 1] = sw ? di[i] : ti;
      dd[i] = sw ? td : dd[i];
      di[i] = sw ? ti : di[i];
    }
  }
  double dk = 0.0, sum = 0.0;
  bool have = true;
#pragma unroll
  for (int j = 0; j < KT; ++j)
    if (j < kk) {
      dk = dd[j];
      have = have && di[j] != INT_MAX;
      sum += di[j] != INT_MAX ? a.y[s0 + di[j]] : 0.0;
    }
  // every sample is a candidate when the list is not full (ns < KT)
  bool certain = !full || ns <= KT;
  if (!certain && have) {
    // Dz bounds the FP32 rounding of query minus sample vectors (the query's
    // own, measured here, plus the stored vectors' worst); an outsider o
    // with FP64 distance u <= dk would have an FP32 distance of at most
    // g(u) = u + err(u) <= g(dk) < dlast and so be on the list
    const float* zr = a.zq + (int64_t)a.q_src[q] * a.Epad;
    double qn = 0.0, dq = 0.0;
#pragma unroll
    for (int i = 0; i < kIbkMaxCols; ++i) {
      const int j = l16 + 16 * i;
      qn = fma(qv[i], qv[i], qn);
      if (j < a.E) {
        const double e = (double)zr[j] - qv[i];
        dq = fma(e, e, dq);
      }
    }
    qn = row_sum16(qn);
    dq = row_sum16(dq);
    const double Dz = sqrt(dq) * (1.0 + 1e-12) + a.dt_norm;
    const double rk = sqrt(dk), rq = sqrt(qn);
    // FP32 sums of Epad products with |q32| + |t32| <= 2 |q| + sqrt(dk) + Dz
    const double eps = 1.01 * (double)(a.Epad + 2) * 5.9604644775390625e-8;
    const double span = 2.0 * rq + rk + Dz;
    const double err = 2.0 * rk * Dz + Dz * Dz + eps * span * span + 1e-12 * (1.0 + dk);
    certain = __builtin_isfinite((double)dlast) && __builtin_isfinite(err) && dk + err < (double)dlast;
  }
  if (l16 == 0) {
    if (certain && have) {
      reinterpret_cast<T*>(a.out)[a.q_dst[q]] = (T)(sum / (double)kk);
    } else if (!certain) {
      const int slot = atomicAdd(a.exact_n, 1);
      a.exact_q[slot] = (int32_t)q;
    } else {
      reinterpret_cast<T*>(a.out)[a.q_dst[q]] = qnan<T>();
    }
  }
}

// FP64 search over every sample of the query's optimisation for the queries
// whose candidates were not certain (queue from ibk_refine_kernel); one
// workgroup per query, taken in turn; 16 groups of 16 lanes each keep the
// k nearest of every 16th sample, merged by one thread at the end.
template <typename T>
__global__ void __launch_bounds__(256) ibk_exact_kernel(const IbkKnnArgs a) {
  __shared__ double sd[16 * kIbkMaxK];
  __shared__ int si[16 * kIbkMaxK];
  const int tid = threadIdx.x, l16 = tid & 15, g = tid >> 4;
  const int n = *a.exact_n;
  for (int w = blockIdx.x; w < n; w += gridDim.x) {
    const int64_t q = a.exact_q[w];
    const int o = ibk_query_opt(a, q);
    const int64_t s0 = a.off[o];
    const int ns = (int)(a.off[o + 1] - s0);
    const int kk = a.k < ns ? a.k : ns;
    double qv[kIbkMaxCols];
    ibk_query64<T>(a, a.q_src[q], l16, qv);
    double ld[kIbkMaxK];
    int li[kIbkMaxK];
#pragma unroll
    for (int j = 0; j < kIbkMaxK; ++j) {
      ld[j] = INFINITY;
      li[j] = INT_MAX;
    }
    for (int s = g; s < ns; s += 16) {   // uniform within the 16-lane group
      const double d = ibk_dist64(a, a.srow[s0 + s], l16, qv);
      if (d < ld[kIbkMaxK - 1] || (d == ld[kIbkMaxK - 1] && s < li[kIbkMaxK - 1])) {
        ld[kIbkMaxK - 1] = d;
        li[kIbkMaxK - 1] = s;
#pragma unroll
        for (int j = kIbkMaxK - 1; j > 0; --j) {
          const bool sw = ld[j] < ld[j - 1] || (ld[j] == ld[j - 1] && li[j] < li[j - 1]);
          const double td = ld[j - 1];
          const int ti = li[j - 1];
          ld[j - 1] = sw ? ld[j] : td;
          li[j - 1] = sw ? li[j] : ti;
          ld[j] = sw ? td : ld[j];
          li[j] = sw ? ti : li[j];
        }
      }
    }
    if (l16 == 0)
#pragma unroll
      for (int j = 0; j < kIbkMaxK; ++j) {
        sd[g * kIbkMaxK + j] = ld[j];
        si[g * kIbkMaxK + j] = li[j];
      }
    __syncthreads();
    if (tid == 0) {
      // the k nearest of the 16 group lists: repeated minimum over the heads
      int head[16];
      for (int h = 0; h < 16; ++h) head[h] = 0;
      double sum = 0.0;
      bool ok = true;
      for (int j = 0; j < kk; ++j) {
        int best = -1;
        for (int h = 0; h < 16; ++h) {
          if (head[h] >= kIbkMaxK) continue;
          const double d = sd[h * kIbkMaxK + head[h]];
          const int i = si[h * kIbkMaxK + head[h]];
          if (best < 0) {
            best = h;
            continue;
          }
          const double bd = sd[best * kIbkMaxK + head[best]];
          const int bi = si[best * kIbkMaxK + head[best]];
          if (d < bd || (d == bd && i < bi)) best = h;
        }
        const int i = si[best * kIbkMaxK + head[best]];
        ok = ok && i != INT_MAX;
        sum += i != INT_MAX ? a.y[s0 + i] : 0.0;
        ++head[best];
      }
      reinterpret_cast<T*>(a.out)[a.q_dst[q]] = ok ? (T)(sum / (double)kk) : qnan<T>();
    }
    __syncthreads();   // the lists are read before the next query writes them
  }
}

template <int EH, int KT, typename T>
hipError_t launch_knn_kt(const IbkKnnArgs& a, int n_tiles, hipStream_t s) {
  hipLaunchKernelGGL((ibk_knn_kernel<EH, KT>), dim3(n_tiles * a.split), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.split > 1) {
    hipLaunchKernelGGL((ibk_merge_kernel<KT>), dim3((unsigned)((a.n_queries + 255) / 256)), dim3(256), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  e = launch_fill_i32(a.exact_n, 0, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((ibk_refine_kernel<T, KT>), dim3((unsigned)((a.n_queries * 16 + 255) / 256)), dim3(256), 0, s,
                     a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((ibk_exact_kernel<T>), dim3(256), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Sample shares per query tile.
template <int EH, int KT>
int split_kt(int n_tiles, int cus) {
  // Sample shares per query tile: enough workgroups for one round of two per
  // compute unit (the search's occupancy), as a divisor of 8.  Workgroups go
  // to the eight XCDs in turn (workgroup w to XCD w mod 8) and workgroup w
  // takes share w mod split of its tile, so share s of every tile runs on
  // the XCDs s, s + split, ...: their L2s serve that share's samples to all
  // of the optimisation's tiles.  Measured on 252 query tiles: 8 shares
  // 2.77 ms, 4 shares 2.31, 2 shares 2.11, 1 share 2.68 (half the compute
  // units idle).
  const double want = 2.0 * cus / std::max(1, n_tiles);
  int split = 1;
  while (split < 8 && 2 * split <= want * 1.5) split *= 2;
  return split;
}

int ibk_split(int Epad, int k, int n_tiles, int cus) {
  auto by_k = [&](auto eh) -> int {
    constexpr int EH = decltype(eh)::value;
    const int kt = ibk_kt(k);
    if (kt == 8) return split_kt<EH, 8>(n_tiles, cus);
    if (kt == 16) return split_kt<EH, 16>(n_tiles, cus);
    return split_kt<EH, 24>(n_tiles, cus);
  };
  if (Epad == 32) return by_k(std::integral_constant<int, 16>{});
  if (Epad == 64) return by_k(std::integral_constant<int, 32>{});
  if (Epad == 128) return by_k(std::integral_constant<int, 64>{});
  return by_k(std::integral_constant<int, 128>{});
}

template <int EH, typename T>
hipError_t launch_knn_eh(const IbkKnnArgs& a, int n_tiles, hipStream_t s) {
  if (a.kt == 8) return launch_knn_kt<EH, 8, T>(a, n_tiles, s);
  if (a.kt == 16) return launch_knn_kt<EH, 16, T>(a, n_tiles, s);
  return launch_knn_kt<EH, 24, T>(a, n_tiles, s);
}

template <typename T>
hipError_t launch_ibk_knn(const IbkKnnArgs& a, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  if (a.kt != ibk_kt(a.k) || a.E > 16 * kIbkMaxCols || a.k > kIbkMaxK) return hipErrorInvalidValue;
  (void)hipGetLastError();
  switch (a.Epad) {
    case 32: return launch_knn_eh<16, T>(a, n_tiles, s);
    case 64: return launch_knn_eh<32, T>(a, n_tiles, s);
    case 128: return launch_knn_eh<64, T>(a, n_tiles, s);
    case 256: return launch_knn_eh<128, T>(a, n_tiles, s);
    default: return hipErrorInvalidValue;
  }
}

// ---- composition along the ascending chain, then the top-n ------------------
// L(S) = L(S without its highest bit b) + step(S), step(S) = the prediction of
// adding b to S without it (the same sum, in the same order, as adding the
// steps of the chain from the baseline one by one), in TE; outputs in TO.
// One wave per kernel.
template <typename TE, typename TO, int KT>
__global__ void __launch_bounds__(64) ibk_compose_kernel(const TE* __restrict__ edges, const TO* __restrict__ grid,
                                                         int grid_ld, const int64_t* __restrict__ row_off,
                                                         const int32_t* __restrict__ nopts, int K, TO* table,
                                                         int32_t* idx_out, TO* score_out, int32_t* count_out, int n,
                                                         TE tau) {
  extern __shared__ __align__(16) unsigned char smem[];
  TE* L = reinterpret_cast<TE*>(smem);
  const int k = blockIdx.x, lane = threadIdx.x;
  if (k >= K) return;
  const int B = nopts[k];
  const int64_t r0 = row_off[k];
  if (lane == 0) L[0] = TE(0);
  __syncthreads();
  for (int b = 0; b < B; ++b) {
    const int lo = 1 << b;
    for (int S = lo + lane; S < 2 * lo; S += kWave) {
      const TE e = edges ? edges[r0 + S] : (TE)grid[(r0 + S - lo) * grid_ld + b];
      L[S] = L[S - lo] + e;
    }
    __syncthreads();
  }
  Entry<TE> lst[KT];
#pragma unroll
  for (int i = 0; i < KT; ++i) lst[i] = empty_entry<TE>();
  for (int S = lane; S < (1 << B); S += kWave) {
    const TE v = L[S];
    if (table) table[r0 + S] = (TO)v;
    if (S != 0 && v > tau) {
      Entry<TE> e;
      e.v = v;
      e.s = S;
      list_insert<TE, KT>(lst, e);
    }
  }
  if (idx_out) {
    group_merge<TE, KT>(lst, kWave);
    if (lane == 0) {
      int cnt = 0;
#pragma unroll
      for (int i = 0; i < KT; ++i)
        if (i < n) {
          const bool ok = lst[i].s >= 0;
          idx_out[(int64_t)k * n + i] = ok ? lst[i].s : -1;
          score_out[(int64_t)k * n + i] = ok ? (TO)lst[i].v : qnan<TO>();
          cnt += ok ? 1 : 0;
        }
      count_out[k] = cnt;
    }
  }
}

template <typename TE, typename TO>
hipError_t launch_ibk_compose(const TE* edges, const TO* grid, int32_t grid_ld, const int64_t* row_off,
                              const int32_t* nopts, int32_t K, int32_t Bmax, TO* table, int32_t* idx_out,
                              TO* score_out, int32_t* count_out, int32_t n, TE tau, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  const size_t smem = sizeof(TE) * ((size_t)1 << Bmax);
  (void)hipGetLastError();
  if (n <= 4)
    hipLaunchKernelGGL((ibk_compose_kernel<TE, TO, 4>), dim3(K), dim3(64), smem, s, edges, grid, grid_ld, row_off,
                       nopts, K, table, idx_out, score_out, count_out, n, tau);
  else
    hipLaunchKernelGGL((ibk_compose_kernel<TE, TO, 8>), dim3(K), dim3(64), smem, s, edges, grid, grid_ld, row_off,
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
  template hipError_t launch_ibk_compose<T, T>(const T*, const T*, int32_t, const int64_t*, const int32_t*,  \
                                               int32_t, int32_t, T*, int32_t*, T*, int32_t*, int32_t, T,     \
                                               hipStream_t);                                                 \
  template hipError_t launch_ibk_nan<T>(T*, int64_t, hipStream_t);
SUGG_INST(float)
SUGG_INST(double)
#undef SUGG_INST
template hipError_t launch_ibk_compose<double, float>(const double*, const float*, int32_t, const int64_t*,
                                                      const int32_t*, int32_t, int32_t, float*, int32_t*, float*,
                                                      int32_t*, int32_t, double, hipStream_t);

}  // namespace sugg
