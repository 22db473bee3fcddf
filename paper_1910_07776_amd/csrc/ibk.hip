// Instance-based Tier 2 model (IBK, Section 3.4): k nearest neighbours of a
// standardised feature vector among the stored before/after samples of one
// optimisation, by Euclidean distance; the prediction is the mean of their
// labels.  Distances come from FP32 matrix-core products,
// |q - t|^2 = |q|^2 + |t|^2 - 2 q.t, one 32 x 32 block of (sample, query)
// pairs per v_mfma_f32_32x32x2_f32 sweep over the features.
#include <hip/hip_runtime.h>

#include <climits>
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

// ---- the k-nearest-neighbour search ------------------------------------------
// Each lane keeps the 16 nearest samples seen so far, ascending by (distance,
// sample index), in LDS (entry j of thread t at [j * 256 + t]); the current
// 16th is cached in registers so most candidates cost one comparison.
struct KnnList {
  float* d;
  int* i;
  float wd;
  int wi;
  __device__ __forceinline__ void init(float* ld, int* li, int tid) {
    d = ld + tid;
    i = li + tid;
    for (int j = 0; j < kIbkList; ++j) {
      d[j * 256] = INFINITY;
      i[j * 256] = INT_MAX;
    }
    wd = INFINITY;
    wi = INT_MAX;
  }
  __device__ __forceinline__ void insert(float dv, int s) {
    if (dv < wd || (dv == wd && s < wi)) {
      int j = kIbkList - 1;
      for (; j > 0; --j) {
        const float pd = d[(j - 1) * 256];
        const int pi = i[(j - 1) * 256];
        if (pd < dv || (pd == dv && pi < s)) break;
        d[j * 256] = pd;
        i[j * 256] = pi;
      }
      d[j * 256] = dv;
      i[j * 256] = s;
      wd = d[(kIbkList - 1) * 256];
      wi = i[(kIbkList - 1) * 256];
    }
  }
};

// One workgroup: one tile of up to 128 queries of one optimisation (wave w
// owns queries 32w .. 32w+31, one per lane column), sweeping the
// optimisation's samples in tiles of 32 staged in LDS; the next tile's loads
// are in flight while the current one is multiplied.  Lane l holds query
// (l mod 32)'s feature half h = l / 32: the matrix core's k-slot h of step j
// carries feature h*EH + j, for samples (A) and queries (B) alike, so the
// block product is the full dot product.
template <int EH, typename T>
__global__ void __launch_bounds__(256) ibk_knn_kernel(const IbkKnnArgs a) {
  constexpr int EP = 2 * EH;
  constexpr int LS = EP + 4;                           // padded LDS row (floats)
  constexpr int F4 = (kIbkTile * EP / 4) / 256;        // float4 per thread per tile
  static_assert(F4 >= 1 && (kIbkTile * EP / 4) % 256 == 0, "tile staging shape");
  __shared__ __align__(16) float tz[kIbkTile * LS];
  __shared__ float tn[kIbkTile];
  __shared__ float lst_d[kIbkList * 256];
  __shared__ int lst_i[kIbkList * 256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 31, h = lane >> 5;
  const int o = a.tiles[blockIdx.x * 4 + 0];
  const int q0 = a.tiles[blockIdx.x * 4 + 1];
  const int nq = a.tiles[blockIdx.x * 4 + 2];
  const int64_t s0 = a.off[o];
  const int ns = (int)(a.off[o + 1] - s0);
  const int qloc = wave * 32 + col;
  const bool qvalid = qloc < nq;
  const bool wave_live = wave * 32 < nq;

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
  KnnList L;
  L.init(lst_d, lst_i, tid);

  float4 stg[F4];
  float stn = INFINITY;
  auto fetch = [&](int t0) {
#pragma unroll
    for (int f = 0; f < F4; ++f) {
      const int idx = tid + f * 256;
      const int row = idx / (EP / 4), c4 = idx - row * (EP / 4);
      const int s = t0 + row;
      if (s < ns) {
        const int32_t r = a.srow[s0 + s];
        stg[f] = *reinterpret_cast<const float4*>(a.Z + (int64_t)r * EP + c4 * 4);
      } else {
        stg[f] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      }
    }
    if (tid < kIbkTile) {
      const int s = t0 + tid;
      stn = s < ns ? a.norm[a.srow[s0 + s]] : INFINITY;
    }
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

  fetch(0);
  for (int t0 = 0; t0 < ns; t0 += kIbkTile) {   // uniform over the workgroup
    store();
    __syncthreads();
    if (t0 + kIbkTile < ns) fetch(t0 + kIbkTile);   // in flight during the products
    if (wave_live) {
      floatx16 acc;
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
      const float* ar = &tz[col * LS + h * EH];
#pragma unroll
      for (int j = 0; j < EH; j += 4) {
        const float4 av = *reinterpret_cast<const float4*>(ar + j);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, qv[j], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, qv[j + 1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.z, qv[j + 2], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av.w, qv[j + 3], acc, 0, 0, 0);
      }
      // block entry r of this lane: sample (r/4)*8 + h*4 + r%4, query col
      float dd[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = (r >> 2) * 8 + h * 4 + (r & 3);
        dd[r] = t0 + i < ns ? qn + tn[i] - 2.0f * acc[r] : INFINITY;
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) L.insert(dd[r], t0 + (r >> 2) * 8 + h * 4 + (r & 3));
    }
    __syncthreads();   // the tile is consumed before the next store
  }
  // the two lanes of a query column saw disjoint samples: merge the partner's
  // list into the lane of half 0, then average the k nearest labels
  if (h == 0) {
    const float* pd = lst_d + (tid ^ 32);
    const int* pi = lst_i + (tid ^ 32);
    for (int j = 0; j < kIbkList; ++j) L.insert(pd[j * 256], pi[j * 256]);
    if (qvalid) {
      const int kk = a.k < ns ? a.k : ns;
      double sum = 0.0;
      for (int j = 0; j < kk; ++j) sum += a.y[s0 + L.i[j * 256]];
      reinterpret_cast<T*>(a.out)[a.q_dst[q0 + qloc]] = (T)(sum / (double)kk);
    }
  }
}

template <typename T>
hipError_t launch_ibk_knn(const IbkKnnArgs& a, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  (void)hipGetLastError();
  switch (a.Epad) {
    case 32:
      hipLaunchKernelGGL((ibk_knn_kernel<16, T>), dim3(n_tiles), dim3(256), 0, s, a);
      break;
    case 64:
      hipLaunchKernelGGL((ibk_knn_kernel<32, T>), dim3(n_tiles), dim3(256), 0, s, a);
      break;
    case 128:
      hipLaunchKernelGGL((ibk_knn_kernel<64, T>), dim3(n_tiles), dim3(256), 0, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
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
