// Tier 1 statistics and feature kernels (Section 2: counters divided by the
// cycle count, then standardised per column), the generic Tier 3 ranking
// kernel, and small utilities.
#include "kernels.hpp"
#include "path_impl.hpp"

namespace sugg {

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

// ---- column statistics in FP64 -------------------------------------------
// Each workgroup owns a contiguous chunk of rows; 16 lanes share a row and
// each lane owns columns l16 + 16 i.  Sums of d = x - x(row 0) and d^2 are
// accumulated per lane, combined across the 16 row groups in a fixed order,
// and the chunks are combined in a fixed order by the final kernel, so the
// result is bit-reproducible.
constexpr int kMaxColsPerLane = 16;   // 256 events / 16 lanes
constexpr int kStatThreads = 256;

int colstats_chunks(int64_t N) {
  int64_t c = (N + 255) / 256;
  if (c > 1024) c = 1024;
  if (c < 1) c = 1;
  return (int)c;
}

template <typename T>
__global__ void __launch_bounds__(kStatThreads) colstats_partial_kernel(
    const T* __restrict__ c, const T* __restrict__ cyc, int64_t N, int E, int64_t rows_per_chunk,
    double* __restrict__ partial, int32_t* status) {
  const int tid = threadIdx.x, l16 = tid & 15, grp = tid >> 4;
  const int64_t r0 = blockIdx.x * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < N ? r0 + rows_per_chunk : N;
  __shared__ double red[16][16][2];
  const double lc0 = log((double)cyc[0]);
  double sh[kMaxColsPerLane], s1[kMaxColsPerLane], s2[kMaxColsPerLane];
#pragma unroll
  for (int i = 0; i < kMaxColsPerLane; ++i) {
    const int col = l16 + 16 * i;
    sh[i] = col < E ? log((double)c[col]) - lc0 : 0.0;
    s1[i] = 0.0;
    s2[i] = 0.0;
  }
  bool bad = false;
  for (int64_t r = r0 + grp; r < r1; r += 16) {
    const double lc = log((double)cyc[r]);
    const T* rp = c + r * E;
#pragma unroll
    for (int i = 0; i < kMaxColsPerLane; ++i) {
      const int col = l16 + 16 * i;
      if (col < E) {
        const double x = log((double)rp[col]) - lc;
        bad |= !__builtin_isfinite(x);
        const double d = x - sh[i];
        s1[i] += d;
        s2[i] = fma(d, d, s2[i]);
      }
    }
  }
  if (__ballot(bad) != 0 && (tid & 63) == 0) atomicOr(status, (int)kStatusBadCounter);
  double* out = partial + (int64_t)blockIdx.x * 2 * E;
#pragma unroll
  for (int i = 0; i < kMaxColsPerLane; ++i) {
    if (16 * i >= E) break;
    red[grp][l16][0] = s1[i];
    red[grp][l16][1] = s2[i];
    __syncthreads();
    if (grp == 0) {
      double a = 0.0, b = 0.0;
      for (int g = 0; g < 16; ++g) {
        a += red[g][l16][0];
        b += red[g][l16][1];
      }
      const int col = l16 + 16 * i;
      if (col < E) {
        out[col] = a;
        out[E + col] = b;
      }
    }
    __syncthreads();
  }
}

template <typename T>
__global__ void colstats_final_kernel(const T* __restrict__ c, const T* __restrict__ cyc, int64_t N,
                                      int E, const double* __restrict__ partial, int nchunks,
                                      double* mu64, double* sig64, T* mu_t, T* isg_t) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= E) return;
  const double sh = log((double)c[j]) - log((double)cyc[0]);
  double a = 0.0, b = 0.0;
  for (int q = 0; q < nchunks; ++q) {
    a += partial[(int64_t)q * 2 * E + j];
    b += partial[(int64_t)q * 2 * E + E + j];
  }
  const double m = a / (double)N;
  double var = b / (double)N - m * m;
  if (var < 0.0) var = 0.0;
  double sg = sqrt(var);
  if (sg < 1e-12) sg = 1.0;
  const double mu = sh + m;
  mu64[j] = mu;
  sig64[j] = sg;
  mu_t[j] = (T)mu;
  isg_t[j] = (T)(1.0 / sg);
}

template <typename T>
hipError_t launch_colstats(const T* counters, const T* cycles, int64_t N, int32_t E, double* partial,
                           int32_t nchunks, double* mu64, double* sig64, T* mu_t, T* isg_t,
                           int32_t* status, hipStream_t s) {
  if (N <= 0) return hipErrorInvalidValue;
  const int64_t per = (N + nchunks - 1) / nchunks;
  const int used = (int)((N + per - 1) / per);
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL(colstats_partial_kernel<T>, dim3(used), dim3(kStatThreads), 0, s, counters,
                     cycles, N, (int)E, per, partial, status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(colstats_final_kernel<T>, dim3((E + 255) / 256), dim3(256), 0, s, counters, cycles,
                     N, (int)E, partial, used, mu64, sig64, mu_t, isg_t);
  return hipGetLastError();
}

// ---- standardised features in the plan dtype -----------------------------
template <typename T>
__global__ void standardize_kernel(const T* __restrict__ c, const T* __restrict__ cyc, int64_t N, int E,
                                   const T* __restrict__ mu, const T* __restrict__ isg, T* __restrict__ z,
                                   int32_t* status) {
  const int64_t total = N * E;
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / E;
    const int j = (int)(i - r * E);
    const T x = dlog<T>(c[i]) - dlog<T>(cyc[r]);
    bad |= !__builtin_isfinite(x);
    z[i] = (x - mu[j]) * isg[j];
  }
  if (__ballot(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(status, (int)kStatusBadCounter);
}

template <typename T>
hipError_t launch_standardize(const T* counters, const T* cycles, int64_t N, int32_t E, const T* mu,
                              const T* isg, T* z, int32_t* status, hipStream_t s) {
  const int64_t total = N * E;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL(standardize_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, counters, cycles,
                     N, (int)E, mu, isg, z, status);
  return hipGetLastError();
}

// ---- standardised features of selected rows ------------------------------
// z[i][j] for row rows[i] (the baseline versions of a batch: rows = row_off),
// in the output type TO (the plan dtype, or BF16 for the surrogate's input):
// each 16-lane group takes one row at a time (ln of its cycle count once),
// its lanes striding over the columns; the value is (x - mu) * isg with
// x = ln c - ln cyc, rounded once to TO.
template <typename T, typename TO>
__global__ void standardize_rows_kernel(const T* __restrict__ c, const T* __restrict__ cyc,
                                        const int64_t* __restrict__ rows, int64_t nrows, int E,
                                        const T* __restrict__ mu, const T* __restrict__ isg, TO* __restrict__ z,
                                        int ldz, int32_t* status) {
  const int l16 = threadIdx.x & 15;
  const int64_t g0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 4, ng = ((int64_t)gridDim.x * blockDim.x) >> 4;
  bool bad = false;
  for (int64_t q = g0; q < nrows; q += ng) {
    const int64_t r = rows[q];
    const T lc = dlog<T>(cyc[r]);
    for (int j = l16; j < E; j += 16) {
      const T x = dlog<T>(c[r * E + j]) - lc;
      bad |= !__builtin_isfinite(x);
      z[q * ldz + j] = (TO)((x - mu[j]) * isg[j]);
    }
  }
  if (__ballot(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(status, (int)kStatusBadCounter);
}

template <typename T, typename TO>
hipError_t launch_standardize_rows_t(const T* counters, const T* cycles, const int64_t* rows, int64_t nrows, int32_t E,
                                     const T* mu, const T* isg, TO* z, int ldz, int32_t* status, hipStream_t s) {
  if (nrows <= 0 || E <= 0) return hipSuccess;
  int64_t blocks = (nrows + 15) / 16;   // 16 rows per workgroup of 256
  if (blocks > 16384) blocks = 16384;
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL((standardize_rows_kernel<T, TO>), dim3((unsigned)blocks), dim3(256), 0, s, counters, cycles,
                     rows, nrows, (int)E, mu, isg, z, ldz, status);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_standardize_rows(const T* counters, const T* cycles, const int64_t* rows, int64_t nrows, int32_t E,
                                   const T* mu, const T* isg, T* z, int32_t* status, hipStream_t s) {
  return launch_standardize_rows_t<T, T>(counters, cycles, rows, nrows, E, mu, isg, z, E, status, s);
}

hipError_t launch_standardize_rows_bf16(const float* counters, const float* cycles, const int64_t* rows, int64_t nrows,
                                        int32_t E, const float* mu, const float* isg, __bf16* z, int32_t ldz,
                                        int32_t* status, hipStream_t s) {
  return launch_standardize_rows_t<float, __bf16>(counters, cycles, rows, nrows, E, mu, isg, z, ldz, status, s);
}

// ---- FP64 features for the regression ------------------------------------
template <typename T>
__global__ void zfeat64_kernel(const T* __restrict__ c, const T* __restrict__ cyc, int64_t N, int E,
                               const double* __restrict__ mu, const double* __restrict__ sig,
                               double* __restrict__ z, double* __restrict__ lcyc) {
  const int64_t total = N * E;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / E;
    const int j = (int)(i - r * E);
    const double lc = log((double)cyc[r]);
    const double x = log((double)c[i]) - lc;
    z[i] = (x - mu[j]) / sig[j];
    if (j == 0) lcyc[r] = lc;
  }
}

template <typename T>
hipError_t launch_zfeat64(const T* counters, const T* cycles, int64_t N, int32_t E, const double* mu64,
                          const double* sig64, double* z64, double* lcyc64, hipStream_t s) {
  const int64_t total = N * E;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL(zfeat64_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, counters, cycles, N,
                     (int)E, mu64, sig64, z64, lcyc64);
  return hipGetLastError();
}

// ---- generic segmented Tier 3 ranking ------------------------------------
// One wave per segment: lanes stride over the segment keeping a best-first
// list each, then a butterfly of bitonic merges across the wave.
template <typename T, int KT>
__global__ void __launch_bounds__(256) rank_kernel(const T* __restrict__ scores,
                                                   const int64_t* __restrict__ seg_off, int nseg,
                                                   int skip, int n, T tau, int32_t* idx_out,
                                                   T* score_out, int32_t* count_out, int64_t seg_len) {
  const int lane = threadIdx.x & 63;
  const int seg = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (seg >= nseg) return;
  const int64_t b0 = seg_off ? seg_off[seg] : seg * seg_len, b1 = seg_off ? seg_off[seg + 1] : b0 + seg_len;
  const int64_t len = b1 - b0;
  Entry<T> lst[KT];
#pragma unroll
  for (int i = 0; i < KT; ++i) lst[i] = empty_entry<T>();
  for (int64_t p = skip + lane; p < len; p += kWave) {
    const T v = scores[b0 + p];
    if (v > tau) {
      Entry<T> e;
      e.v = v;
      e.s = (int32_t)p;
      list_insert<T, KT>(lst, e);
    }
  }
  group_merge<T, KT>(lst, kWave);
  if (lane == 0) write_list<T, KT>(lst, seg, n, idx_out, score_out, count_out);
}

template <typename T>
hipError_t launch_rank(const T* scores, const int64_t* seg_off, int32_t nseg, int32_t skip_head, int32_t n,
                       T tau, int32_t* idx_out, T* score_out, int32_t* count_out, hipStream_t s, int64_t seg_len) {
  if (nseg <= 0) return hipSuccess;
  const int blocks = (nseg + 3) / 4;
  (void)hipGetLastError();  // report only this launch's status
  if (n <= 4)
    hipLaunchKernelGGL((rank_kernel<T, 4>), dim3(blocks), dim3(256), 0, s, scores, seg_off, nseg, skip_head,
                       n, tau, idx_out, score_out, count_out, seg_len);
  else
    hipLaunchKernelGGL((rank_kernel<T, 8>), dim3(blocks), dim3(256), 0, s, scores, seg_off, nseg, skip_head,
                       n, tau, idx_out, score_out, count_out, seg_len);
  return hipGetLastError();
}

// Threshold band of a short suggestion list: for each segment whose top list
// (top_idx / top_count, as written by rank_kernel) holds fewer than n
// entries, the other entries p >= skip with score >= lo (compared in FP64),
// in ascending p, at most C of them; flag_out = 1 when there were more.  A
// full list has an empty band.  One wave per segment; the wave's ballot and
// prefix count place each taken entry, so the order is ascending.
template <typename T>
__global__ void __launch_bounds__(256) band_kernel(const T* __restrict__ scores,
                                                   const int64_t* __restrict__ seg_off, int nseg, int skip,
                                                   const int32_t* __restrict__ top_idx,
                                                   const int32_t* __restrict__ top_count, int n, double lo, int C,
                                                   int32_t* cand_out, T* ref_out, int32_t* flag_out) {
  const int lane = threadIdx.x & 63;
  const int seg = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (seg >= nseg) return;
  int32_t listed[kMaxSuggest];
  const int cnt = top_count[seg];
#pragma unroll
  for (int i = 0; i < kMaxSuggest; ++i) listed[i] = i < cnt && i < n ? top_idx[(int64_t)seg * n + i] : -1;
  int64_t total = 0;
  if (cnt < n) {
    const int64_t b0 = seg_off[seg], len = seg_off[seg + 1] - b0;
    for (int64_t base = skip; base < len; base += kWave) {   // uniform per wave
      const int64_t p = base + lane;
      bool take = false;
      T v = T(0);
      if (p < len) {
        v = scores[b0 + p];
        take = (double)v >= lo;
#pragma unroll
        for (int i = 0; i < kMaxSuggest; ++i) take = take && listed[i] != (int32_t)p;
      }
      const uint64_t m = __ballot(take);
      const int64_t pos = total + __popcll(m & ((1ull << lane) - 1ull));
      if (take && pos < C) {
        cand_out[(int64_t)seg * C + pos] = (int32_t)p;
        ref_out[(int64_t)seg * C + pos] = v;
      }
      total += __popcll(m);
    }
  }
  for (int64_t j = (total < C ? total : C) + lane; j < C; j += kWave) {
    cand_out[(int64_t)seg * C + j] = -1;
    ref_out[(int64_t)seg * C + j] = qnan<T>();
  }
  if (lane == 0) flag_out[seg] = total > C ? 1 : 0;
}

template <typename T>
hipError_t launch_band(const T* scores, const int64_t* seg_off, int32_t nseg, int32_t skip_head,
                       const int32_t* top_idx, const int32_t* top_count, int32_t n, double lo, int32_t C,
                       int32_t* cand_out, T* ref_out, int32_t* flag_out, hipStream_t s) {
  if (nseg <= 0) return hipSuccess;
  const int blocks = (nseg + 3) / 4;
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL((band_kernel<T>), dim3(blocks), dim3(256), 0, s, scores, seg_off, nseg, skip_head, top_idx,
                     top_count, n, lo, C, cand_out, ref_out, flag_out);
  return hipGetLastError();
}

// Tier 3's contract on a served kernel's kept answer (Section 2: only choices
// above the threshold, sorted by expected benefit), judged by the plain
// values: a listed subset whose plain value is not above tau, or a band
// subset whose plain value is above it, flags the kernel (flags already set
// stay set); an unflagged kernel's list is sorted by its plain values
// (descending, equal values by the smaller subset).  One thread per kernel.
__global__ void confirm_kernel(int K, int n, int32_t* __restrict__ idx, float* __restrict__ plain,
                               const int32_t* __restrict__ count, const int32_t* __restrict__ band_idx,
                               const float* __restrict__ band_plain, int C, float tau, int32_t* flag) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K || flag[k]) return;
  const int cnt = count[k] < n ? count[k] : n;
  bool bad = false;
  for (int i = 0; i < cnt; ++i) bad |= !(plain[(int64_t)k * n + i] > tau);
  for (int j = 0; j < C; ++j)
    if (band_idx[(int64_t)k * C + j] >= 0) bad |= band_plain[(int64_t)k * C + j] > tau;
  if (bad) {
    flag[k] = 1;
    return;
  }
  // insertion sort of at most SUGG_MAX_SUGGEST entries
  int32_t* ip = idx + (int64_t)k * n;
  float* vp = plain + (int64_t)k * n;
  for (int i = 1; i < cnt; ++i) {
    const float v = vp[i];
    const int32_t s = ip[i];
    int j = i;
    while (j > 0 && (vp[j - 1] < v || (vp[j - 1] == v && ip[j - 1] > s))) {
      vp[j] = vp[j - 1];
      ip[j] = ip[j - 1];
      --j;
    }
    vp[j] = v;
    ip[j] = s;
  }
}

hipError_t launch_confirm(int32_t K, int32_t n, int32_t* idx, float* plain, const int32_t* count,
                          const int32_t* band_idx, const float* band_plain, int32_t C, float tau, int32_t* flag,
                          hipStream_t s) {
  if (K <= 0) return hipSuccess;
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL(confirm_kernel, dim3((K + 255) / 256), dim3(256), 0, s, K, n, idx, plain, count, band_idx,
                     band_plain, C, tau, flag);
  return hipGetLastError();
}

#define SUGG_INST(T)                                                                                     \
  template hipError_t launch_colstats<T>(const T*, const T*, int64_t, int32_t, double*, int32_t, double*, \
                                         double*, T*, T*, int32_t*, hipStream_t);                         \
  template hipError_t launch_standardize<T>(const T*, const T*, int64_t, int32_t, const T*, const T*, T*, \
                                            int32_t*, hipStream_t);                                       \
  template hipError_t launch_standardize_rows<T>(const T*, const T*, const int64_t*, int64_t, int32_t, const T*, \
                                                 const T*, T*, int32_t*, hipStream_t);                         \
  template hipError_t launch_zfeat64<T>(const T*, const T*, int64_t, int32_t, const double*,              \
                                        const double*, double*, double*, hipStream_t);                    \
  template hipError_t launch_rank<T>(const T*, const int64_t*, int32_t, int32_t, int32_t, T, int32_t*, T*, \
                                     int32_t*, hipStream_t, int64_t);                                     \
  template hipError_t launch_band<T>(const T*, const int64_t*, int32_t, int32_t, const int32_t*,         \
                                     const int32_t*, int32_t, double, int32_t, int32_t*, T*, int32_t*,    \
                                     hipStream_t);
SUGG_INST(float)
SUGG_INST(double)
#undef SUGG_INST

}  // namespace sugg
