// Tier 2 training (Section 2: before/after samples of each optimisation;
// Section 3.4: regression): per global optimisation o, the ridge normal
// equations
//   (X^T X + lambda diag(1,..,1,0)) w_o = X^T y,   X = [z(before), 1],
//   y = ln cyc(before) - ln cyc(after),
// over every pair (version S without o, version S with o) of the training
// kernels, accumulated and solved in FP64.
//
// gram_kernel   one workgroup per chunk of one optimisation's pairs: stages
//               32 samples' z rows in LDS, each thread accumulates an 8x8
//               register block of Z^T Z (plus the column sums for the
//               intercept row and X^T y); the partial goes to a workspace.
// solve_kernel  one workgroup per optimisation: sums its chunks in a fixed
//               order, adds the ridge term, factorises A = L L^T (right-looking,
//               in LDS when it fits) and solves two triangular systems.
#include "kernels.hpp"

namespace sugg {

constexpr int kGramThreads = 256;
constexpr int kGramStage = 32;
constexpr int kBlk = 8;

__device__ __forceinline__ int64_t insert_zero_bit(int64_t q, int b) {
  return ((q >> b) << (b + 1)) | (q & ((1ll << b) - 1));
}

__global__ void __launch_bounds__(kGramThreads) gram_kernel(const GramArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int E = a.E;
  double* zs = reinterpret_cast<double*>(smem);            // [kGramStage][E]
  double* ys = zs + kGramStage * E;                          // [kGramStage]
  int64_t* rows = reinterpret_cast<int64_t*>(ys + kGramStage);
  const GramWork w = a.work[blockIdx.x];
  const int tid = threadIdx.x;
  const int nb = (E + kBlk - 1) / kBlk;
  const int nblocks = nb * (nb + 1) / 2;   // blocks on and below the diagonal (Z^T Z is symmetric)
  const int64_t stride = (int64_t)E * E + 2 * E + 2;
  double* out = a.partial + (int64_t)blockIdx.x * stride;

  // column sums (first pass only): thread j < E owns column j
  double cz = 0.0, czy = 0.0, sy = 0.0;
  const int64_t ns = w.s_end - w.s_begin;

  for (int pass = 0; pass * kGramThreads < nblocks; ++pass) {
    const int blk = pass * kGramThreads + tid;
    const bool active = blk < nblocks;
    // lower-triangle block t = bi (bi + 1) / 2 + bj, bj <= bi
    int bi = 0, bj = 0;
    if (active) {
      bi = (int)((sqrt(8.0 * blk + 1.0) - 1.0) * 0.5);
      while (bi * (bi + 1) / 2 > blk) --bi;
      while ((bi + 1) * (bi + 2) / 2 <= blk) ++bi;
      bj = blk - bi * (bi + 1) / 2;
    }
    double acc[kBlk][kBlk];
#pragma unroll
    for (int i = 0; i < kBlk; ++i)
#pragma unroll
      for (int j = 0; j < kBlk; ++j) acc[i][j] = 0.0;

    for (int64_t s0 = 0; s0 < ns; s0 += kGramStage) {
      const int cnt = (int)((ns - s0) < kGramStage ? (ns - s0) : kGramStage);
      if (tid < cnt) {
        const int64_t s = w.s_begin + s0 + tid;
        int lo = w.list_begin, hi = w.list_end - 1;
        while (lo < hi) {   // last entry with pair_base <= s
          const int mid = (lo + hi + 1) >> 1;
          if (a.pair_base[mid] <= s) lo = mid; else hi = mid - 1;
        }
        const int b = a.pair_bit[lo];
        const int64_t S = insert_zero_bit(s - a.pair_base[lo], b);
        const int64_t row = a.pair_row0[lo] + S;
        rows[tid] = row;
        ys[tid] = a.lcyc64[row] - a.lcyc64[row + (1ll << b)];
      }
      __syncthreads();
      for (int i = tid; i < cnt * E; i += kGramThreads) {
        const int q = i / E, j = i - q * E;
        zs[i] = a.z64[rows[q] * E + j];
      }
      __syncthreads();
      if (active) {
        for (int q = 0; q < cnt; ++q) {
          const double* zq = zs + q * E;
          double zi[kBlk], zj[kBlk];
#pragma unroll
          for (int i = 0; i < kBlk; ++i) {
            const int ci = bi * kBlk + i, cj = bj * kBlk + i;
            zi[i] = ci < E ? zq[ci] : 0.0;
            zj[i] = cj < E ? zq[cj] : 0.0;
          }
#pragma unroll
          for (int i = 0; i < kBlk; ++i)
#pragma unroll
            for (int j = 0; j < kBlk; ++j) acc[i][j] = fma(zi[i], zj[j], acc[i][j]);
        }
      }
      if (pass == 0) {
        for (int j = tid; j < E; j += kGramThreads) {
          // a thread owns at most one column when E <= 256
          for (int q = 0; q < cnt; ++q) {
            const double zv = zs[q * E + j];
            cz += zv;
            czy = fma(zv, ys[q], czy);
          }
        }
        if (tid == 0)
          for (int q = 0; q < cnt; ++q) sy += ys[q];
      }
      __syncthreads();
    }
    if (active) {
#pragma unroll
      for (int i = 0; i < kBlk; ++i)
#pragma unroll
        for (int j = 0; j < kBlk; ++j) {
          const int ci = bi * kBlk + i, cj = bj * kBlk + j;
          if (ci < E && cj < E) out[(int64_t)ci * E + cj] = acc[i][j];
        }
    }
  }
  for (int j = tid; j < E; j += kGramThreads) {
    out[(int64_t)E * E + j] = cz;
    out[(int64_t)E * E + E + j] = czy;
  }
  if (tid == 0) {
    out[(int64_t)E * E + 2 * E] = sy;
    out[(int64_t)E * E + 2 * E + 1] = (double)ns;
  }
}

hipError_t launch_gram(const GramArgs& a, hipStream_t s) {
  if (a.n_work <= 0) return hipSuccess;
  const size_t smem = sizeof(double) * ((size_t)kGramStage * a.E + kGramStage) + sizeof(int64_t) * kGramStage;
  if (smem > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(gram_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
  }
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL(gram_kernel, dim3(a.n_work), dim3(kGramThreads), smem, s, a);
  return hipGetLastError();
}

// Sum the partials of each optimisation's chunks in a fixed order; adjacent
// threads read adjacent words of a chunk's partial.
__global__ void __launch_bounds__(256) gram_reduce_kernel(const double* __restrict__ partial,
                                                          const int32_t* __restrict__ opt_work_begin,
                                                          int64_t stride, double* __restrict__ out) {
  const int o = blockIdx.y;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= stride) return;
  const int wb = opt_work_begin[o], we = opt_work_begin[o + 1];
  double v = 0.0;
  for (int q = wb; q < we; ++q) v += partial[(int64_t)q * stride + i];
  out[(int64_t)o * stride + i] = v;
}

constexpr int kSolveThreads = 256;
constexpr size_t kSolveLdsMax = 150 * 1024;

__global__ void __launch_bounds__(kSolveThreads) solve_kernel(const SolveArgs a, const int use_lds) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int o = blockIdx.x;
  const int E = a.E, n1 = E + 1;
  const int tid = threadIdx.x;
  const int wb = a.opt_work_begin[o], we = a.opt_work_begin[o + 1];
  if (wb == we) {
    for (int j = tid; j < n1; j += kSolveThreads) {
      a.W64[(int64_t)o * n1 + j] = __builtin_nan("");
      a.W32[(int64_t)o * w32_ld(E) + j] = 0.0f;
    }
    return;
  }
  double* A = use_lds ? reinterpret_cast<double*>(smem) : a.A + (int64_t)o * n1 * n1;
  __shared__ double y[SUGG_MAX_EVENTS + 1];
  const int64_t stride = (int64_t)E * E + 2 * E + 2;
  const double* G = a.reduced + (int64_t)o * stride;   // this optimisation's summed partial
  for (int idx = tid; idx < n1 * n1; idx += kSolveThreads) {
    const int i = idx / n1, j = idx - i * n1;
    int64_t off;
    if (i < E && j < E) off = i >= j ? (int64_t)i * E + j : (int64_t)j * E + i;   // lower triangle
    else if (i < E) off = (int64_t)E * E + i;          // column sums
    else if (j < E) off = (int64_t)E * E + j;
    else off = (int64_t)E * E + 2 * E + 1;             // sample count
    double v = G[off];
    if (i == j && i < E) v += a.lambda;
    A[idx] = v;
  }
  for (int i = tid; i < n1; i += kSolveThreads)
    y[i] = G[i < E ? (int64_t)E * E + E + i : (int64_t)E * E + 2 * E];
  __syncthreads();
  // A = L L^T, lower triangle in place (right-looking).  Every thread reads
  // the pivot itself, so a step needs two barriers; the trailing update uses a
  // 16 x 16 thread tile over the lower triangle.
  bool bad = false;
  const int ty = tid >> 4, tx = tid & 15;
  for (int k = 0; k < n1; ++k) {
    double d = A[k * n1 + k];
    if (!(d > 0.0)) {
      bad = true;
      d = 1.0;
    }
    const double piv = sqrt(d);
    __syncthreads();
    if (tid == 0) A[k * n1 + k] = piv;
    for (int i = k + 1 + tid; i < n1; i += kSolveThreads) A[i * n1 + k] /= piv;
    __syncthreads();
    for (int i = k + 1 + ty; i < n1; i += 16) {
      const double aik = A[i * n1 + k];
      for (int j = k + 1 + tx; j <= i; j += 16) A[i * n1 + j] -= aik * A[j * n1 + k];
    }
    __syncthreads();
  }
  // L t = rhs, then L^T w = t (column-oriented, one barrier per step)
  for (int k = 0; k < n1; ++k) {
    const double yk = y[k] / A[k * n1 + k];
    __syncthreads();
    if (tid == 0) y[k] = yk;
    for (int i = k + 1 + tid; i < n1; i += kSolveThreads) y[i] -= A[i * n1 + k] * yk;
    __syncthreads();
  }
  for (int k = n1 - 1; k >= 0; --k) {
    const double yk = y[k] / A[k * n1 + k];
    __syncthreads();
    if (tid == 0) y[k] = yk;
    for (int i = tid; i < k; i += kSolveThreads) y[i] -= A[k * n1 + i] * yk;
    __syncthreads();
  }
  for (int j = tid; j < n1; j += kSolveThreads) {
    a.W64[(int64_t)o * n1 + j] = y[j];
    a.W32[(int64_t)o * w32_ld(E) + j] = (float)y[j];
  }
  if (tid == 0 && bad) atomicOr(a.status, (int)kStatusSingular);
}

hipError_t launch_solve(const SolveArgs& a, hipStream_t s) {
  if (a.D <= 0) return hipSuccess;
  const size_t need = sizeof(double) * (size_t)(a.E + 1) * (a.E + 1);
  const int use_lds = need <= kSolveLdsMax ? 1 : 0;
  const size_t smem = use_lds ? need : 0;
  if (smem > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(solve_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
  }
  const int64_t stride = (int64_t)a.E * a.E + 2 * a.E + 2;
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((stride + 255) / 256), a.D), dim3(256), 0, s, a.partial,
                     a.opt_work_begin, stride, a.reduced);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(solve_kernel, dim3(a.D), dim3(kSolveThreads), smem, s, a, use_lds);
  return hipGetLastError();
}

}  // namespace sugg
