// The learned surrogate: an MLP in -> h -> h -> out with exact-erf GELU after
// each hidden layer that maps a kernel's standardised baseline counters to the
// composed log-speedups of all its optimisation subsets in one pass.  This
// extends the paper (whose Tier 2 scores one optimisation at a time); it is
// trained on tables the plain Tier 2 path produces.
//
// Every product is one GEMM form, C[M x N] = A[M x K] . Bt[N x K]^T, with both
// operands K-contiguous in BF16 and FP32 accumulation on the gfx950
// v_mfma_f32_32x32x16_bf16 matrix cores.  To keep every operand K-contiguous,
// activations and their gradients are written twice by the producing
// epilogue (row-major for the next layer, transposed for the weight
// gradient), and the BF16 working weights are packed in both layouts.
//
//   forward   A_l = H_{l-1} W_l^T + b_l, H_l = gelu(A_l); Y = H_2 W_3^T + b_3
//   loss      mean over batch and outputs of (Y - T)^2, dY = 2 (Y - T) / (B out)
//   backward  dW_l = dA_l^T H_{l-1} (split over the batch, summed in order),
//             db_l = column sums of dA_l, dA_{l-1} = (dA_l W_l) * gelu'(A_{l-1})
//   Adam      on FP32 master weights, bias-corrected.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace sugg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kKStep = 32;    // K per LDS stage (two MFMAs of K 16)
constexpr int kKVec = kKStep / 32;   // 8-element vectors per thread and tile row per stage
constexpr int kLdsRow = kKStep + 8;   // padded LDS row (bf16 elements)

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// Load 8 consecutive K elements of row `row` (zero outside [0, rows) x [0, K)).
__device__ __forceinline__ bf16x8 load8(const __bf16* p, int ld, int row, int rows, int k, int K) {
  bf16x8 v;
  if (row < rows && k + 8 <= K) {
    v = *reinterpret_cast<const bf16x8*>(p + (int64_t)row * ld + k);
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = (row < rows && k + i < K) ? p[(int64_t)row * ld + k + i] : (__bf16)0.0f;
  }
  return v;
}

// Workgroup of 4 waves in a 2 x 2 arrangement; each wave computes TM x TN
// MFMA tiles of 32 x 32, so the workgroup tile is (64 TM) x (64 TN).  EX: the
// tiles cover M, N and each K range exactly and rows are 16-byte aligned, so
// operand loads and output stores need no bounds checks.
template <int EPI, int TM, int TN, bool EX>
__global__ void __launch_bounds__(256, 3) gemm_nt_kernel(const GemmArgs g) {
  constexpr int WGM = 64 * TM, WGN = 64 * TN;
  __shared__ __align__(16) __bf16 As[2][WGM * kLdsRow];
  __shared__ __align__(16) __bf16 Bs[2][WGN * kLdsRow];
  __shared__ float red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * WGM, n0 = blockIdx.x * WGN;
  const int split = blockIdx.z;
  const int kb = split * g.k_per_split;
  const int ke = min(g.K, kb + g.k_per_split);
  // staging: thread t moves 8 elements at K offsets (t%4)*8 + 32 v of tile
  // rows t/4 + 64 i
  const int lr = tid >> 2, lk = (tid & 3) * 8;

  floatx16 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.0f;

  bf16x8 ra[TM][kKVec], rb[TN][kKVec];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int v = 0; v < kKVec; ++v) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
        ra[i][v] = EX ? *reinterpret_cast<const bf16x8*>(g.A + (int64_t)(m0 + lr + 64 * i) * g.lda + k0 + lk + 32 * v)
                      : load8(g.A, g.lda, m0 + lr + 64 * i, g.M, k0 + lk + 32 * v, ke);
#pragma unroll
      for (int i = 0; i < TN; ++i)
        rb[i][v] = EX ? *reinterpret_cast<const bf16x8*>(g.Bt + (int64_t)(n0 + lr + 64 * i) * g.ldb + k0 + lk + 32 * v)
                      : load8(g.Bt, g.ldb, n0 + lr + 64 * i, g.N, k0 + lk + 32 * v, ke);
    }
  };
  fetch(kb);
  int buf = 0;
  for (int k0 = kb; k0 < ke; k0 += kKStep) {
#pragma unroll
    for (int v = 0; v < kKVec; ++v) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
        *reinterpret_cast<bf16x8*>(&As[buf][(lr + 64 * i) * kLdsRow + lk + 32 * v]) = ra[i][v];
#pragma unroll
      for (int i = 0; i < TN; ++i)
        *reinterpret_cast<bf16x8*>(&Bs[buf][(lr + 64 * i) * kLdsRow + lk + 32 * v]) = rb[i][v];
    }
    __syncthreads();
    if (k0 + kKStep < ke) fetch(k0 + kKStep);
#pragma unroll
    for (int s = 0; s < kKStep; s += 16) {
      const int kk = s + (lane >> 5) * 8;
      bf16x8 fa[TM], fb[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a)
        fa[a] = *reinterpret_cast<const bf16x8*>(&As[buf][(wm * 32 * TM + a * 32 + (lane & 31)) * kLdsRow + kk]);
#pragma unroll
      for (int b = 0; b < TN; ++b)
        fb[b] = *reinterpret_cast<const bf16x8*>(&Bs[buf][(wn * 32 * TN + b * 32 + (lane & 31)) * kLdsRow + kk]);
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    buf ^= 1;
  }

  // epilogue: lane holds C[row(r)][col] of each 32 x 32 tile with
  // col = lane % 32, row(r) = (r / 4) * 8 + (lane / 32) * 4 + r % 4
  float sse = 0.0f;
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int col = n0 + wn * 32 * TN + b * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm * 32 * TM + a * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        if (!EX && (row >= g.M || col >= g.N)) continue;
        const float v = acc[a][b][r];
        if (EPI == kEpiWgrad) {
          g.Cf[(int64_t)split * g.M * g.N + (int64_t)row * g.N + col] = v;
        } else if (EPI == kEpiFwdHidden) {
          const float z = v + g.bias[col];
          if (g.Cf) g.Cf[(int64_t)row * g.ldcf + col] = z;
          const float h = gelu_f(z);
          if (g.Cb) g.Cb[(int64_t)row * g.ldcb + col] = to_bf16(h);
          if (g.Ct) g.Ct[(int64_t)col * g.ldct + row] = to_bf16(h);
        } else if (EPI == kEpiFwdOut) {
          const float y = v + g.bias[col];
          if (g.Cf) g.Cf[(int64_t)row * g.ldcf + col] = y;
          if (g.target) {
            const float d = y - g.target[(int64_t)row * g.ldt + col];
            sse = fmaf(d, d, sse);
            const float dy = g.scale * d;
            g.Cb[(int64_t)row * g.ldcb + col] = to_bf16(dy);
            g.Ct[(int64_t)col * g.ldct + row] = to_bf16(dy);
          }
        } else {  // kEpiBwdHidden
          const float d = v * gelu_grad_f(g.gact[(int64_t)row * g.ldg + col]);
          if (g.Cb) g.Cb[(int64_t)row * g.ldcb + col] = to_bf16(d);
          if (g.Ct) g.Ct[(int64_t)col * g.ldct + row] = to_bf16(d);
        }
      }
    }
  if (EPI == kEpiFwdOut && g.target) {
    // fixed-order reduction of the tile's squared errors
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) sse += __shfl_xor(sse, off, 64);
    if (lane == 0) red[wave] = sse;
    __syncthreads();
    if (tid == 0) g.loss_part[blockIdx.y * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
  }
}

template <int EPI, int TM, int TN>
void launch_gemm_t(const GemmArgs& g, int splits, hipStream_t s, int32_t* info) {
  const dim3 grid((g.N + 64 * TN - 1) / (64 * TN), (g.M + 64 * TM - 1) / (64 * TM), splits);
  // every split's K range non-empty and a whole number of stages
  const bool ex = g.M % (64 * TM) == 0 && g.N % (64 * TN) == 0 && g.K > 0 && g.K % kKStep == 0 &&
                  g.k_per_split % kKStep == 0 && (int64_t)g.k_per_split * (splits - 1) < g.K && g.lda % 8 == 0 &&
                  g.ldb % 8 == 0 && reinterpret_cast<uintptr_t>(g.A) % 16 == 0 &&
                  reinterpret_cast<uintptr_t>(g.Bt) % 16 == 0;
  if (ex) hipLaunchKernelGGL((gemm_nt_kernel<EPI, TM, TN, true>), grid, dim3(256), 0, s, g);
  else hipLaunchKernelGGL((gemm_nt_kernel<EPI, TM, TN, false>), grid, dim3(256), 0, s, g);
  if (info) {
    info[0] = 64 * TM;
    info[1] = 64 * TN;
    info[2] = splits;
    info[3] = ex ? 1 : 0;
  }
}

template <int EPI>
void launch_gemm_e(const GemmArgs& g, int splits, hipStream_t s, int32_t* info) {
  // largest tile that still gives at least 256 workgroups; the loss partials
  // of a training forward are laid out per 64 x 64 tile
  const int64_t t22 = (int64_t)((g.N + 127) / 128) * ((g.M + 127) / 128) * splits;
  const int64_t t21 = (int64_t)((g.N + 63) / 64) * ((g.M + 127) / 128) * splits;
  if (EPI == kEpiFwdOut && g.target) launch_gemm_t<EPI, 1, 1>(g, splits, s, info);
  else if (t22 >= 256) launch_gemm_t<EPI, 2, 2>(g, splits, s, info);
  else if (t21 >= 256) launch_gemm_t<EPI, 2, 1>(g, splits, s, info);
  else launch_gemm_t<EPI, 1, 1>(g, splits, s, info);
}

hipError_t launch_gemm(const GemmArgs& g, int epi, int splits, hipStream_t s, int32_t* info) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  (void)hipGetLastError();  // report only this launch's status
  switch (epi) {
    case kEpiWgrad: launch_gemm_e<kEpiWgrad>(g, splits, s, info); break;
    case kEpiFwdHidden: launch_gemm_e<kEpiFwdHidden>(g, splits, s, info); break;
    case kEpiFwdOut: launch_gemm_e<kEpiFwdOut>(g, splits, s, info); break;
    default: launch_gemm_e<kEpiBwdHidden>(g, splits, s, info); break;
  }
  return hipGetLastError();
}

// ---- small kernels --------------------------------------------------------
// FP32 [rows x cols] -> BF16 row-major copy and BF16 transposed copy [cols x rows]
__global__ void pack_bf16_kernel(const float* __restrict__ src, int rows, int cols, __bf16* dst, int ldd,
                                 __bf16* dst_t, int ldt) {
  __shared__ float tile[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 32 x 8
  for (int i = ty; i < 32; i += 8) {
    const int r = r0 + i, c = c0 + tx;
    const float v = (r < rows && c < cols) ? src[(int64_t)r * cols + c] : 0.0f;
    tile[i][tx] = v;
    if (dst && r < rows && c < cols) dst[(int64_t)r * ldd + c] = to_bf16(v);
  }
  __syncthreads();
  if (dst_t)
    for (int i = ty; i < 32; i += 8) {
      const int c = c0 + i, r = r0 + tx;
      if (r < rows && c < cols) dst_t[(int64_t)c * ldt + r] = to_bf16(tile[tx][i]);
    }
}

hipError_t launch_pack(const float* src, int rows, int cols, __bf16* dst, int ldd, __bf16* dst_t, int ldt,
                       hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL(pack_bf16_kernel, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(256), 0, s, src, rows, cols,
                     dst, ldd, dst_t, ldt);
  return hipGetLastError();
}

// Sum of split-K partials in order: out[i] = sum_s part[s][i].
__global__ void splitk_sum_kernel(const float* __restrict__ part, int64_t n, int splits, float* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  float v = 0.0f;
  for (int s = 0; s < splits; ++s) v += part[(int64_t)s * n + i];
  out[i] = v;
}

// Row sums of a BF16 [rows x cols] matrix (bias gradients from transposed
// activation gradients): one wave per row, lane-strided sums, fixed tree.
__global__ void rowsum_kernel(const __bf16* __restrict__ x, int rows, int cols, int ld, float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= rows) return;
  float s = 0.0f;
  for (int c = lane; c < cols; c += 64) s += (float)x[(int64_t)row * ld + c];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) out[row] = s;
}

// Loss from per-tile partial sums, in order.
__global__ void loss_sum_kernel(const float* __restrict__ part, int n, float scale, float* __restrict__ loss) {
  __shared__ float red[256];
  float s = 0.0f;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] * scale;
}

// Adam with bias correction (Kingma and Ba, 2015) on FP32 master weights.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ gr, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float g = gr[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

hipError_t launch_splitk_sum(const float* part, int64_t n, int splits, float* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL(splitk_sum_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, n, splits, out);
  return hipGetLastError();
}

hipError_t launch_rowsum(const __bf16* x, int rows, int cols, int ld, float* out, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL(rowsum_kernel, dim3((rows + 3) / 4), dim3(256), 0, s, x, rows, cols, ld, out);
  return hipGetLastError();
}

hipError_t launch_loss_sum(const float* part, int n, float scale, float* loss, hipStream_t s) {
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(256), 0, s, part, n, scale, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace sugg
