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

// K per LDS stage (KS, a template parameter: 32, 64 or 128, each stage two to
// eight MFMAs of K 16 per tile); a stage's rows are padded by 8 elements.
template <int KS>
__host__ __device__ constexpr int lds_row() { return KS + 8; }
template <int TM, int TN, int KS>
__host__ __device__ constexpr size_t gemm_lds_bytes() {
  // operand stages, or the BF16 output tile of the epilogue if larger
  return sizeof(__bf16) * (2 * 64 * (TM + TN) * lds_row<KS>() > 64 * TM * (64 * TN + 8)
                               ? 2 * 64 * (TM + TN) * lds_row<KS>()
                               : 64 * TM * (64 * TN + 8));
}

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }

// erf by Abramowitz and Stegun, Handbook of Mathematical Functions, formula
// 7.1.26: erf(a) = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) e^(-a^2) with
// t = 1 / (1 + p a) for a >= 0 (odd extension below 0), absolute error at
// most 1.5e-7 in exact arithmetic; in FP32 (hardware reciprocal and
// exponential) a few units of 1e-7 more, far below the BF16 rounding of
// every output it feeds.  Two transcendental and six fused operations in
// place of the library's erff.
__device__ __forceinline__ float erf_as(float x) {
  const float a = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, a, 1.0f));
  const float poly =
      t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f), 0.254829592f);
  return copysignf(1.0f - poly * __expf(-a * a), x);
}
__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erf_as(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erf_as(x * 0.70710678118654752f)) + x * 0.39894228040143268f * __expf(-0.5f * x * x);
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

// Tier 3 of the output rows held in an LDS tile y [rows x ldy]: thread t
// takes row t / 2 and half t % 2 of its W columns (columns >= skip), keeps a
// best-first list of KT, merges it with its partner's and writes the row's
// top n (as rank_kernel: -1 / NaN padded, count).
template <int KT, int W>
__device__ __forceinline__ void rank_rows(const GemmArgs& g, const float* y, int ldy, int m0, int tid, bool exact) {
  const int r = tid >> 1, half = tid & 1, row = m0 + r;
  Entry<float> lst[KT];
#pragma unroll
  for (int i = 0; i < KT; ++i) lst[i] = empty_entry<float>();
  const int c0 = half * (W / 2);
  for (int c = c0 < g.skip ? g.skip : c0; c < c0 + W / 2; ++c) {
    const float v = y[r * ldy + c];
    if (v > g.tau) {
      Entry<float> e;
      e.v = v;
      e.s = c;
      list_insert<float, KT>(lst, e);
    }
  }
  group_merge<float, KT>(lst, 2);
  if (half == 0 && (exact || row < g.M)) {
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < KT; ++i)
      if (i < g.n) {
        const bool ok = lst[i].s >= 0;
        g.idx_out[(int64_t)row * g.n + i] = ok ? lst[i].s : -1;
        g.score_out[(int64_t)row * g.n + i] = ok ? lst[i].v : __builtin_nanf("");
        cnt += ok ? 1 : 0;
      }
    g.count_out[row] = cnt;
  }
}

// Workgroup of 4 waves in a 2 x 2 arrangement; each wave computes TM x TN
// MFMA tiles of 32 x 32, so the workgroup tile is (64 TM) x (64 TN).  EX: the
// tiles cover M, N and each K range exactly and rows are 16-byte aligned, so
// operand loads and output stores need no bounds checks.
// One workgroup's tile (bx, by) of split bz; gx: tiles along N (the loss
// partials are laid out per tile); gsm: the dynamic LDS.
template <int EPI, int TM, int TN, bool EX, int KS>
__device__ __forceinline__ void gemm_nt_tile(const GemmArgs& g, int bx, int by, int bz, int gx, unsigned char* gsm) {
  constexpr int WGM = 64 * TM, WGN = 64 * TN;
  constexpr int kKVec = KS / 32;          // 8-element vectors per thread and tile row per stage
  constexpr int kLdsRow = lds_row<KS>();
  __bf16 (*As)[WGM * kLdsRow] = reinterpret_cast<__bf16 (*)[WGM * kLdsRow]>(gsm);
  __bf16 (*Bs)[WGN * kLdsRow] = reinterpret_cast<__bf16 (*)[WGN * kLdsRow]>(gsm + sizeof(__bf16) * 2 * WGM * kLdsRow);
  __shared__ float red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = by * WGM, n0 = bx * WGN;
  const int split = bz;
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

  // Two stages in flight in registers: stage s is written to LDS buffer s % 2
  // while the loads of stage s + 1 are still outstanding, then the loads of
  // stage s + 2 are issued and stage s is multiplied, so a global load has two
  // stages of matrix work to arrive.  Every load is unconditional (the K
  // offset clamped to the last stage; the surplus loads are not used), so
  // each wait is for one stage's loads, never for all of them.
  bf16x8 ra[2][TM][kKVec], rb[2][TN][kKVec];
  const int nst = ke > kb ? (ke - kb + KS - 1) / KS : 0;   // stages of this split
  const int klast = nst > 0 ? kb + (nst - 1) * KS : kb;     // (an empty split loads nothing: k >= ke)
  auto fetch = [&](auto slot, int k0) {
    constexpr int sl = decltype(slot)::value;
    k0 = k0 < klast ? k0 : klast;
#pragma unroll
    for (int v = 0; v < kKVec; ++v) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
        ra[sl][i][v] = EX ? *reinterpret_cast<const bf16x8*>(g.A + (int64_t)(m0 + lr + 64 * i) * g.lda + k0 + lk + 32 * v)
                          : load8(g.A, g.lda, m0 + lr + 64 * i, g.M, k0 + lk + 32 * v, ke);
#pragma unroll
      for (int i = 0; i < TN; ++i)
        rb[sl][i][v] = EX ? *reinterpret_cast<const bf16x8*>(g.Bt + (int64_t)(n0 + lr + 64 * i) * g.ldb + k0 + lk + 32 * v)
                          : load8(g.Bt, g.ldb, n0 + lr + 64 * i, g.N, k0 + lk + 32 * v, ke);
    }
  };
  // one stage: registers of `slot` into LDS buffer `slot`, the loads of the
  // stage two ahead, the products of this one
  auto run_stage = [&](auto slot, int k0) {
    constexpr int sl = decltype(slot)::value;
#pragma unroll
    for (int v = 0; v < kKVec; ++v) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
        *reinterpret_cast<bf16x8*>(&As[sl][(lr + 64 * i) * kLdsRow + lk + 32 * v]) = ra[sl][i][v];
#pragma unroll
      for (int i = 0; i < TN; ++i)
        *reinterpret_cast<bf16x8*>(&Bs[sl][(lr + 64 * i) * kLdsRow + lk + 32 * v]) = rb[sl][i][v];
    }
    __syncthreads();
    fetch(slot, k0 + 2 * KS);
#pragma unroll
    for (int s = 0; s < KS; s += 16) {
      const int kk = s + (lane >> 5) * 8;
      bf16x8 fa[TM], fb[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a)
        fa[a] = *reinterpret_cast<const bf16x8*>(&As[sl][(wm * 32 * TM + a * 32 + (lane & 31)) * kLdsRow + kk]);
#pragma unroll
      for (int b = 0; b < TN; ++b)
        fb[b] = *reinterpret_cast<const bf16x8*>(&Bs[sl][(wn * 32 * TN + b * 32 + (lane & 31)) * kLdsRow + kk]);
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
  };
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  fetch(S0{}, kb);
  fetch(S1{}, kb + KS);
  int st = 0;
  for (; st + 2 <= nst; st += 2) {
    run_stage(S0{}, kb + st * KS);
    run_stage(S1{}, kb + (st + 1) * KS);
  }
  if (st < nst) run_stage(S0{}, kb + st * KS);

  // epilogue: lane holds C[row(r)][col] of each 32 x 32 tile with
  // col = lane % 32, row(r) = (r / 4) * 8 + (lane / 32) * 4 + r % 4.  FP32
  // outputs are written from there (each half-wave 128 contiguous bytes);
  // BF16 outputs go through an LDS copy of the tile, from which the
  // row-major copy and the transposed copy are written 16 bytes per thread
  // (so the transposed one is as coalesced as the row-major one).
  constexpr int TLD = WGN + 8;
  __bf16* T = reinterpret_cast<__bf16*>(gsm);
  const bool stage = EPI != kEpiWgrad && (g.Cb || g.Ct);
  // every input of the epilogue (bias, pre-activation, target) is loaded
  // before its first store, all loads in flight together (a load after a
  // store to memory that might alias it would wait for that store)
  float bcol[TN], pre[TM][TN][16];
  if (EPI == kEpiFwdHidden || EPI == kEpiFwdOut || EPI == kEpiFwdRank) {
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int col = n0 + wn * 32 * TN + b * 32 + (lane & 31);
      bcol[b] = (EX || col < g.N) ? g.bias[col] : 0.0f;
    }
  }
  if (EPI == kEpiBwdHidden || (EPI == kEpiFwdOut && g.target)) {
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm * 32 * TM + a * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        const bool rok = EX || row < g.M;
        int64_t src = row;
        if (EPI == kEpiFwdOut && g.trow && rok) src = g.trow[row];
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          const int col = n0 + wn * 32 * TN + b * 32 + (lane & 31);
          const bool ok = rok && (EX || col < g.N);
          if (EPI == kEpiBwdHidden) pre[a][b][r] = ok ? g.gact[src * g.ldg + col] : 0.0f;
          else pre[a][b][r] = ok ? g.target[src * g.ldt + col] : 0.0f;
        }
      }
  }
  if (stage || EPI == kEpiFwdRank) __syncthreads();   // every wave is done with the operand tiles
  float* Ty = reinterpret_cast<float*>(gsm);           // kEpiFwdRank: the FP32 tile
  constexpr int YLD = WGN + 1;
  float sse = 0.0f;
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int tc = wn * 32 * TN + b * 32 + (lane & 31);
      const int col = n0 + tc;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int tr = wm * 32 * TM + a * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        const int row = m0 + tr;
        if (!EX && (row >= g.M || col >= g.N)) continue;
        const float v = acc[a][b][r];
        float o = 0.0f;   // the BF16 output
        if (EPI == kEpiWgrad) {
          g.Cf[(int64_t)split * g.M * g.N + (int64_t)row * g.N + col] = v;
        } else if (EPI == kEpiFwdHidden) {
          const float z = v + bcol[b];
          if (g.Cf) g.Cf[(int64_t)row * g.ldcf + col] = z;
          o = gelu_f(z);
        } else if (EPI == kEpiFwdOut) {
          const float y = v + bcol[b];
          if (g.Cf) g.Cf[(int64_t)row * g.ldcf + col] = y;
          if (g.target) {
            const float d = y - pre[a][b][r];
            sse = fmaf(d, d, sse);
            o = g.scale * d;
          }
        } else if (EPI == kEpiFwdRank) {
          const float y = v + bcol[b];
          if (g.Cf) g.Cf[(int64_t)row * g.ldcf + col] = y;
          Ty[tr * YLD + tc] = y;
        } else {  // kEpiBwdHidden
          o = v * gelu_grad_f(pre[a][b][r]);
        }
        if (stage) T[tr * TLD + tc] = to_bf16(o);
      }
    }
  if (stage) {
    __syncthreads();
    const int mr = min(WGM, g.M - m0), nc = min(WGN, g.N - n0);   // the tile's valid extent
    if (g.Cb) {
      const bool vec = reinterpret_cast<uintptr_t>(g.Cb) % 16 == 0 && g.ldcb % 8 == 0;
      for (int v = tid; v < WGM * (WGN / 8); v += 256) {
        const int r = v / (WGN / 8), c = (v % (WGN / 8)) * 8;
        if (r >= mr) continue;
        __bf16* dst = g.Cb + (int64_t)(m0 + r) * g.ldcb + n0 + c;
        if (vec && c + 8 <= nc) {
          *reinterpret_cast<bf16x8*>(dst) = *reinterpret_cast<const bf16x8*>(T + r * TLD + c);
        } else {
          for (int i = 0; i < 8 && c + i < nc; ++i) dst[i] = T[r * TLD + c + i];
        }
      }
    }
    if (g.Ct) {
      const bool vec = reinterpret_cast<uintptr_t>(g.Ct) % 16 == 0 && g.ldct % 8 == 0;
      for (int v = tid; v < WGN * (WGM / 8); v += 256) {
        const int c = v / (WGM / 8), r = (v % (WGM / 8)) * 8;
        if (c >= nc) continue;
        __bf16* dst = g.Ct + (int64_t)(n0 + c) * g.ldct + m0 + r;
        if (vec && r + 8 <= mr) {
          bf16x8 q;
#pragma unroll
          for (int i = 0; i < 8; ++i) q[i] = T[(r + i) * TLD + c];
          *reinterpret_cast<bf16x8*>(dst) = q;
        } else {
          for (int i = 0; i < 8 && r + i < mr; ++i) dst[i] = T[(r + i) * TLD + c];
        }
      }
    }
  }
  if constexpr (EPI == kEpiFwdRank) {
    // two threads per row of the tile (the row's N = WGN outputs), each a
    // best-first list of its half (value descending, column ascending), the
    // pair's lists merged; lists of 4 where n <= 4
    static_assert(WGM * 2 == 256, "two threads per tile row");
    __syncthreads();
    if (g.n <= 4) rank_rows<4, WGN>(g, Ty, YLD, m0, tid, EX);
    else rank_rows<kMaxSuggest, WGN>(g, Ty, YLD, m0, tid, EX);
  }
  if (EPI == kEpiFwdOut && g.target) {
    // fixed-order reduction of the tile's squared errors
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) sse += __shfl_xor(sse, off, 64);
    if (lane == 0) red[wave] = sse;
    __syncthreads();
    if (tid == 0) g.loss_part[by * gx + bx] = ((red[0] + red[1]) + red[2]) + red[3];
  }
}

// The tile (bx, by) of the i-th workgroup of an nx x ny grid.  Workgroups go
// to the eight XCDs in turn (i mod 8); where ny is a multiple of 8 (and the
// grid starts on XCD 0), the nx tiles of a row block all go to one XCD, so
// the block's A rows are fetched into that XCD's L2 once and used nx times
// there (in row-major order each went to another XCD and was fetched nx
// times).  The tiles and their arithmetic are the same either way.
__device__ __forceinline__ void xcd_tile(int i, int nx, int ny, bool xcd, int& bx, int& by) {
  if (xcd && ny % 8 == 0) {
    const int x = i % 8, s = i / 8;
    by = x + 8 * (s / nx);
    bx = s % nx;
  } else {
    by = i / nx;
    bx = i % nx;
  }
}

template <int EPI, int TM, int TN, bool EX, int KS>
__global__ void __launch_bounds__(256, 2) gemm_nt_kernel(const GemmArgs g) {
  extern __shared__ __align__(16) unsigned char gsm[];
  int bx, by;
  xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x, gridDim.y, true, bx, by);
  gemm_nt_tile<EPI, TM, TN, EX, KS>(g, bx, by, blockIdx.z, gridDim.x, gsm);
}

// Two independent GEMMs in one launch (workgroups [0, n1) take the first,
// the rest the second), each tile computed exactly as by its own launch.
struct GemmGrid {
  int nx, ny, nz;
};
template <int E1, int TM1, int TN1, bool EX1, int KS1, int E2, int TM2, int TN2, bool EX2, int KS2>
__global__ void __launch_bounds__(256, 2) gemm_pair_kernel(const GemmArgs g1, const GemmGrid d1, const GemmArgs g2,
                                                         const GemmGrid d2) {
  extern __shared__ __align__(16) unsigned char gsm[];
  const int n1 = d1.nx * d1.ny * d1.nz;
  int b = blockIdx.x, bx, by;
  if (b < n1) {
    const int xy = d1.nx * d1.ny, z = b / xy, r = b - z * xy;
    xcd_tile(r, d1.nx, d1.ny, true, bx, by);
    gemm_nt_tile<E1, TM1, TN1, EX1, KS1>(g1, bx, by, z, d1.nx, gsm);
  } else {
    b -= n1;
    const int xy = d2.nx * d2.ny, z = b / xy, r = b - z * xy;
    xcd_tile(r, d2.nx, d2.ny, n1 % 8 == 0, bx, by);
    gemm_nt_tile<E2, TM2, TN2, EX2, KS2>(g2, bx, by, z, d2.nx, gsm);
  }
}

// LDS bytes of an instance (the ranking epilogue keeps the FP32 output tile,
// rows padded by one)
template <int EPI, int TM, int TN, int KS>
constexpr size_t gemm_lds() {
  constexpr size_t ty = EPI == kEpiFwdRank ? sizeof(float) * 64 * TM * (64 * TN + 1) : 0;
  return gemm_lds_bytes<TM, TN, KS>() > ty ? gemm_lds_bytes<TM, TN, KS>() : ty;
}

template <int EPI, int TM, int TN, bool EX, int KS>
hipError_t launch_gemm_k(const GemmArgs& g, dim3 grid, hipStream_t s) {
  constexpr size_t lds = gemm_lds<EPI, TM, TN, KS>();
  auto kern = gemm_nt_kernel<EPI, TM, TN, EX, KS>;
  if (lds > 64 * 1024) {
    static const hipError_t attr =
        hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess) return attr;
  }
  hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, g);
  return hipSuccess;
}

// The instance a GEMM runs: workgroup tile (64 tm) x (64 tn), K stage ks,
// exact tiles (no bounds checks).
struct GemmPick {
  int tm, tn, ks;
  bool ex;
  bool operator==(const GemmPick& o) const { return tm == o.tm && tn == o.tn && ks == o.ks && ex == o.ex; }
};

// K stage: 32 for 128 x 128 workgroup tiles (three workgroups fit a compute
// unit's LDS); for smaller tiles 128 where every split's K range is a
// multiple of 128, else 64 where a multiple of 64, else 32.  The ranking
// epilogue stops at 64: its 128 x 64 tiles then fit two workgroups per
// compute unit (a surrogate pass over 65,536 kernels took 140 instead of
// 157 us).
GemmPick pick_ks(int epi, const GemmArgs& g, int splits, int TM, int TN) {
  const bool k128 = g.K % 128 == 0 && g.k_per_split % 128 == 0 && epi != kEpiFwdRank;
  const int ks = TM * TN > 2 ? 32   // 128 x 128 tiles: three workgroups per compute unit
                 : k128 ? 128
                 : (g.K % 64 == 0 && g.k_per_split % 64 == 0) ? 64 : 32;
  // every split's K range non-empty and a whole number of stages
  const bool ex = g.M % (64 * TM) == 0 && g.N % (64 * TN) == 0 && g.K > 0 && g.K % ks == 0 &&
                  g.k_per_split % ks == 0 && (int64_t)g.k_per_split * (splits - 1) < g.K && g.lda % 8 == 0 &&
                  g.ldb % 8 == 0 && reinterpret_cast<uintptr_t>(g.A) % 16 == 0 &&
                  reinterpret_cast<uintptr_t>(g.Bt) % 16 == 0;
  return GemmPick{TM, TN, ex ? ks : 32, ex};
}

// largest tile that still gives at least 256 workgroups (128 columns only
// where they divide N; a hidden layer's forward takes 128 x 64 tiles only
// from 512 workgroups: at the training batch 4096 its 64 x 64 tiles made a
// step 3 % faster); the loss partials of a training forward are laid out per
// 64 x 64 tile
GemmPick pick_gemm(int epi, const GemmArgs& g, int splits) {
  const int64_t t22 = (int64_t)((g.N + 127) / 128) * ((g.M + 127) / 128) * splits;
  const int64_t t21 = (int64_t)((g.N + 63) / 64) * ((g.M + 127) / 128) * splits;
  if (epi == kEpiFwdOut && g.target) return pick_ks(epi, g, splits, 1, 1);
  if (t22 >= 256 && g.N % 128 == 0) return pick_ks(epi, g, splits, 2, 2);
  if (t21 >= (epi == kEpiFwdHidden ? 512 : 256)) return pick_ks(epi, g, splits, 2, 1);
  return pick_ks(epi, g, splits, 1, 1);
}

GemmGrid gemm_grid(const GemmArgs& g, const GemmPick& p, int splits) {
  return GemmGrid{(g.N + 64 * p.tn - 1) / (64 * p.tn), (g.M + 64 * p.tm - 1) / (64 * p.tm), splits};
}

void gemm_info(const GemmPick& p, int splits, int32_t* info) {
  if (!info) return;
  info[0] = 64 * p.tm;
  info[1] = 64 * p.tn;
  info[2] = splits;
  info[3] = p.ex ? p.ks : 0;
}

template <int EPI, int TM, int TN>
hipError_t launch_gemm_t(const GemmArgs& g, int splits, hipStream_t s, int32_t* info) {
  const GemmPick p = pick_ks(EPI, g, splits, TM, TN);
  const GemmGrid d = gemm_grid(g, p, splits);
  const dim3 grid(d.nx, d.ny, d.nz);
  hipError_t e;
  if (p.ex && p.ks == 128) e = launch_gemm_k<EPI, TM, TN, true, 128>(g, grid, s);
  else if (p.ex && p.ks == 64) e = launch_gemm_k<EPI, TM, TN, true, 64>(g, grid, s);
  else if (p.ex) e = launch_gemm_k<EPI, TM, TN, true, 32>(g, grid, s);
  else e = launch_gemm_k<EPI, TM, TN, false, 32>(g, grid, s);
  gemm_info(p, splits, info);
  return e;
}

template <int EPI>
hipError_t launch_gemm_e(const GemmArgs& g, int splits, hipStream_t s, int32_t* info) {
  const GemmPick p = pick_gemm(EPI, g, splits);
  if (p.tm == 2 && p.tn == 2) return launch_gemm_t<EPI, 2, 2>(g, splits, s, info);
  if (p.tm == 2) return launch_gemm_t<EPI, 2, 1>(g, splits, s, info);
  return launch_gemm_t<EPI, 1, 1>(g, splits, s, info);
}

template <int E1, int TM1, int TN1, int KS1, int E2, int TM2, int TN2, int KS2>
hipError_t launch_pair_k(const GemmArgs& g1, const GemmGrid& d1, const GemmArgs& g2, const GemmGrid& d2,
                         hipStream_t s) {
  constexpr size_t l1 = gemm_lds<E1, TM1, TN1, KS1>(), l2 = gemm_lds<E2, TM2, TN2, KS2>();
  constexpr size_t lds = l1 > l2 ? l1 : l2;
  auto kern = gemm_pair_kernel<E1, TM1, TN1, true, KS1, E2, TM2, TN2, true, KS2>;
  if (lds > 64 * 1024) {
    static const hipError_t attr =
        hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess) return attr;
  }
  const int n = d1.nx * d1.ny * d1.nz + d2.nx * d2.ny * d2.nz;
  hipLaunchKernelGGL(kern, dim3(n), dim3(256), lds, s, g1, d1, g2, d2);
  return hipSuccess;
}

hipError_t launch_gemm_rank(const GemmArgs& g, hipStream_t s, int32_t* info) {
  if (g.M <= 0) return hipSuccess;
  if ((g.N != 64 && g.N != 128) || g.n < 1 || g.n > kMaxSuggest || g.skip < 0) return hipErrorInvalidValue;
  (void)hipGetLastError();  // report only this launch's status
  const hipError_t e = g.N == 64 ? launch_gemm_t<kEpiFwdRank, 2, 1>(g, 1, s, info)
                                 : launch_gemm_t<kEpiFwdRank, 2, 2>(g, 1, s, info);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

// A weight gradient (split over K) and a hidden-layer backward in one launch
// where both run the instances of the surrogate's training shapes (a 64 x 64
// weight-gradient tile with K stage 128; a 128 x 64 backward tile with K
// stage 64 or 128), else in two launches; the results are the same.
hipError_t launch_gemm_pair(const GemmArgs& gw, int splits, const GemmArgs& gb, hipStream_t s, int32_t* info_w,
                            int32_t* info_b) {
  const GemmPick pw = pick_gemm(kEpiWgrad, gw, splits), pb = pick_gemm(kEpiBwdHidden, gb, 1);
  const bool live_w = gw.M > 0 && gw.N > 0, live_b = gb.M > 0 && gb.N > 0;
  const bool w_ok = pw == GemmPick{1, 1, 128, true};
  const bool b64 = pb == GemmPick{2, 1, 64, true}, b128 = pb == GemmPick{2, 1, 128, true};
  if (live_w && live_b && w_ok && (b64 || b128)) {
    (void)hipGetLastError();  // report only this launch's status
    const GemmGrid dw = gemm_grid(gw, pw, splits), db = gemm_grid(gb, pb, 1);
    const hipError_t e = b64 ? launch_pair_k<kEpiWgrad, 1, 1, 128, kEpiBwdHidden, 2, 1, 64>(gw, dw, gb, db, s)
                             : launch_pair_k<kEpiWgrad, 1, 1, 128, kEpiBwdHidden, 2, 1, 128>(gw, dw, gb, db, s);
    if (e != hipSuccess) return e;
    gemm_info(pw, splits, info_w);
    gemm_info(pb, 1, info_b);
    return hipGetLastError();
  }
  hipError_t e = launch_gemm(gw, kEpiWgrad, splits, s, info_w);
  if (e == hipSuccess) e = launch_gemm(gb, kEpiBwdHidden, 1, s, info_b);
  return e;
}

hipError_t launch_gemm(const GemmArgs& g, int epi, int splits, hipStream_t s, int32_t* info) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  (void)hipGetLastError();  // report only this launch's status
  hipError_t e;
  switch (epi) {
    case kEpiWgrad: e = launch_gemm_e<kEpiWgrad>(g, splits, s, info); break;
    case kEpiFwdHidden: e = launch_gemm_e<kEpiFwdHidden>(g, splits, s, info); break;
    case kEpiFwdOut: e = launch_gemm_e<kEpiFwdOut>(g, splits, s, info); break;
    default: e = launch_gemm_e<kEpiBwdHidden>(g, splits, s, info); break;
  }
  if (e != hipSuccess) return e;
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

// pack_bf16_kernel of the rows idx[0..rows) of src (one read per element):
// the 32 x 32 tile (bx, by)
__device__ __forceinline__ void gather_pack_tile(const GatherArgs& g, int bx, int by) {
  __shared__ float tile[32][33];
  __shared__ int64_t srow[32];
  const int r0 = by * 32, c0 = bx * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  if (threadIdx.x < 32) {
    const int r = r0 + threadIdx.x;
    int64_t q = 0;
    if (r < g.rows) {
      q = g.idx[r];
      if (q < 0 || q >= g.src_rows) {
        atomicOr(g.status, (int)kStatusBadIndex);
        q = 0;
      }
      if (bx == 0) g.rows_out[r] = (int32_t)q;
    }
    srow[threadIdx.x] = q;
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int r = r0 + i, c = c0 + tx;
    const float v = (r < g.rows && c < g.cols) ? g.src[srow[i] * g.cols + c] : 0.0f;
    tile[i][tx] = v;
    if (r < g.rows && c < g.cols) g.dst[(int64_t)r * g.ldd + c] = to_bf16(v);
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int c = c0 + i, r = r0 + tx;
    if (r < g.rows && c < g.cols) g.dst_t[(int64_t)c * g.ldt + r] = to_bf16(tile[tx][i]);
  }
}

__global__ void __launch_bounds__(256) gather_pack_kernel(const GatherArgs g) {
  gather_pack_tile(g, blockIdx.x, blockIdx.y);
}

hipError_t launch_gather_pack(const GatherArgs& g, hipStream_t s) {
  if (g.rows <= 0 || g.cols <= 0) return hipSuccess;
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL(gather_pack_kernel, dim3((g.cols + 31) / 32, (g.rows + 31) / 32), dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_pack(const float* src, int rows, int cols, __bf16* dst, int ldd, __bf16* dst_t, int ldt,
                       hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL(pack_bf16_kernel, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(256), 0, s, src, rows, cols,
                     dst, ldd, dst_t, ldt);
  return hipGetLastError();
}

// The end of a weight gradient: its blocks [0, nsum) sum the split-K
// partials in split order (256 outputs each), the others take the row sums of
// the transposed activation gradient (its bias gradient), 4 rows each.
__device__ __forceinline__ int64_t wgrad_nsum(const WgradJob& j) { return (j.n + 255) / 256; }
__device__ __forceinline__ int64_t wgrad_blocks(const WgradJob& j) { return wgrad_nsum(j) + (j.rows + 3) / 4; }

__device__ __forceinline__ void wgrad_finish_block(const WgradJob& j, int b) {
  const int nsum = (int)wgrad_nsum(j);
  if (b < nsum) {
    const int64_t i = b * (int64_t)blockDim.x + threadIdx.x;
    if (i >= j.n) return;
    float v = 0.0f;
    for (int q = 0; q < j.splits; ++q) v += j.part[(int64_t)q * j.n + i];
    j.out[i] = v;
    return;
  }
  const int lane = threadIdx.x & 63;
  const int row = (b - nsum) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= j.rows) return;
  // lane sums of 8 consecutive elements per 512 (eight loads in flight),
  // then the lane tree: one fixed order
  const __bf16* xr = j.x + (int64_t)row * j.ld;
  float sm = 0.0f;
  const bool vec = (j.ld % 8) == 0 && (reinterpret_cast<uintptr_t>(j.x) % 16) == 0;
  int c0 = 0;
  if (vec) {
    for (; c0 + 512 * 8 <= j.cols; c0 += 512 * 8) {
      bf16x8 q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) q[u] = *reinterpret_cast<const bf16x8*>(xr + c0 + 512 * u + lane * 8);
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int i = 0; i < 8; ++i) sm += (float)q[u][i];
    }
    for (; c0 + 512 <= j.cols; c0 += 512) {
      const bf16x8 q = *reinterpret_cast<const bf16x8*>(xr + c0 + lane * 8);
#pragma unroll
      for (int i = 0; i < 8; ++i) sm += (float)q[i];
    }
  }
  for (int c = c0 + lane; c < j.cols; c += 64) sm += (float)xr[c];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) sm += __shfl_xor(sm, off, 64);
  if (lane == 0) j.bias_out[row] = sm;
}

// Loss from per-tile partial sums, in order (one block of 256 threads).
__device__ __forceinline__ void loss_block(const float* __restrict__ part, int n, float scale,
                                           float* __restrict__ loss) {
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

// Blocks go to the jobs in order, then one block to the loss.
__global__ void __launch_bounds__(256) wgrad_finish_kernel(const FinishArgs a) {
  int b = blockIdx.x;
  for (int q = 0; q < a.njobs; ++q) {
    const int nb = (int)wgrad_blocks(a.job[q]);
    if (b < nb) {
      wgrad_finish_block(a.job[q], b);
      return;
    }
    b -= nb;
  }
  if (a.loss) loss_block(a.loss_part, a.loss_n, a.loss_scale, a.loss);
}

hipError_t launch_wgrad_finish(const FinishArgs& a, hipStream_t s) {
  int64_t blocks = a.loss ? 1 : 0;
  for (int q = 0; q < a.njobs; ++q) blocks += (a.job[q].n + 255) / 256 + (a.job[q].rows + 3) / 4;
  if (blocks <= 0) return hipSuccess;
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL(wgrad_finish_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) loss_sum_kernel(const float* __restrict__ part, int n, float scale,
                                                       float* __restrict__ loss) {
  loss_block(part, n, scale, loss);
}

// Adam with bias correction (Kingma and Ba, 2015) on FP32 master weights:
// one parameter, returns its new value (the one expression both Adam
// kernels use).
__device__ __forceinline__ float adam_update(float* __restrict__ p, const float* __restrict__ gr,
                                             float* __restrict__ m, float* __restrict__ v, int64_t i, float lr,
                                             float b1, float b2, float eps, float c1, float c2) {
  const float g = gr[i];
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float pn = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pn;
  return pn;
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ gr, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    (void)adam_update(p, gr, m, v, i, lr, b1, b2, eps, c1, c2);
}

// Adam over the flat parameters with the three weight matrices' BF16 working
// copies written from the updated values: blocks [0, tiles) take 32 x 32
// tiles of the matrices (layer after layer, row-major tile order), updating
// them and writing the row-major copy directly and the transposed copy
// through LDS; the remaining blocks update every other parameter (the
// biases), 256 per block.
__device__ __forceinline__ void adam_pack_block(const AdamPackArgs& a, int tiles0, int tiles1, int tiles2, int b) {
  __shared__ float tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 32 x 8
  const int tl[3] = {tiles0, tiles1, tiles2};
  int l = 0;
  while (l < 3 && b >= tl[l]) b -= tl[l++];
  if (l < 3) {
    const int R = a.rows[l], Cc = a.cols[l], tcols = (Cc + 31) / 32;
    const int r0 = (b / tcols) * 32, c0 = (b % tcols) * 32;
    for (int i = ty; i < 32; i += 8) {
      const int r = r0 + i, c = c0 + tx;
      float w = 0.0f;
      if (r < R && c < Cc) {
        w = adam_update(a.p, a.g, a.m, a.v, a.off[l] + (int64_t)r * Cc + c, a.lr, a.b1, a.b2, a.eps, a.c1, a.c2);
        a.w[l][(int64_t)r * Cc + c] = (__bf16)w;
      }
      tile[i][tx] = w;
    }
    if (a.wt[l]) {
      __syncthreads();
      for (int i = ty; i < 32; i += 8) {
        const int c = c0 + i, r = r0 + tx;
        if (r < R && c < Cc) a.wt[l][(int64_t)c * R + r] = (__bf16)tile[tx][i];
      }
    }
    return;
  }
  // the rest: parameters outside the three matrices, in order
  const int64_t j = (int64_t)b * 256 + threadIdx.x;
  int64_t i = j;
  for (int q = 0; q < 3; ++q) {   // skip the matrices that come before
    const int64_t sz = (int64_t)a.rows[q] * a.cols[q];
    if (i >= a.off[q]) i += sz;
  }
  if (i < a.n) (void)adam_update(a.p, a.g, a.m, a.v, i, a.lr, a.b1, a.b2, a.eps, a.c1, a.c2);
}

__global__ void __launch_bounds__(256) adam_pack_kernel(const AdamPackArgs a, int tiles0, int tiles1, int tiles2) {
  adam_pack_block(a, tiles0, tiles1, tiles2, blockIdx.x);
}

// Adam of one step and the gather of the next mini-batch (which does not
// depend on it) in one launch: blocks [0, n_adam) update, the rest gather.
__global__ void __launch_bounds__(256) adam_gather_kernel(const AdamPackArgs a, int tiles0, int tiles1, int tiles2,
                                                          int n_adam, const GatherArgs g, int gx) {
  const int b = blockIdx.x;
  if (b < n_adam) adam_pack_block(a, tiles0, tiles1, tiles2, b);
  else gather_pack_tile(g, (b - n_adam) % gx, (b - n_adam) / gx);
}

namespace {
// bias corrections of the step and the block counts of the three matrices'
// tiles and of the remaining parameters
int adam_pack_setup(AdamPackArgs& a, int step, int (&t)[3]) {
  a.c1 = 1.0f - powf(a.b1, (float)step);
  a.c2 = 1.0f - powf(a.b2, (float)step);
  int64_t inside = 0;
  for (int l = 0; l < 3; ++l) {
    t[l] = ((a.rows[l] + 31) / 32) * ((a.cols[l] + 31) / 32);
    inside += (int64_t)a.rows[l] * a.cols[l];
  }
  const int64_t rest = a.n - inside;
  return t[0] + t[1] + t[2] + (int)((rest + 255) / 256);
}
}  // namespace

hipError_t launch_adam_pack(const AdamPackArgs& a0, int step, hipStream_t s) {
  AdamPackArgs a = a0;
  int t[3];
  const int blocks = adam_pack_setup(a, step, t);
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL(adam_pack_kernel, dim3(blocks), dim3(256), 0, s, a, t[0], t[1], t[2]);
  return hipGetLastError();
}

hipError_t launch_adam_gather(const AdamPackArgs& a0, int step, const GatherArgs& g, hipStream_t s) {
  if (g.rows <= 0 || g.cols <= 0) return launch_adam_pack(a0, step, s);
  AdamPackArgs a = a0;
  int t[3];
  const int n_adam = adam_pack_setup(a, step, t);
  const int gx = (g.cols + 31) / 32, gy = (g.rows + 31) / 32;
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL(adam_gather_kernel, dim3(n_adam + gx * gy), dim3(256), 0, s, a, t[0], t[1], t[2], n_adam, g, gx);
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
