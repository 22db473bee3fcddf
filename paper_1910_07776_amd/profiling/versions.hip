// Profiled versions for the suggestion tool on real MI355X counters.
//
// Two programs, each built in all 2^6 combinations of six binary source
// optimisations (Section 3.3: every subset is a version), run on three inputs
// three times each (Section 5: repeated runs), one after another in a fixed
// order, so a profiler's dispatch list maps to (program, input, run, version):
//
//   program 0  all-pairs gravitational acceleration (regular accesses)
//   program 1  potential from a fixed number of gathered neighbours per target
//              (irregular accesses)
//
//   bit 0  FAST    reciprocal square root instruction instead of 1 / sqrt
//   bit 1  UNROLL  inner loop unrolled four times
//   bit 2  LDS     operands staged through LDS (body tiles / neighbour lists)
//   bit 3  VEC     16-byte loads of (x, y, z, w) instead of four arrays
//   bit 4  FMA     fused multiply-adds instead of separately rounded ones
//   bit 5  TWO     two outputs per thread
//
// The results are not checked: the versions are workloads to profile.  Every
// access is in bounds by construction (sizes are multiples of the tile).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#define CK(x)                                                                     \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      std::fprintf(stderr, "%s at %s:%d\n", hipGetErrorString(e_), __FILE__, __LINE__); \
      std::exit(1);                                                               \
    }                                                                             \
  } while (0)

namespace versions {

constexpr int kThreads = 256;
constexpr int kNbr = 16;                 // neighbours per target (program 1)
constexpr float kEps = 1e-3f;

template <int F> constexpr bool has(int b) { return (F >> b) & 1; }

template <int F>
__device__ __forceinline__ float inv_r(float d2) {
  if constexpr (has<F>(0)) return rsqrtf(d2);
  else return 1.0f / sqrtf(d2);
}

template <int F>
__device__ __forceinline__ float madd(float a, float b, float c) {
  if constexpr (has<F>(4)) return fmaf(a, b, c);
  else return __fadd_rn(__fmul_rn(a, b), c);
}

template <int F>
__device__ __forceinline__ float4 body(const float4* p4, const float* px, const float* py, const float* pz,
                                       const float* pw, int j) {
  if constexpr (has<F>(3)) return p4[j];
  else return make_float4(px[j], py[j], pz[j], pw[j]);
}

template <int F>
__device__ __forceinline__ void interact(float4 bi, float4 bj, float3& a) {
  const float dx = bj.x - bi.x, dy = bj.y - bi.y, dz = bj.z - bi.z;
  const float d2 = madd<F>(dz, dz, madd<F>(dy, dy, madd<F>(dx, dx, kEps)));
  const float ir = inv_r<F>(d2);
  const float s = bj.w * ir * ir * ir;
  a.x = madd<F>(dx, s, a.x);
  a.y = madd<F>(dy, s, a.y);
  a.z = madd<F>(dz, s, a.z);
}

// program 0: a[i] = sum_j m_j (r_j - r_i) / (|r_j - r_i|^2 + eps)^(3/2)
template <int F>
__global__ void __launch_bounds__(kThreads) nbody(const float4* p4, const float* px, const float* py, const float* pz,
                                                  const float* pw, float4* out, int n) {
  constexpr int NO = has<F>(5) ? 2 : 1;
  __shared__ float4 tile[kThreads];
  const int stride = n / NO;                        // n is a multiple of 2 * kThreads
  const int i0 = blockIdx.x * kThreads + threadIdx.x;
  float4 bi[NO];
  float3 a[NO];
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    bi[o] = body<F>(p4, px, py, pz, pw, i0 + o * stride);
    a[o] = make_float3(0.f, 0.f, 0.f);
  }
  for (int t = 0; t < n; t += kThreads) {
    if constexpr (has<F>(2)) {
      __syncthreads();
      tile[threadIdx.x] = body<F>(p4, px, py, pz, pw, t + threadIdx.x);
      __syncthreads();
    }
    if constexpr (has<F>(1)) {
#pragma unroll 4
      for (int j = 0; j < kThreads; ++j) {
        const float4 bj = has<F>(2) ? tile[j] : body<F>(p4, px, py, pz, pw, t + j);
#pragma unroll
        for (int o = 0; o < NO; ++o) interact<F>(bi[o], bj, a[o]);
      }
    } else {
#pragma unroll 1
      for (int j = 0; j < kThreads; ++j) {
        const float4 bj = has<F>(2) ? tile[j] : body<F>(p4, px, py, pz, pw, t + j);
#pragma unroll
        for (int o = 0; o < NO; ++o) interact<F>(bi[o], bj, a[o]);
      }
    }
  }
#pragma unroll
  for (int o = 0; o < NO; ++o) out[i0 + o * stride] = make_float4(a[o].x, a[o].y, a[o].z, 0.f);
}

// program 1: phi[i] = sum_k q_nbr / sqrt(|x_i - x_nbr|^2 + eps) over kNbr
// gathered neighbours nbr[i * kNbr + k] of target i
template <int F>
__global__ void __launch_bounds__(kThreads) gather(const float4* p4, const float* px, const float* py, const float* pz,
                                                   const float* pw, const int* nbr, float* out, int nt) {
  constexpr int NO = has<F>(5) ? 2 : 1;
  __shared__ int lst[NO * kThreads * kNbr];
  const int stride = nt / NO;
  const int i0 = blockIdx.x * kThreads + threadIdx.x;
  if constexpr (has<F>(2)) {
    // the block's neighbour lists, read once in coalesced order
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      const int base = (blockIdx.x * kThreads + o * stride) * kNbr;
      for (int e = threadIdx.x; e < kThreads * kNbr; e += kThreads) lst[o * kThreads * kNbr + e] = nbr[base + e];
    }
    __syncthreads();
  }
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    const int i = i0 + o * stride;
    const float4 bi = body<F>(p4, px, py, pz, pw, i);
    float phi = 0.f;
    auto term = [&](int k) {
      const int j = has<F>(2) ? lst[(o * kThreads + threadIdx.x) * kNbr + k] : nbr[i * kNbr + k];
      const float4 bj = body<F>(p4, px, py, pz, pw, j);
      const float dx = bj.x - bi.x, dy = bj.y - bi.y, dz = bj.z - bi.z;
      const float d2 = madd<F>(dz, dz, madd<F>(dy, dy, madd<F>(dx, dx, kEps)));
      phi = madd<F>(bj.w, inv_r<F>(d2), phi);
    };
    if constexpr (has<F>(1)) {
#pragma unroll 4
      for (int k = 0; k < kNbr; ++k) term(k);
    } else {
#pragma unroll 1
      for (int k = 0; k < kNbr; ++k) term(k);
    }
    out[i] = phi;
  }
}

struct Data {
  float4* p4;
  float *px, *py, *pz, *pw;
  int* nbr;
  float4* out4;
  float* out1;
};

template <int F>
void launch(int prog, const Data& d, int n) {
  constexpr int NO = has<F>(5) ? 2 : 1;
  const dim3 grid((unsigned)(n / NO / kThreads)), block(kThreads);
  if (prog == 0)
    hipLaunchKernelGGL((nbody<F>), grid, block, 0, 0, d.p4, d.px, d.py, d.pz, d.pw, d.out4, n);
  else
    hipLaunchKernelGGL((gather<F>), grid, block, 0, 0, d.p4, d.px, d.py, d.pz, d.pw, d.nbr, d.out1, n);
}

template <int... F>
void launch_any(int S, int prog, const Data& d, int n, std::integer_sequence<int, F...>) {
  ((S == F ? launch<F>(prog, d, n) : void()), ...);
}

}  // namespace versions

int main(int argc, char** argv) {
  using namespace versions;
  const int runs = argc > 1 ? std::atoi(argv[1]) : 3;
  // inputs: bodies for program 0, targets (= sources) for program 1
  const int sizes[2][3] = {{8192, 12288, 16384}, {1 << 18, 1 << 19, 3 << 18}};
  const int nmax = 3 << 18;
  std::vector<float> h(4 * (size_t)nmax);
  std::vector<int> hn((size_t)nmax * kNbr);
  uint64_t s = 1910;
  auto rnd = [&]() {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return (float)((s >> 40) & 0xffffff) / 16777216.0f;
  };
  for (auto& v : h) v = rnd();
  Data d{};
  CK(hipMalloc(&d.p4, sizeof(float4) * nmax));
  CK(hipMalloc(&d.px, sizeof(float) * nmax));
  CK(hipMalloc(&d.py, sizeof(float) * nmax));
  CK(hipMalloc(&d.pz, sizeof(float) * nmax));
  CK(hipMalloc(&d.pw, sizeof(float) * nmax));
  CK(hipMalloc(&d.nbr, sizeof(int) * (size_t)nmax * kNbr));
  CK(hipMalloc(&d.out4, sizeof(float4) * nmax));
  CK(hipMalloc(&d.out1, sizeof(float) * nmax));
  CK(hipMemcpy(d.p4, h.data(), sizeof(float4) * nmax, hipMemcpyHostToDevice));
  std::vector<float> soa((size_t)nmax);
  float* dst[4] = {d.px, d.py, d.pz, d.pw};
  for (int c = 0; c < 4; ++c) {
    for (int i = 0; i < nmax; ++i) soa[i] = h[4 * (size_t)i + c];
    CK(hipMemcpy(dst[c], soa.data(), sizeof(float) * nmax, hipMemcpyHostToDevice));
  }
  for (int prog = 0; prog < 2; ++prog)
    for (int inp = 0; inp < 3; ++inp) {
      const int n = sizes[prog][inp];
      if (prog == 1) {   // neighbours of target i: random sources among the n
        for (size_t e = 0; e < (size_t)n * kNbr; ++e) hn[e] = (int)(rnd() * (float)n) % n;
        CK(hipMemcpy(d.nbr, hn.data(), sizeof(int) * (size_t)n * kNbr, hipMemcpyHostToDevice));
      }
      for (int run = 0; run < runs; ++run)
        for (int S = 0; S < 64; ++S) {
          launch_any(S, prog, d, n, std::make_integer_sequence<int, 64>{});
          CK(hipGetLastError());
          CK(hipDeviceSynchronize());
        }
      std::printf("program %d input %d (n=%d): %d runs x 64 versions\n", prog, inp, n, runs);
      std::fflush(stdout);
    }
  hipFree(d.p4); hipFree(d.px); hipFree(d.py); hipFree(d.pz); hipFree(d.pw);
  hipFree(d.nbr); hipFree(d.out4); hipFree(d.out1);
  return 0;
}
