// The fused scoring kernel: normalise -> predict -> compose -> rank.
//
// Section 2's three tiers applied to a ragged batch of kernels in one
// launch.  Workgroup g first takes item g; when the grid is smaller than the
// work list, workgroups then pull further items from an atomic counter
// (persistent mode).  An item is a few whole kernels of equal B, or one large
// kernel.  For every item:
//
//  rows     Sixteen lanes share one counter row (one DPP row): each lane owns
//           VPL columns and loads them with 16-byte vector loads (the 16 lanes
//           cover 256 contiguous bytes).  Tier 1's feature, the log of counter
//           over cycles, is standardised as z = (ln c - ln cyc - mu) / sigma;
//           in FP32 the hardware base-2 logarithm is used and the ln 2 factor
//           is folded into 1/sigma, so an element costs one log and one FMA.
//           The weights of each optimisation sit in LDS; a 4-step DPP
//           rotate-add sums the 16 partial dot products.  Only the predictions
//           the composed table needs are formed: row S predicts adding b for
//           every b above its highest set bit, which gives every subset S'
//           exactly one incoming edge e[S'] = P(S' without its top bit, top
//           bit).  With a grid output every b not in S is predicted.
//  compose  L[S] = sum over bits b of S, ascending, of e[S & (2^(b+1) - 1)]
//           (the prediction for adding b to S & (2^b - 1)), from LDS.
//  rank     Tier 3: per kernel, candidates S >= 1 with L > tau, best first
//           (score descending, S ascending); per-lane best-first lists are
//           merged with a butterfly of bitonic merges across lanes, and for
//           kernels with more than 64 versions across waves through LDS.
//
// Each row's arithmetic, and each kernel's composition and ranking, depend
// only on that kernel's data, never on its position in the batch, so ragged
// batches give bit-identical results to single-kernel batches.
#pragma once

#include "kernels.hpp"

namespace sugg {

template <typename T, int VW>
struct alignas(sizeof(T) * VW) VecN {
  T v[VW];
};

// Natural log in FP64 without the library's double-double steps (a third of
// its instructions; the prediction kernels take one per counter).  With
// x = 2^e m, m in [sqrt(1/2), sqrt(2)): ln x = e ln 2 + 2 atanh(s),
// s = (m - 1) / (m + 1), |s| <= 0.1716, and 2 atanh(s) = 2 s (1 + s^2/3 + ...
// + s^18/19) (the first omitted term is below 2.5e-17 of the sum).  s is the
// quotient by a Newton-refined hardware reciprocal with a residual step that
// also takes in the rounding of m + 1; ln 2 is split so that e times its high
// part is exact.  Error within 1.2 units in the last place (against long
// double over 2e7 arguments, 1e-300..1e300 and around 1); 0 gives -inf, a
// negative or NaN argument NaN, +inf +inf; subnormals are exact inputs.
__device__ __forceinline__ double flog64(double x) {
  double m = __builtin_amdgcn_frexp_mant(x);   // [0.5, 1)
  int e = __builtin_amdgcn_frexp_exp(x);
  const bool lo = m < 0.70710678118654752440;
  m = lo ? m * 2.0 : m;
  e = lo ? e - 1 : e;
  const double n = m - 1.0;          // exact
  const double d = m + 1.0;
  const double dl = m - (d - 1.0);   // the rounding error of d, exact
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  r = fma(fma(-d, r, 1.0), r, r);
  double s = n * r;
  s = fma(fma(-s, dl, fma(-s, d, n)), r, s);
  const double s2 = s * s;
  double p = 1.0 / 19;
  p = fma(p, s2, 1.0 / 17);
  p = fma(p, s2, 1.0 / 15);
  p = fma(p, s2, 1.0 / 13);
  p = fma(p, s2, 1.0 / 11);
  p = fma(p, s2, 1.0 / 9);
  p = fma(p, s2, 1.0 / 7);
  p = fma(p, s2, 1.0 / 5);
  p = fma(p, s2, 1.0 / 3);
  const double t = 2.0 * s;
  const double ed = (double)e;
  const double tail = fma(t * s2, p, ed * 0x1.9ef35793c7673p-41);
  const double y = fma(ed, 0x1.62e42fefa2000p-1, t + tail);
  const double inf = __builtin_huge_val();
  return (x > 0.0 && x < inf) ? y : (x == 0.0 ? -inf : (x == inf ? inf : __builtin_nan("")));
}

// Natural log for FP64; base-2 hardware log for FP32 (callers scale by ln 2).
template <typename T> __device__ __forceinline__ T dlog(T x);
template <> __device__ __forceinline__ float dlog<float>(float x) { return logf(x); }
template <> __device__ __forceinline__ double dlog<double>(double x) { return log(x); }
template <typename T> __device__ __forceinline__ T feat_log(T x);
template <> __device__ __forceinline__ float feat_log<float>(float x) { return __builtin_amdgcn_logf(x); }
template <> __device__ __forceinline__ double feat_log<double>(double x) { return flog64(x); }
template <typename T> __device__ __forceinline__ T feat_log_unit();
template <> __device__ __forceinline__ float feat_log_unit<float>() { return 0.69314718055994530942f; }
template <> __device__ __forceinline__ double feat_log_unit<double>() { return 1.0; }

// Row arithmetic shared by every kernel that predicts from a counter row, so
// that they all produce bit-identical predictions.  A lane holds NCH chunks of
// VW columns of one row; 16 lanes (a DPP row) hold the whole row.
template <typename T, int NCH, int VW>
__device__ __forceinline__ T row_features(const T (&c)[NCH][VW], T cyc, const T (&s)[NCH][VW],
                                          const T (&m)[NCH][VW], T (&z)[NCH][VW]) {
  const T lc = feat_log<T>(cyc);
  T chk = lc;
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
    for (int v = 0; v < VW; ++v) {
      const T x = feat_log<T>(c[ch][v]) - lc;
      chk += x;
      z[ch][v] = fma(x, s[ch][v], m[ch][v]);
    }
  return chk;   // NaN or infinite when a counter or the cycle count is bad
}

template <typename T, int NCH, int VW>
__device__ __forceinline__ T row_dot(const T (&z)[NCH][VW], const T* wrow, int l16) {
  T part = T(0);
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const VecN<T, VW> w = *reinterpret_cast<const VecN<T, VW>*>(wrow + (l16 + kRowLanes * ch) * VW);
#pragma unroll
    for (int v = 0; v < VW; ++v) part = fma(z[ch][v], w.v[v], part);
  }
  return row_sum16(part);
}

// Weights into LDS: D rows of EP columns (zero past E) plus the intercepts.
// FULL (E == EP): FP32 rows are 16-byte aligned (stride w32_ld(E)), copied as
// float4.
template <typename T, bool FULL>
__device__ __forceinline__ void stage_weights(const T* W, int ldw, int D, int E, int EP, T* Wl, T* Wb, int tid,
                                              int nthr) {
  if (FULL && sizeof(T) == 4) {
    const int q = EP / 4;
    for (int i = tid; i < D * q; i += nthr) {
      const int o = i / q, j = (i - o * q) * 4;
      *reinterpret_cast<float4*>(Wl + o * EP + j) = *reinterpret_cast<const float4*>(W + (int64_t)o * ldw + j);
    }
  } else {
    for (int i = tid; i < D * EP; i += nthr) {
      const int o = i / EP, j = i - o * EP;
      Wl[i] = (FULL || j < E) ? W[(int64_t)o * ldw + j] : T(0);
    }
  }
  for (int o = tid; o < D; o += nthr) Wb[o] = W[(int64_t)o * ldw + E];
}

// This lane's column constants: z = fma(log(c) - log(cyc), s, m) with
// s = unit / sigma and m = -mu / sigma (zero past E).
template <typename T, int NCH, int VW, bool FULL>
__device__ __forceinline__ void column_constants(const T* mu, const T* isg, int E, int l16, T (&s)[NCH][VW],
                                                 T (&m)[NCH][VW]) {
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int c0 = (l16 + kRowLanes * ch) * VW;
    T iv[VW], mv[VW];
    if (FULL || c0 + VW <= E) {
      const VecN<T, VW> qi = *reinterpret_cast<const VecN<T, VW>*>(isg + c0);
      const VecN<T, VW> qm = *reinterpret_cast<const VecN<T, VW>*>(mu + c0);
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        iv[v] = qi.v[v];
        mv[v] = qm.v[v];
      }
    } else {
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        const bool ok = c0 + v < E;
        iv[v] = ok ? isg[c0 + v] : T(0);
        mv[v] = ok ? mu[c0 + v] : T(0);
      }
    }
#pragma unroll
    for (int v = 0; v < VW; ++v) {
      s[ch][v] = iv[v] * feat_log_unit<T>();
      m[ch][v] = -mv[v] * iv[v];
    }
  }
}

// Dynamic LDS layout of the fused kernel (host and device agree on it).
struct PathSmem {
  int ep;        // padded weight row length
  size_t W, Wb, sm, e, L, kro, kid, kop, xw, total;
};

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

template <typename T, int VPL, int KT>
__host__ __device__ inline PathSmem path_smem(int D, int max_rows, int max_nk, int max_B, int nwaves) {
  PathSmem s;
  s.ep = kRowLanes * VPL;
  size_t o = 0;
  s.W = o;   o += sizeof(T) * (size_t)D * s.ep;
  s.Wb = o;  o += sizeof(T) * (size_t)D;
  o = align_up(o, 16);
  s.sm = o;  o += sizeof(T) * 2 * (size_t)s.ep;
  s.e = o;   o += sizeof(T) * (size_t)max_rows;
  s.L = o;   o += sizeof(T) * (size_t)max_rows;
  o = align_up(o, 16);
  s.kro = o; o += sizeof(int64_t) * (size_t)max_nk;
  s.kid = o; o += sizeof(int32_t) * (size_t)max_nk;
  s.kop = o; o += sizeof(int32_t) * (size_t)(max_nk * (max_B > 0 ? max_B : 1));
  o = align_up(o, 16);
  s.xw = o;  o += sizeof(Entry<T>) * (size_t)KT * nwaves;
  s.total = align_up(o, 16);
  return s;
}

template <typename T> __device__ __forceinline__ T lane_read(T v, int l);
template <> __device__ __forceinline__ float lane_read<float>(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
template <> __device__ __forceinline__ double lane_read<double>(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// Maximum over aligned groups of G lanes (G a power of two <= 64), received
// by every lane of the group.  Groups of 16 or more reduce each 16-lane row
// with DPP rotations and combine rows through lane reads; smaller groups
// exchange through lane shuffles.
template <typename T>
__device__ __forceinline__ T group_max(T v, int G, int lane) {
  if (G < kRowLanes) {
    for (int off = 1; off < G; off <<= 1) v = fmax(v, __shfl_xor(v, off, kWave));
    return v;
  }
  v = fmax(v, row_ror<8>(v));
  v = fmax(v, row_ror<4>(v));
  v = fmax(v, row_ror<2>(v));
  v = fmax(v, row_ror<1>(v));
  if (G == kRowLanes) return v;
  const T r0 = lane_read(v, 0), r1 = lane_read(v, 16), r2 = lane_read(v, 32), r3 = lane_read(v, 48);
  if (G == 32) return lane < 32 ? fmax(r0, r1) : fmax(r2, r3);
  return fmax(fmax(r0, r1), fmax(r2, r3));
}

template <typename T, int KT>
__device__ __forceinline__ void write_list(const Entry<T> (&L)[KT], int k, int n, int32_t* idx_out,
                                           T* score_out, int32_t* count_out) {
  int cnt = 0;
#pragma unroll
  for (int i = 0; i < KT; ++i) {
    if (i < n) {
      const bool ok = L[i].s >= 0;
      idx_out[(int64_t)k * n + i] = ok ? L[i].s : -1;
      score_out[(int64_t)k * n + i] = ok ? L[i].v : qnan<T>();
      cnt += ok ? 1 : 0;
    }
  }
  count_out[k] = cnt;
}

// FULL: E == 16 * VPL (every lane column is a real column, no bounds checks).
// GRID: the per-optimisation grid is written (every b not in S predicted).
template <typename T, int VPL, int VW, int U, int KT, bool FULL, bool GRID>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu((U == 1 && !GRID && KT <= 4) ? 5 : 1, 8))) path_kernel(const PathArgs<T> a, const int max_rows,
                                                   const int max_nk, const int max_B) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NCH = VPL / VW;
  const int E = a.E, D = a.D;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int wave = tid >> 6, nwaves = nthr >> 6;
  const int lane = tid & 63, l16 = lane & 15, grp = lane >> 4;
  const PathSmem ly = path_smem<T, VPL, KT>(D, max_rows, max_nk, max_B, nwaves);
  T* Wl = reinterpret_cast<T*>(smem + ly.W);
  T* Wb = reinterpret_cast<T*>(smem + ly.Wb);
  T* eb = reinterpret_cast<T*>(smem + ly.e);
  T* Lb = reinterpret_cast<T*>(smem + ly.L);
  int64_t* kro = reinterpret_cast<int64_t*>(smem + ly.kro);
  int32_t* kid = reinterpret_cast<int32_t*>(smem + ly.kid);
  int32_t* kop = reinterpret_cast<int32_t*>(smem + ly.kop);
  Entry<T>* xw = reinterpret_cast<Entry<T>*>(smem + ly.xw);
  __shared__ int s_next, s_any;
  const bool dynamic = (int)gridDim.x < a.n_items;

  const int EP = ly.ep;
  // this lane's columns: chunk ch covers columns (l16 + 16 ch) * VW + [0, VW);
  // z = fma(log(c) - log(cyc), s, m) with s = unit / sigma, m = -mu / sigma
  T* sml = reinterpret_cast<T*>(smem + ly.sm);
  // weights, intercepts and column constants are staged after the first
  // item's row loads are in flight (so the two memory latencies overlap)
  auto stage_model = [&]() {
    stage_weights<T, FULL>(a.W, a.ldw, D, E, EP, Wl, Wb, tid, nthr);
    if (tid < kRowLanes) {
      T s0[NCH][VW], m0[NCH][VW];
      column_constants<T, NCH, VW, FULL>(a.mu, a.isg, E, l16, s0, m0);
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int v = 0; v < VW; ++v) {
          sml[(l16 + kRowLanes * ch) * VW + v] = s0[ch][v];
          sml[EP + (l16 + kRowLanes * ch) * VW + v] = m0[ch][v];
        }
    }
  };
  bool staged = false;
  T ca[U][NCH][VW], cb[U][NCH][VW];
  T cya[U], cyb[U];
  bool bad = false;

  auto get_item = [&](int i) -> Item {
    Item t;
    if (a.uni_B >= 0) {
      // every kernel has uni_B optimisations and items take uni_nk adjacent
      // kernels in batch order: the item needs no lookup
      t.first = i * a.uni_nk;
      t.nk = min(a.uni_nk, a.K - t.first);
      t.B = a.uni_B;
      t.R = t.nk << a.uni_B;
      t.row0 = (int64_t)t.first << a.uni_B;
    } else {
      t = a.items[i];
    }
    return t;
  };
  const int step = nwaves * 4 * U;
  const int b0 = wave * 4 * U;
  int it = blockIdx.x;
  while (it < a.n_items) {
    if (dynamic && tid == 0) s_next = (int)gridDim.x + atomicAdd(a.queue, 1);
    const Item item = get_item(it);
    const int B = item.B, nk = item.nk, R = item.R;
    const uint32_t mask = (1u << B) - 1u;
    const bool contig = item.row0 >= 0;
    // Rows past the item are clamped to its last row (read, never written).
    auto row_addr = [&](int r) -> int64_t {
      r = r < R ? r : R - 1;
      return contig ? item.row0 + r : kro[r >> B] + (r & mask);
    };
    // adjacent kernels: rows addressed by 32-bit offsets from the item's first row
    const T* ibase = a.counters + (contig ? item.row0 : 0) * E;
    const T* icyc = a.cycles + (contig ? item.row0 : 0);
    auto load = [&](int base, T (&c)[U][NCH][VW], T (&cy)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        int rr = base + u * 4 + grp;
        rr = rr < R ? rr : R - 1;
        const int64_t grow = contig ? 0 : kro[rr >> B] + (rr & mask);
        const T* rp = contig ? ibase + (uint32_t)(rr * E) : a.counters + grow * E;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
          const int c0 = (l16 + kRowLanes * ch) * VW;
          if (FULL || c0 < E) {
            const VecN<T, VW> q = *reinterpret_cast<const VecN<T, VW>*>(rp + c0);
#pragma unroll
            for (int v = 0; v < VW; ++v) c[u][ch][v] = q.v[v];
          } else {
#pragma unroll
            for (int v = 0; v < VW; ++v) c[u][ch][v] = T(1);
          }
        }
        cy[u] = contig ? icyc[rr] : a.cycles[grow];
      }
    };
    if (a.kmask) {   // masked runs: the selection flag starts clear
      if (tid == 0) s_any = 0;
      __syncthreads();
    }
    if (a.uni_B >= 0 && a.uni_ops) {
      // same ids everywhere: the records hold nothing the item does not know
      for (int i = tid; i < nk; i += nthr) {
        kid[i] = item.first + i;
        kro[i] = (int64_t)(item.first + i) << B;
        if (a.kmask && a.kmask[item.first + i]) s_any = 1;
      }
      for (int i = tid; i < nk * B; i += nthr) {
        const int b = i % B;
        kop[i] = (int)(((b < 8 ? a.uni_opt_lo >> (8 * b) : a.uni_opt_hi >> (8 * (b - 8)))) & 0xffu);
      }
    } else {
      for (int i = tid; i < nk; i += nthr) {
        const KRec& rec = a.recs[item.first + i];
        kid[i] = rec.kid;
        kro[i] = rec.row_off;
        if (a.kmask && a.kmask[rec.kid]) s_any = 1;
      }
      for (int i = tid; i < nk * B; i += nthr) {
        const int kk = i / B, b = i - kk * B;
        kop[i] = a.recs[item.first + kk].opt[b];
      }
    }

    // ---- rows: Tier 1 features and Tier 2 predictions ----------------------
    auto compute = [&](int base, const T (&c)[U][NCH][VW], const T (&cy)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r0 = base + u * 4;          // row of lane group 0 (uniform)
        if (r0 >= R) break;
        const int r = r0 + grp;
        const bool live = r < R;
        T z[NCH][VW];
        T s_r[NCH][VW], m_r[NCH][VW];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
          const VecN<T, VW> qs = *reinterpret_cast<const VecN<T, VW>*>(sml + (l16 + kRowLanes * ch) * VW);
          const VecN<T, VW> qm = *reinterpret_cast<const VecN<T, VW>*>(sml + EP + (l16 + kRowLanes * ch) * VW);
#pragma unroll
          for (int v = 0; v < VW; ++v) {
            s_r[ch][v] = qs.v[v];
            m_r[ch][v] = qm.v[v];
          }
        }
        const T chk = row_features<T, NCH, VW>(c[u], cy[u], s_r, m_r, z);
        // a non-positive, non-normal or non-finite counter or cycle count
        // makes the checksum NaN or infinite
        bad |= live && !__builtin_isfinite(chk);
        const uint32_t S0 = (uint32_t)r0 & mask;
        const int hlo = (GRID || S0 == 0) ? 0 : msb(S0) + 1;
        const int kk = live ? (r >> B) : 0;
        const uint32_t S = (uint32_t)r & mask;
        const int ms = msb(S);
        // Q independent dot products at a time (their weight reads and row
        // reductions overlap); each is the same arithmetic as row_dot alone
        auto dots = [&](auto qc, int h0) {
          constexpr int Q = decltype(qc)::value;
          T p[Q];
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            const int o = kop[kk * B + h0 + q];
            p[q] = row_dot<T, NCH, VW>(z, Wl + o * EP, l16) + Wb[o];
          }
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            const int h = h0 + q;
            if (l16 == 0 && live) {
              if (GRID) a.grid[row_addr(r) * a.grid_ld + h] = ((S >> h) & 1u) ? qnan<T>() : p[q];
              if (h > ms) eb[r | (1 << h)] = p[q];
            }
          }
        };
        int h0 = hlo;
        for (; h0 + 2 <= B; h0 += 2) dots(std::integral_constant<int, 2>{}, h0);
        if (h0 < B) dots(std::integral_constant<int, 1>{}, h0);
        if (GRID && l16 == 0 && live) {
          const int64_t grow = row_addr(r);
          for (int b = B; b < a.grid_ld; ++b) a.grid[grow * a.grid_ld + b] = qnan<T>();
        }
      }
    };

    __syncthreads();   // item metadata and the selection flag are visible
    if (a.kmask && !s_any) {   // masked run: no selected kernel in this item
      it = dynamic ? s_next : a.n_items;
      __syncthreads();
      continue;
    }
    // Two register buffers: the next rows load while the current ones
    // compute.  Every load is issued unconditionally (rows past the item
    // re-read its last row) and the loop has one exit, so the loads in flight
    // are the same on every path and a step waits only for its own rows.
    load(b0, ca, cya);
    load(b0 + step, cb, cyb);
    if (!staged) {   // the model's loads overlap the first rows'
      stage_model();
      staged = true;
    }
    __syncthreads();   // weights visible
    const int pairs = b0 < R ? (R - b0 + 2 * step - 1) / (2 * step) : 0;
    for (int i = 0, base = b0; i < pairs; ++i, base += 2 * step) {
      compute(base, ca, cya);
      load(base + 2 * step, ca, cya);
      compute(base + step, cb, cyb);
      load(base + 3 * step, cb, cyb);
    }
    __syncthreads();
    const int nit = dynamic ? s_next : a.n_items;

    // ---- compose the subset table -----------------------------------------
    // L(S) = sum over the bits b of S, ascending, of the edge into
    // S & (2^(b+1) - 1); thread r composes row r of the item
    auto compose_row = [&](int r) -> T {
      const uint32_t S = (uint32_t)r & mask;
      const int kb = r & ~(int)mask;
      T L = T(0);
      for (int b = 0; b < B; ++b)
        if ((S >> b) & 1u) L += eb[kb | (int)(S & ((2u << b) - 1u))];
      if (a.table && (!a.kmask || a.kmask[kid[r >> B]])) a.table[(contig ? item.row0 + r : kro[r >> B] + S)] = L;
      return L;
    };
    if (B > 6 || !a.idx_out) {
      for (int r = tid; r < R; r += nthr) Lb[r] = compose_row(r);
      __syncthreads();
    }

    // ---- Tier 3 ranking -----------------------------------------------------
    if (a.idx_out) {
      if (B <= 6) {
        // a kernel's 2^B subsets sit in one aligned group of G lanes of the
        // wave that composes them: the top n by n rounds of a group maximum
        // (ties: the lowest lane, i.e. the smallest S), each winner dropping
        // out of the next round
        const int G = 1 << B;
        const int gbase = lane & ~(G - 1);
        const uint64_t gmask = G == kWave ? ~0ull : ((1ull << G) - 1ull);
        for (int c0 = wave * kWave; c0 < R; c0 += nwaves * kWave) {
          const int r = c0 + lane;
          const int S = r & (int)mask;
          T x = -__builtin_inf();
          if (r < R) {
            const T v = compose_row(r);
            if (S != 0 && v > a.tau) x = v;
          }
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
          const bool sel = r < R && (!a.kmask || a.kmask[kid[r >> B]]);
          if (sel && place >= 0) {
            const int k = kid[r >> B];
            a.idx_out[(int64_t)k * a.n + place] = S;
            a.score_out[(int64_t)k * a.n + place] = x;
          }
          if (sel && S == 0) {
            const int k = kid[r >> B];
            for (int j = cnt; j < a.n; ++j) {
              a.idx_out[(int64_t)k * a.n + j] = -1;
              a.score_out[(int64_t)k * a.n + j] = qnan<T>();
            }
            a.count_out[k] = cnt;
          }
        }
      } else {
        for (int kk = 0; kk < nk; ++kk) {
          Entry<T> lst[KT];
#pragma unroll
          for (int i = 0; i < KT; ++i) lst[i] = empty_entry<T>();
          for (int S = tid; S < (1 << B); S += nthr) {
            const T v = Lb[(kk << B) + S];
            if (S != 0 && v > a.tau) {
              Entry<T> e;
              e.v = v;
              e.s = S;
              list_insert<T, KT>(lst, e);
            }
          }
          group_merge<T, KT>(lst, kWave);
          if (lane == 0)
#pragma unroll
            for (int i = 0; i < KT; ++i) xw[wave * KT + i] = lst[i];
          __syncthreads();
          if (tid == 0) {
            for (int w = 1; w < nwaves; ++w) {
              Entry<T> o[KT];
#pragma unroll
              for (int i = 0; i < KT; ++i) o[i] = xw[w * KT + i];
              list_merge<T, KT>(lst, o);
            }
            if (!a.kmask || a.kmask[kid[kk]]) write_list<T, KT>(lst, kid[kk], a.n, a.idx_out, a.score_out, a.count_out);
          }
          __syncthreads();
        }
      }
    }
    if (!dynamic) break;   // one item per workgroup
    __syncthreads();       // this item's LDS is no longer read (nor s_next)
    it = nit;
  }
  if (__ballot(bad) != 0 && lane == 0) atomicOr(a.status, (int)kStatusBadCounter);
  // In persistent mode the last workgroup to finish re-arms the work counter
  // (queue[0] = next item, queue[1] = finished workgroups), so a launch needs
  // no reset node before it and can be replayed from a graph.
  if (dynamic && tid == 0) {
    __threadfence();
    if (atomicAdd(a.queue + 1, 1) == (int)gridDim.x - 1) {
      atomicExch(a.queue, 0);
      atomicExch(a.queue + 1, 0);
    }
  }
}

template <typename T, int VPL, int VW, int U, int KT, bool FULL, bool GRID>
hipError_t launch_path_t(const PathArgs<T>& a, int max_rows, int max_nk, int max_B,
                         const PathLaunch& cfg, hipStream_t s) {
  const int nw = cfg.waves;
  const PathSmem ly = path_smem<T, VPL, KT>(a.D, max_rows, max_nk, max_B, nw);
  auto kern = path_kernel<T, VPL, VW, U, KT, FULL, GRID>;
  if (ly.total > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)ly.total);
    if (e != hipSuccess) return e;
  }
  int grid = cfg.grid;
  if (grid <= 0) {
    int dev = 0, cus = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(kern), nw * 64, ly.total);
    if (e != hipSuccess) return e;
    grid = cus * (per > 0 ? per : 1);
  }
  if (grid > a.n_items) grid = a.n_items;
  if (grid <= 0) return hipSuccess;
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL(kern, dim3(grid), dim3(nw * 64), ly.total, s, a, max_rows, max_nk, max_B);
  return hipGetLastError();
}

template <typename T, int VPL, int VW, int KT, bool FULL, bool GRID>
hipError_t dispatch_u(const PathArgs<T>& a, int mr, int mk, int mb, const PathLaunch& c, hipStream_t s) {
  if (c.unroll >= 4) return launch_path_t<T, VPL, VW, 4, KT, FULL, GRID>(a, mr, mk, mb, c, s);
  if (c.unroll == 2) return launch_path_t<T, VPL, VW, 2, KT, FULL, GRID>(a, mr, mk, mb, c, s);
  return launch_path_t<T, VPL, VW, 1, KT, FULL, GRID>(a, mr, mk, mb, c, s);
}

template <typename T, int VPL, int VW, int KT, bool FULL>
hipError_t dispatch_g(const PathArgs<T>& a, int mr, int mk, int mb, const PathLaunch& c, hipStream_t s) {
  if (a.grid) return dispatch_u<T, VPL, VW, KT, FULL, true>(a, mr, mk, mb, c, s);
  return dispatch_u<T, VPL, VW, KT, FULL, false>(a, mr, mk, mb, c, s);
}

// Judge: the plain composed log-speedup of given subsets only.  One wave per
// (kernel, candidate); the chain terms (one per bit b of S, from version
// S & (2^b - 1)) are spread over the four 16-lane groups and summed in
// ascending b, with the fused kernel's row arithmetic, so the value equals the
// fused kernel's table entry bit for bit.
template <typename T, int VPL, int VW>
__global__ void __launch_bounds__(256) judge_kernel(const JudgeArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NCH = VPL / VW;
  const int E = a.E, D = a.D, EP = kRowLanes * VPL;
  const int tid = threadIdx.x, lane = tid & 63, l16 = lane & 15, grp = lane >> 4;
  T* Wl = reinterpret_cast<T*>(smem);
  T* Wb = Wl + D * EP;
  stage_weights<T, false>(a.W, a.ldw, D, E, EP, Wl, Wb, tid, (int)blockDim.x);
  T s_r[NCH][VW], m_r[NCH][VW];
  column_constants<T, NCH, VW, false>(a.mu, a.isg, E, l16, s_r, m_r);
  __syncthreads();   // the only barrier: waves below work independently
  // jobs [0, K C) are the first set's, the next K C2 the second's
  int64_t job = (int64_t)blockIdx.x * 4 + (tid >> 6);
  const int64_t n1 = (int64_t)a.K * a.C;
  if (job >= n1 + (int64_t)a.K * a.C2) return;
  const bool second = job >= n1;
  if (second) job -= n1;
  const int k = (int)(job / (second ? a.C2 : a.C));
  const int32_t S = second ? a.cand2[job] : a.cand[job];
  T* const out = second ? a.out2 : a.out;
  const T* const ref = second ? a.ref2 : a.ref;
  const int B = a.nopts[k];
  if (S <= 0 || S >= (1 << B)) {
    if (lane == 0) out[job] = S == 0 ? T(0) : qnan<T>();
    return;   // no candidate: nothing to disagree with
  }
  const int nt = __popc((uint32_t)S);
  const int64_t r0 = a.row_off[k];
  bool bad = false;
  T L = T(0);   // meaningful in lane 0
  for (int t0 = 0; t0 < nt; t0 += 4) {   // uniform per wave
    const int t = t0 + grp;
    uint32_t rest = (uint32_t)S;          // drop the t lowest set bits
    for (int i = 0; i < t && rest; ++i) rest &= rest - 1;
    const int b = t < nt ? __ffs(rest) - 1 : 0;
    const uint32_t Sp = t < nt ? ((uint32_t)S & ((1u << b) - 1u)) : 0u;
    const T* rp = a.counters + (r0 + Sp) * E;
    T c[NCH][VW];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const int cc = (l16 + kRowLanes * ch) * VW;
      if (cc < E) {
        const VecN<T, VW> q = *reinterpret_cast<const VecN<T, VW>*>(rp + cc);
#pragma unroll
        for (int v = 0; v < VW; ++v) c[ch][v] = q.v[v];
      } else {
#pragma unroll
        for (int v = 0; v < VW; ++v) c[ch][v] = T(1);
      }
    }
    T z[NCH][VW];
    const T chk = row_features<T, NCH, VW>(c, a.cycles[r0 + Sp], s_r, m_r, z);
    bad |= t < nt && !__builtin_isfinite(chk);
    const int o = a.opt_ids[a.opt_off[k] + b];
    const T p = row_dot<T, NCH, VW>(z, Wl + o * EP, l16) + Wb[o];
    // terms t0 .. t0+3 sit in lanes 0, 16, 32, 48: add them in ascending order
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const T pg = __shfl(p, g * 16, kWave);
      if (t0 + g < nt) L += pg;
    }
  }
  if (lane == 0) {
    out[job] = L;
    // fallback test: the reference (surrogate) value of this subset differs
    // from the plain value by more than tol
    if (a.flag && !(fabs((double)ref[job] - (double)L) <= a.tol)) atomicOr(a.flag + k, 1);
  }
  if (__ballot(bad) != 0 && lane == 0) atomicOr(a.status, (int)kStatusBadCounter);
}

template <typename T, int VPL>
hipError_t launch_judge_vpl(const JudgeArgs<T>& a, hipStream_t s) {
  constexpr int VEC = 16 / sizeof(T);
  const int64_t jobs = (int64_t)a.K * a.C + (int64_t)a.K * a.C2;
  if (jobs <= 0) return hipSuccess;
  const size_t smem = sizeof(T) * ((size_t)a.D * kRowLanes * VPL + a.D);
  const dim3 grid((unsigned)((jobs + 3) / 4));
  if (a.flag && !a.accumulate) {
    const hipError_t e = launch_fill_i32(a.flag, 0, a.K, s);
    if (e != hipSuccess) return e;
  }
  (void)hipGetLastError();  // report only this launch's status
  if ((a.E % VEC) == 0 && (reinterpret_cast<uintptr_t>(a.counters) % 16) == 0)
    hipLaunchKernelGGL((judge_kernel<T, VPL, VEC>), grid, dim3(256), smem, s, a);
  else
    hipLaunchKernelGGL((judge_kernel<T, VPL, 1>), grid, dim3(256), smem, s, a);
  return hipGetLastError();
}

// All launch variants for one column count per lane (one translation unit
// each, so the variants compile in parallel).
template <typename T, int VPL>
hipError_t launch_path_vpl(const PathArgs<T>& a, int mr, int mk, int mb, const PathLaunch& c, hipStream_t s) {
  if (a.judge) return launch_judge_vpl<T, VPL>(*a.judge, s);
  constexpr int VEC = 16 / sizeof(T);
  const bool vec_ok = (a.E % VEC) == 0 && (reinterpret_cast<uintptr_t>(a.counters) % 16) == 0;
  if (a.n <= 4) {
    if (vec_ok) {
      if (a.E == kRowLanes * VPL) return dispatch_g<T, VPL, VEC, 4, true>(a, mr, mk, mb, c, s);
      return dispatch_g<T, VPL, VEC, 4, false>(a, mr, mk, mb, c, s);
    }
    return dispatch_g<T, VPL, 1, 4, false>(a, mr, mk, mb, c, s);
  }
  if (vec_ok) {
    if (a.E == kRowLanes * VPL) return dispatch_g<T, VPL, VEC, 8, true>(a, mr, mk, mb, c, s);
    return dispatch_g<T, VPL, VEC, 8, false>(a, mr, mk, mb, c, s);
  }
  return dispatch_g<T, VPL, 1, 8, false>(a, mr, mk, mb, c, s);
}

}  // namespace sugg
