// The scoring pass (Section 2, Tiers 1-3) in its streaming form, for ragged
// batches: each workgroup takes one chunk of consecutive whole kernels in
// memory order (of any mix of B, about a target number of rows; a larger
// kernel is a chunk alone), streams its rows (one contiguous read), forms
// Tier 1's features and Tier 2's chain edges into LDS, then composes the
// subset tables and takes Tier 3's top n of every kernel of the chunk.
//
// Unlike the persistent fused kernel, whose workgroups walk a work list of
// equal-B kernels and stop streaming at each item's composition, the chunks
// here are independent workgroups in memory order: the hardware dispatcher
// keeps every compute unit streaming while some of its workgroups compose,
// no work counter or item list is read, and a chunk's first rows need no
// metadata.  Row, edge and composition arithmetic are the fused kernel's
// (each edge, each table entry bit for bit); the ranking takes the same top
// n by (score descending, subset ascending).
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "path_impl.hpp"

namespace sugg {

constexpr int kChunkThreads = 256;

struct ChunkSmem {
  int ep;
  size_t W, Wb, sm, e, L, kr, rk, total;
};

template <typename T>
__host__ __device__ inline ChunkSmem chunk_smem(int D, int E, int max_rows, int max_nk) {
  ChunkSmem s;
  s.ep = E <= 64 ? 64 : (E <= 128 ? 128 : 256);
  size_t o = 0;
  s.W = o;   o += sizeof(T) * (size_t)D * s.ep;
  s.Wb = o;  o += sizeof(T) * (size_t)D;
  o = align_up(o, 16);
  s.sm = o;  o += sizeof(T) * 2 * (size_t)s.ep;
  s.e = o;   o += sizeof(T) * (size_t)max_rows;
  s.L = o;   o += sizeof(T) * (size_t)max_rows;
  o = align_up(o, 16);
  s.kr = o;  o += sizeof(CRec) * (size_t)max_nk;
  s.rk = o;  o += sizeof(int16_t) * (size_t)max_rows;
  s.total = align_up(o, 16);
  return s;
}

size_t path_chunk_lds(size_t tsize, int D, int E, int max_rows, int max_nk) {
  return tsize == 4 ? chunk_smem<float>(D, E, max_rows, max_nk).total
                    : chunk_smem<double>(D, E, max_rows, max_nk).total;
}

// One 16-byte vector of the weight image in LDS (D rows of EP columns, zero
// past E): vector i of the row-major image.
template <typename T, bool FULL>
__device__ __forceinline__ VecN<T, 16 / sizeof(T)> weight_vec(const T* W, int ldw, int E, int EP, int i) {
  constexpr int VEC = 16 / sizeof(T);
  const int q = EP / VEC, o = i / q, j = (i - o * q) * VEC;
  VecN<T, VEC> r;
  if (FULL && sizeof(T) == 4) {   // rows of stride w32_ld(E): 16-byte aligned
    r = *reinterpret_cast<const VecN<T, VEC>*>(W + (int64_t)o * ldw + j);
  } else {
#pragma unroll
    for (int v = 0; v < VEC; ++v) r.v[v] = (FULL || j + v < E) ? W[(int64_t)o * ldw + j + v] : T(0);
  }
  return r;
}

template <typename T, int VPL, int VW, int U, int KT, bool FULL>
__global__ void __launch_bounds__(kChunkThreads) path_chunk_kernel(const ChunkArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NCH = VPL / VW;
  constexpr int VEC = 16 / sizeof(T);
  constexpr int kGroups = kChunkThreads / kRowLanes;
  constexpr int kWaves = kChunkThreads / kWave;
  const int E = a.E, D = a.D;
  const int tid = threadIdx.x, g = tid / kRowLanes, l16 = tid % kRowLanes, lane = tid % kWave, wave = tid / kWave;
  const ChunkSmem ly = chunk_smem<T>(D, E, a.max_rows, a.max_nk);
  const int EP = ly.ep;
  T* Wl = reinterpret_cast<T*>(smem + ly.W);
  T* Wb = reinterpret_cast<T*>(smem + ly.Wb);
  T* sml = reinterpret_cast<T*>(smem + ly.sm);
  T* eb = reinterpret_cast<T*>(smem + ly.e);
  T* Lb = reinterpret_cast<T*>(smem + ly.L);
  CRec* kr = reinterpret_cast<CRec*>(smem + ly.kr);
  int16_t* rk = reinterpret_cast<int16_t*>(smem + ly.rk);

  // rows: step i covers chunk rows [kGroups U i, kGroups U (i + 1)); lane
  // group g takes rows kGroups U i + kGroups u + g.  Every load is issued
  // unconditionally (rows past the chunk re-read its last row and are never
  // used), so the loads in flight are the same on every path and a step
  // waits only for its own rows, not for the next step's.
  constexpr int step = kGroups * U;
  auto load = [&](const Chunk& c, int base, T (&cv)[U][NCH][VW], T (&cy)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int r = base + kGroups * u + g;
      r = r < c.R ? r : c.R - 1;
      const T* rp = a.counters + (c.row0 + r) * E;
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        const int cc = (l16 + kRowLanes * ch) * VW;
        if (FULL || cc < E) {
          const VecN<T, VW> q = *reinterpret_cast<const VecN<T, VW>*>(rp + cc);
#pragma unroll
          for (int v = 0; v < VW; ++v) cv[u][ch][v] = q.v[v];
        } else {
#pragma unroll
          for (int v = 0; v < VW; ++v) cv[u][ch][v] = T(1);
        }
      }
      cy[u] = a.cycles[c.row0 + r];
    }
  };
  const int4* recs = reinterpret_cast<const int4*>(a.recs);
  int4* krv = reinterpret_cast<int4*>(kr);
  const Chunk ck = a.chunks[blockIdx.x];
  const int R = ck.R, nk = ck.nk;
  // loads in issue order: this chunk's kernel records and the model (small,
  // needed first), then the first two steps of rows; whatever would wait on
  // a load (a loop over a larger model or many kernels) comes before the rows
  int4 rec = make_int4(0, 0, 0, 0);
  if (tid < nk) rec = recs[ck.k0 + tid];
  const int nwv = D * (EP / VEC);
  VecN<T, VEC> wv0, wv1;
  if (tid < nwv) wv0 = weight_vec<T, FULL>(a.W, a.ldw, E, EP, tid);
  if (tid + kChunkThreads < nwv) wv1 = weight_vec<T, FULL>(a.W, a.ldw, E, EP, tid + kChunkThreads);
  const T wb = tid < D ? a.W[(int64_t)tid * a.ldw + E] : T(0);
  T s0[NCH][VW], m0[NCH][VW];
  if (tid < kRowLanes) column_constants<T, NCH, VW, FULL>(a.mu, a.isg, E, l16, s0, m0);
  for (int i = tid + 2 * kChunkThreads; i < nwv; i += kChunkThreads)   // larger models
    *reinterpret_cast<VecN<T, VEC>*>(Wl + i * VEC) = weight_vec<T, FULL>(a.W, a.ldw, E, EP, i);
  for (int j = tid + kChunkThreads; j < nk; j += kChunkThreads) krv[j] = recs[ck.k0 + j];   // many small kernels
  T ca[U][NCH][VW], cb[U][NCH][VW];
  T cya[U], cyb[U];
  load(ck, 0, ca, cya);
  load(ck, step, cb, cyb);

  // model into LDS (once per workgroup)
  if (tid < nwv) *reinterpret_cast<VecN<T, VEC>*>(Wl + tid * VEC) = wv0;
  if (tid + kChunkThreads < nwv) *reinterpret_cast<VecN<T, VEC>*>(Wl + (tid + kChunkThreads) * VEC) = wv1;
  if (tid < D) Wb[tid] = wb;
  if (tid < kRowLanes) {
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        sml[(l16 + kRowLanes * ch) * VW + v] = s0[ch][v];
        sml[EP + (l16 + kRowLanes * ch) * VW + v] = m0[ch][v];
      }
  }
  bool bad = false;
  if (tid < nk) krv[tid] = rec;
  __syncthreads();
  // each row's kernel: the last one starting at or before it
  for (int r = tid; r < R; r += kChunkThreads) {
    int lo = 0, hi = nk - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (kr[mid].rel <= r) lo = mid;
      else hi = mid - 1;
    }
    rk[r] = (int16_t)lo;
  }
  __syncthreads();

  // ---- rows: Tier 1 features and Tier 2 chain edges into LDS -------------
  auto compute = [&](int base, const T (&c)[U][NCH][VW], const T (&cy)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = base + kGroups * u + g;
      if (r >= R) break;   // uniform per 16-lane group
      const int j = rk[r];
      const int B = kr[j].B;
      const int kb = kr[j].rel;
      const int S = r - kb;
      T z[NCH][VW], s_r[NCH][VW], m_r[NCH][VW];
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
      bad |= !__builtin_isfinite(chk);
      const uint8_t* ops = kr[j].op;
      int b = msb((uint32_t)S) + 1;
      // two independent dot products at a time, each row_dot's arithmetic
      for (; b + 2 <= B; b += 2) {
        const int o0 = ops[b], o1 = ops[b + 1];
        const T p0 = row_dot<T, NCH, VW>(z, Wl + o0 * EP, l16) + Wb[o0];
        const T p1 = row_dot<T, NCH, VW>(z, Wl + o1 * EP, l16) + Wb[o1];
        if (l16 == 0) {
          eb[kb + (S | (1 << b))] = p0;
          eb[kb + (S | (2 << b))] = p1;
        }
      }
      if (b < B) {
        const int o0 = ops[b];
        const T p0 = row_dot<T, NCH, VW>(z, Wl + o0 * EP, l16) + Wb[o0];
        if (l16 == 0) eb[kb + (S | (1 << b))] = p0;
      }
    }
  };
  // pairs of steps, no exit inside (a step past the chunk computes nothing)
  const int pairs = (R + 2 * step - 1) / (2 * step);
  for (int i = 0, base = 0; i < pairs; ++i, base += 2 * step) {
    compute(base, ca, cya);
    load(ck, base + 2 * step, ca, cya);
    compute(base + step, cb, cyb);
    load(ck, base + 3 * step, cb, cyb);
  }
  if (__ballot(bad) != 0 && lane == 0) atomicOr(a.status, (int)kStatusBadCounter);
  __syncthreads();   // every edge of the chunk is in LDS

  // ---- compose: L(S) = sum over the bits b of S, ascending, of the edge
  // into S & (2^(b+1) - 1) (the fused kernel's order) ----------------------
  for (int r = tid; r < R; r += kChunkThreads) {
    const int j = rk[r];
    const int kb = kr[j].rel;
    const uint32_t S = (uint32_t)(r - kb);
    const int B = kr[j].B;
    T L = T(0);
    for (int b = 0; b < B; ++b)
      if ((S >> b) & 1u) L += eb[kb + (int)(S & ((2u << b) - 1u))];
    Lb[r] = L;
    if (a.table) a.table[ck.row0 + r] = L;
  }

  // ---- Tier 3: per kernel, one wave: per-lane best-first lists, merged --
  if (a.idx_out) {
    __syncthreads();
    for (int j = wave; j < nk; j += kWaves) {   // uniform per wave
      const int kb = kr[j].rel;
      const int V = 1 << kr[j].B;
      Entry<T> lst[KT];
#pragma unroll
      for (int i = 0; i < KT; ++i) lst[i] = empty_entry<T>();
      for (int S = lane; S < V; S += kWave) {
        const T v = Lb[kb + S];
        if (S != 0 && v > a.tau) {
          Entry<T> e;
          e.v = v;
          e.s = S;
          list_insert<T, KT>(lst, e);
        }
      }
      group_merge<T, KT>(lst, kWave);
      if (lane == 0) write_list<T, KT>(lst, ck.k0 + j, a.n, a.idx_out, a.score_out, a.count_out);
    }
  }
}

template <typename T, int VPL, int VW, int U, int KT, bool FULL>
hipError_t launch_chunk_k(const ChunkArgs<T>& a, size_t smem, hipStream_t s) {
  auto kern = path_chunk_kernel<T, VPL, VW, U, KT, FULL>;
  if (smem > 64 * 1024) {
    const hipError_t e =
        hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
  }
  (void)hipGetLastError();  // report only this launch's status
  hipLaunchKernelGGL(kern, dim3((unsigned)a.n_chunks), dim3(kChunkThreads), smem, s, a);
  return hipGetLastError();
}

template <typename T, int VPL, int U, int KT>
hipError_t launch_chunk_u(const ChunkArgs<T>& a, hipStream_t s) {
  constexpr int VEC = 16 / sizeof(T);
  constexpr int EP = kRowLanes * VPL;
  const size_t smem = chunk_smem<T>(a.D, a.E, a.max_rows, a.max_nk).total;
  const bool vec_ok = (a.E % VEC) == 0 && (reinterpret_cast<uintptr_t>(a.counters) % 16) == 0;
  if (vec_ok && a.E == EP) return launch_chunk_k<T, VPL, VEC, U, KT, true>(a, smem, s);
  if (vec_ok) return launch_chunk_k<T, VPL, VEC, U, KT, false>(a, smem, s);
  return launch_chunk_k<T, VPL, 1, U, KT, false>(a, smem, s);
}

template <typename T, int VPL>
hipError_t launch_chunk_vpl(const ChunkArgs<T>& a, int unroll, hipStream_t s) {
  if (a.n <= 4) {
    if (unroll >= 4) return launch_chunk_u<T, VPL, 4, 4>(a, s);
    if (unroll == 2) return launch_chunk_u<T, VPL, 2, 4>(a, s);
    return launch_chunk_u<T, VPL, 1, 4>(a, s);
  }
  if (unroll >= 4) return launch_chunk_u<T, VPL, 4, 8>(a, s);
  if (unroll == 2) return launch_chunk_u<T, VPL, 2, 8>(a, s);
  return launch_chunk_u<T, VPL, 1, 8>(a, s);
}

template <typename T>
hipError_t launch_path_chunks(const ChunkArgs<T>& a, int unroll, hipStream_t s) {
  if (a.n_chunks <= 0) return hipSuccess;
  if (a.E <= 16 * 4) return launch_chunk_vpl<T, 4>(a, unroll, s);
  if (a.E <= 16 * 8) return launch_chunk_vpl<T, 8>(a, unroll, s);
  return launch_chunk_vpl<T, 16>(a, unroll, s);
}

template hipError_t launch_path_chunks<float>(const ChunkArgs<float>&, int, hipStream_t);
template hipError_t launch_path_chunks<double>(const ChunkArgs<double>&, int, hipStream_t);

}  // namespace sugg
