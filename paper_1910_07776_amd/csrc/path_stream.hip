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
  size_t W, Wb, sm, e, L, kro, rk, kB, kop, total;
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
  s.kro = o; o += sizeof(int32_t) * (size_t)(max_nk + 1);
  s.rk = o;  o += sizeof(int16_t) * (size_t)max_rows;
  s.kB = o;  o += (size_t)max_nk;
  o = align_up(o, 16);
  s.kop = o; o += (size_t)max_nk * SUGG_MAX_OPTS;
  s.total = align_up(o, 16);
  return s;
}

size_t path_chunk_lds(size_t tsize, int D, int E, int max_rows, int max_nk) {
  return tsize == 4 ? chunk_smem<float>(D, E, max_rows, max_nk).total
                    : chunk_smem<double>(D, E, max_rows, max_nk).total;
}

template <typename T, int VPL, int VW, int U, int KT, bool FULL>
__global__ void __launch_bounds__(kChunkThreads) path_chunk_kernel(const ChunkArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NCH = VPL / VW;
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
  int32_t* kro = reinterpret_cast<int32_t*>(smem + ly.kro);
  int16_t* rk = reinterpret_cast<int16_t*>(smem + ly.rk);
  int8_t* kB = reinterpret_cast<int8_t*>(smem + ly.kB);
  uint8_t* kop = reinterpret_cast<uint8_t*>(smem + ly.kop);
  const Chunk ck = a.chunks[blockIdx.x];
  const int R = ck.R, nk = ck.nk;

  // rows: step i covers chunk rows [kGroups U i, kGroups U (i + 1)); lane
  // group g takes rows kGroups U i + kGroups u + g
  const int step = kGroups * U;
  const T* base_c = a.counters + ck.row0 * E;
  const T* base_y = a.cycles + ck.row0;
  auto load = [&](int base, T (&c)[U][NCH][VW], T (&cy)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int r = base + kGroups * u + g;
      r = r < R ? r : R - 1;   // rows past the chunk re-read its last row (never used)
      const T* rp = base_c + (int64_t)r * E;
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        const int cc = (l16 + kRowLanes * ch) * VW;
        if (FULL || cc < E) {
          const VecN<T, VW> q = *reinterpret_cast<const VecN<T, VW>*>(rp + cc);
#pragma unroll
          for (int v = 0; v < VW; ++v) c[u][ch][v] = q.v[v];
        } else {
#pragma unroll
          for (int v = 0; v < VW; ++v) c[u][ch][v] = T(1);
        }
      }
      cy[u] = base_y[r];
    }
  };
  T ca[U][NCH][VW], cb[U][NCH][VW];
  T cya[U], cyb[U];
  // the first two steps go out first: contiguous rows need no metadata
  load(0, ca, cya);
  if (step < R) load(step, cb, cyb);

  // model: weights, intercepts, column constants
  stage_weights<T, FULL>(a.W, a.ldw, D, E, EP, Wl, Wb, tid, kChunkThreads);
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
  // the chunk's kernels: first rows (relative to the chunk), B, global ids
  for (int j = tid; j <= nk; j += kChunkThreads)
    kro[j] = (int32_t)(a.row_off[ck.k0 + j] - ck.row0);
  for (int j = tid; j < nk; j += kChunkThreads) {
    const int B = a.nopts[ck.k0 + j];
    kB[j] = (int8_t)B;
    const int32_t* ids = a.opt_ids + a.opt_off[ck.k0 + j];
    for (int b = 0; b < B; ++b) kop[j * SUGG_MAX_OPTS + b] = (uint8_t)ids[b];
  }
  __syncthreads();
  // each row's kernel: the last one starting at or before it
  for (int r = tid; r < R; r += kChunkThreads) {
    int lo = 0, hi = nk - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (kro[mid] <= r) lo = mid;
      else hi = mid - 1;
    }
    rk[r] = (int16_t)lo;
  }
  __syncthreads();

  // ---- rows: Tier 1 features and Tier 2 chain edges into LDS ---------------
  bool bad = false;
  auto compute = [&](int base, const T (&c)[U][NCH][VW], const T (&cy)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = base + kGroups * u + g;
      if (r >= R) break;   // uniform per 16-lane group
      const int j = rk[r];
      const int B = kB[j];
      const int kb = kro[j];
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
      const uint8_t* ops = kop + j * SUGG_MAX_OPTS;
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
  for (int base = 0; base < R; base += 2 * step) {
    compute(base, ca, cya);
    if (base + 2 * step < R) load(base + 2 * step, ca, cya);
    if (base + step >= R) break;
    compute(base + step, cb, cyb);
    if (base + 3 * step < R) load(base + 3 * step, cb, cyb);
  }
  if (__ballot(bad) != 0 && lane == 0) atomicOr(a.status, (int)kStatusBadCounter);
  __syncthreads();

  // ---- compose: L(S) = sum over the bits b of S, ascending, of the edge
  // into S & (2^(b+1) - 1) (the fused kernel's order) ------------------------
  for (int r = tid; r < R; r += kChunkThreads) {
    const int j = rk[r];
    const int kb = kro[j];
    const uint32_t S = (uint32_t)(r - kb);
    const int B = kB[j];
    T L = T(0);
    for (int b = 0; b < B; ++b)
      if ((S >> b) & 1u) L += eb[kb + (int)(S & ((2u << b) - 1u))];
    Lb[r] = L;
    if (a.table) a.table[ck.row0 + r] = L;
  }
  if (!a.idx_out) return;
  __syncthreads();

  // ---- Tier 3: per kernel, one wave: per-lane best-first lists, merged ----
  for (int j = wave; j < nk; j += kWaves) {   // uniform per wave
    const int kb = kro[j];
    const int V = 1 << kB[j];
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

template <typename T, int VPL, int U, int KT>
hipError_t launch_chunk_u(const ChunkArgs<T>& a, hipStream_t s) {
  constexpr int VEC = 16 / sizeof(T);
  constexpr int EP = kRowLanes * VPL;
  const size_t smem = chunk_smem<T>(a.D, a.E, a.max_rows, a.max_nk).total;
  const bool vec_ok = (a.E % VEC) == 0 && (reinterpret_cast<uintptr_t>(a.counters) % 16) == 0;
  const dim3 grid((unsigned)a.n_chunks), block(kChunkThreads);
  if (smem > 64 * 1024) {
    for (const void* f : {reinterpret_cast<const void*>(path_chunk_kernel<T, VPL, VEC, U, KT, true>),
                          reinterpret_cast<const void*>(path_chunk_kernel<T, VPL, VEC, U, KT, false>),
                          reinterpret_cast<const void*>(path_chunk_kernel<T, VPL, 1, U, KT, false>)}) {
      const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
      if (e != hipSuccess) return e;
    }
  }
  (void)hipGetLastError();  // report only this launch's status
  if (vec_ok && a.E == EP)
    hipLaunchKernelGGL((path_chunk_kernel<T, VPL, VEC, U, KT, true>), grid, block, smem, s, a);
  else if (vec_ok)
    hipLaunchKernelGGL((path_chunk_kernel<T, VPL, VEC, U, KT, false>), grid, block, smem, s, a);
  else
    hipLaunchKernelGGL((path_chunk_kernel<T, VPL, 1, U, KT, false>), grid, block, smem, s, a);
  return hipGetLastError();
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
