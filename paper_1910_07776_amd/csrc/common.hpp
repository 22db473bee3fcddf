// Shared device helpers of the gfx950 kernels: wave64 lane arithmetic, DPP
// row reductions, the top-n entry type and its bitonic merge.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sugg.h"

namespace sugg {

constexpr int kWave = 64;
constexpr int kMaxSuggest = 8;   // longest suggestion list
constexpr int kRowLanes = 16;   // lanes that share one counter row (one DPP row)

enum StatusBits : int { kStatusBadCounter = 1, kStatusSingular = 2, kStatusBadIndex = 4 };

// One item of the ragged work list: nk kernels of equal B whose records are
// recs[first .. first+nk); R = nk << B rows.  row0 >= 0 when the kernels are
// adjacent in memory in record order (item row r is then row row0 + r).
struct alignas(16) Item {
  int64_t row0;
  int32_t first;
  int32_t nk;
  int32_t B;
  int32_t R;
  int32_t pad[2];
};

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Index of the most significant set bit, -1 for 0.
__device__ __forceinline__ int msb(uint32_t v) { return v ? 31 - __clz(v) : -1; }

// ---- DPP rotate within a row of 16 lanes (row_ror:n, n = 1..15) ----------
template <int N>
__device__ __forceinline__ float row_ror(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x120 + N, 0xF, 0xF, false));
}
template <int N>
__device__ __forceinline__ double row_ror(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, 0x120 + N, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, 0x120 + N, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 16 lanes of a DPP row; every lane receives a total, the value
// of lane 0 of the row is the one the kernels use (fixed association order).
template <typename T>
__device__ __forceinline__ T row_sum16(T v) {
  v += row_ror<8>(v);
  v += row_ror<4>(v);
  v += row_ror<2>(v);
  v += row_ror<1>(v);
  return v;
}

// ---- ranking entries -----------------------------------------------------
// A candidate (score v, index s); s < 0 marks an empty slot.  "better" orders
// by score descending, then index ascending; empty slots are worst.
template <typename T>
struct Entry {
  T v;
  int32_t s;
};

// Without short-circuit evaluation: branches there turn the selections of
// the callers into selections of addresses, which keeps the lists out of
// registers (in private memory).
template <typename T>
__device__ __forceinline__ bool better_vs(T av, int32_t as, T bv, int32_t bs) {
  return (as >= 0) & ((bs < 0) | (av > bv) | ((av == bv) & (as < bs)));
}

template <typename T>
__device__ __forceinline__ bool better(const Entry<T>& a, const Entry<T>& b) {
  return better_vs(a.v, a.s, b.v, b.s);
}

template <typename T>
__device__ __forceinline__ Entry<T> empty_entry() {
  Entry<T> e;
  e.v = T(0);
  e.s = -1;
  return e;
}

// Selections member by member on values read first (a conditional copy of
// the whole struct is lowered, for Entry<double>, through private memory).
template <typename T>
__device__ __forceinline__ void cswap(Entry<T>& a, Entry<T>& b) {
  // after: a is the better of the two
  const T av = a.v, bv = b.v;
  const int32_t as = a.s, bs = b.s;
  const bool sw = better_vs(bv, bs, av, as);
  a.v = sw ? bv : av;
  a.s = sw ? bs : as;
  b.v = sw ? av : bv;
  b.s = sw ? as : bs;
}

// Insert e into a best-first list of KT entries, dropping the worst.
template <typename T, int KT>
__device__ __forceinline__ void list_insert(Entry<T> (&L)[KT], Entry<T> e) {
#pragma unroll
  for (int i = 0; i < KT; ++i) cswap(L[i], e);
}

// Top-KT of two best-first lists: pairing A[i] with B[KT-1-i] and keeping the
// better forms a bitonic sequence holding the top KT; half-cleaners sort it.
template <typename T, int KT>
__device__ __forceinline__ void list_merge(Entry<T> (&A)[KT], const Entry<T> (&B)[KT]) {
#pragma unroll
  for (int i = 0; i < KT; ++i) {
    const T av = A[i].v, bv = B[KT - 1 - i].v;
    const int32_t as = A[i].s, bs = B[KT - 1 - i].s;
    const bool tb = better_vs(bv, bs, av, as);
    A[i].v = tb ? bv : av;
    A[i].s = tb ? bs : as;
  }
#pragma unroll
  for (int d = KT / 2; d >= 1; d >>= 1) {
#pragma unroll
    for (int i = 0; i < KT; ++i)
      if ((i & d) == 0) cswap(A[i], A[i + d]);
  }
}

template <typename T>
__device__ __forceinline__ Entry<T> shfl_xor_entry(const Entry<T>& e, int m) {
  Entry<T> r;
  r.v = __shfl_xor(e.v, m, kWave);
  r.s = __shfl_xor(e.s, m, kWave);
  return r;
}

// Butterfly merge of per-lane lists across aligned groups of G lanes
// (G a power of two <= 64); afterwards every lane of a group holds the
// group's top KT.
template <typename T, int KT>
__device__ __forceinline__ void group_merge(Entry<T> (&L)[KT], int G) {
  for (int m = 1; m < G; m <<= 1) {
    Entry<T> o[KT];
#pragma unroll
    for (int i = 0; i < KT; ++i) o[i] = shfl_xor_entry(L[i], m);
    list_merge<T, KT>(L, o);
  }
}

template <typename T> __device__ __forceinline__ T qnan();
template <> __device__ __forceinline__ float qnan<float>() { return __builtin_nanf(""); }
template <> __device__ __forceinline__ double qnan<double>() { return __builtin_nan(""); }

}  // namespace sugg
