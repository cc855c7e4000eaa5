// Device helpers shared by the HIP kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include "devtypes.h"

namespace nnms {

// Pointers taken from descriptors are generic; accesses through them compile
// to flat instructions with 64-bit per-lane addresses, and flat loads also
// count as LDS operations, so every LDS wait would drain outstanding
// device-memory loads.  Kernels access device memory through
// global-address-space pointers instead.
#define GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLOBAL T* gptr(T* p) {
  return (GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ const GLOBAL T* gptr(const T* p) {
  return (const GLOBAL T*)p;
}

// Work-groups of a launch are handed to the eight XCDs in turn (block b to
// XCD b mod 8), and every XCD has its own L2.  This maps the hardware block
// index to a logical one so that each XCD works through one contiguous range
// of logical blocks (a bijection on [0, nb)): neighbouring rows, whose
// gathers touch neighbouring parts of the input vector, share an L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

// Index of the descriptor whose first block is the largest one <= b.
template <typename D>
__device__ __forceinline__ int find_desc(const D* d, int nd, int b) {
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (d[mid].blk0 <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ bool slot_active(const KState* st, int when) {
  if (!st) return true;
  if (st->status != ST_RUNNING) return false;
  return when == WHEN_RUNNING ? true : (st->cycle_end != 0);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ int atomic_load_acq(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int atomic_load_rlx(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_store_rel(int32_t* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// 16-byte chunk of a factor tile: 2 doubles or 4 floats.
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
template <typename F>
struct Chunk;
template <>
struct Chunk<double> {
  using type = dvec2;
  static constexpr int W = 2;
};
template <>
struct Chunk<float> {
  using type = fvec4;
  static constexpr int W = 4;
};

__device__ __forceinline__ double chunk_dot(const dvec2& a, const dvec2& y) { return a.x * y.x + a.y * y.y; }
__device__ __forceinline__ float chunk_dot(const fvec4& a, const fvec4& y) {
  return a.x * y.x + a.y * y.y + a.z * y.z + a.w * y.w;
}

// Offset of element (r, c) inside a 64x64 tile stored column-group-major:
// groups of W adjacent columns, each group holding 64 rows of W values, so a
// wave reading one 16-byte chunk per lane (lane = row) is fully coalesced.
template <typename F>
__device__ __host__ __forceinline__ int tile_off(int r, int c) {
  constexpr int W = 16 / sizeof(F);
  return ((c / W) * 64 + r) * W + (c % W);
}

}  // namespace nnms
