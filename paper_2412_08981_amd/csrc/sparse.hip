// CSR sparse matrix-vector products (level operators, residuals, the
// transposed transfer P^T) and the ELL-4 prolongation P (Section 2.3 of the
// paper: residuals r - J z and inter-level transfers of the V-cycle).
//
// SpMV maps one row to a group of G lanes of a wave (G = 16 covers the at
// most 15 entries per row of a P1 tetrahedral operator in one pass): the
// group reads the row's values and column ids contiguously, gathers x and
// reduces with cross-lane shuffles in a fixed order (deterministic).
#include "devcommon.h"
#include "kernels.h"

namespace nnms {

template <typename T, int G>
__global__ __launch_bounds__(256) void k_spmv(const SpmvDesc* __restrict__ d, int nd) {
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const SpmvDesc D = d[find_desc(d, nd, b)];
  if (!slot_active(D.st, D.when)) return;
  const int lb = b - D.blk0;
  const int row = lb * (256 / G) + int(threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  const GLOBAL T* __restrict__ x = gptr((const T*)D.x);
  if (D.x_jstride) x += int64_t(D.st->j) * D.x_jstride;
  const GLOBAL T* __restrict__ val = gptr((const T*)D.val);
  const GLOBAL int32_t* __restrict__ col = gptr(D.col);
  T sum = 0;
  if (row < D.n) {
    const int s = gptr(D.rp)[row], e = gptr(D.rp)[row + 1];
    for (int k = s + lane; k < e; k += G) sum += val[k] * x[col[k]];
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, G);
  T out = 0;
  if (lane == 0 && row < D.n) {
    out = D.r ? ((const T*)D.r)[row] - sum : sum;
    ((T*)D.y)[row] = out;
  }
  if (D.nrm) {  // partial sum of squares of this block's outputs (fixed order)
    __shared__ double red[4];
    double q = (lane == 0 && row < D.n) ? double(out) * double(out) : 0.0;
    q = wave_sum(q);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) D.nrm[lb] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// One lane's row of a sliced-ELL slice: the sum of val[64k] * x[col[64k]]
// over the steps k = k0, k0 + ks, ... < w, accumulated in that order.
template <typename T>
__device__ __forceinline__ T sell_row(const GLOBAL int32_t* col, const GLOBAL T* val, const GLOBAL T* x, int k0,
                                      int ks, int w) {
  T sum = 0;
#pragma unroll 4
  for (int k = k0; k < w; k += ks) sum += val[64 * k] * x[col[64 * k]];
  return sum;
}

// Sliced ELL (the level operators): one wave per 64-row slice, lane = row,
// the slice's columns stored column-major, so every load of a step is 64
// consecutive values; no row pointers, no cross-lane reduction, each row
// summed in order (deterministic).  Same descriptor as the CSR kernel with
// rp = slice offsets, col / val = the ELL arrays; 4 slices per block.
template <typename T>
__global__ __launch_bounds__(256) void k_sell(const SpmvDesc* __restrict__ d, int nd) {
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const SpmvDesc D = d[find_desc(d, nd, b)];
  if (!slot_active(D.st, D.when)) return;
  const int lb = b - D.blk0;
  const int lane = threadIdx.x & 63;
  const int slice = lb * 4 + (threadIdx.x >> 6);
  const int row = slice * 64 + lane;
  const GLOBAL T* __restrict__ x = gptr((const T*)D.x);
  if (D.x_jstride) x += int64_t(D.st->j) * D.x_jstride;
  T sum = 0;
  if (slice * 64 < D.n) {
    const int e0 = gptr(D.rp)[slice], w = (gptr(D.rp)[slice + 1] - e0) >> 6;
    sum = sell_row<T>(gptr(D.col) + e0 + lane, gptr((const T*)D.val) + e0 + lane, x, 0, 1, w);
  }
  T out = 0;
  if (row < D.n) {
    out = D.r ? ((const T*)D.r)[row] - sum : sum;
    ((T*)D.y)[row] = out;
  }
  if (D.nrm) {  // partial sum of squares of this block's outputs (fixed order)
    __shared__ double red[4];
    double q = row < D.n ? double(out) * double(out) : 0.0;
    q = wave_sum(q);
    if (lane == 0) red[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) D.nrm[lb] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// Sliced ELL with one slice per block: wave w of the four takes the slice's
// steps w, w + 4, ..., and the four partial sums of a row are added in a
// fixed order.  Four times the waves of k_sell with a quarter of the steps
// each, for matrices with few rows of many entries (P^T: ~30 per row),
// where one wave per slice leaves too few loads in flight.
template <typename T>
__global__ __launch_bounds__(256) void k_sell4(const SpmvDesc* __restrict__ d, int nd) {
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const SpmvDesc D = d[find_desc(d, nd, b)];
  if (!slot_active(D.st, D.when)) return;
  const int slice = b - D.blk0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = slice * 64 + lane;
  const GLOBAL T* __restrict__ x = gptr((const T*)D.x);
  if (D.x_jstride) x += int64_t(D.st->j) * D.x_jstride;
  T sum;
  {
    const int e0 = gptr(D.rp)[slice], w = (gptr(D.rp)[slice + 1] - e0) >> 6;
    sum = sell_row<T>(gptr(D.col) + e0 + lane, gptr((const T*)D.val) + e0 + lane, x, wave, 4, w);
  }
  __shared__ T part[4][64];
  part[wave][lane] = sum;
  __syncthreads();
  if (wave == 0) {
    const T s = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
    T out = 0;
    if (row < D.n) {
      out = D.r ? ((const T*)D.r)[row] - s : s;
      ((T*)D.y)[row] = out;
    }
    if (D.nrm) {  // partial sum of squares of this slice's outputs (fixed order)
      const double q = wave_sum(row < D.n ? double(out) * double(out) : 0.0);
      if (lane == 0) D.nrm[slice] = q;
    }
  }
}

// Column-sorted slices (the restriction P^T, whose rows gather ~30 fine
// entries from a few grid lines each): one 64-row slice per block.  The
// slice's entries are stored in column order, so the gathers of a wave fall
// on a few runs of consecutive fine entries instead of one scattered entry
// per row; each product goes to its row-major position in LDS, and after a
// barrier four lanes per row sum the row's products (lane q positions q,
// q + 4, ..., in order; the four partial sums added pairwise).
template <typename T>
__global__ __launch_bounds__(256) void k_csort(const SpmvDesc* __restrict__ d, int nd) {
  extern __shared__ __align__(16) unsigned char csort_lds[];
  T* prod = reinterpret_cast<T*>(csort_lds);
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const SpmvDesc D = d[find_desc(d, nd, b)];
  if (!slot_active(D.st, D.when)) return;
  const int slice = b - D.blk0;
  const int r0 = slice * 64;
  const GLOBAL int32_t* __restrict__ rp = gptr(D.rp);
  const int e0 = rp[r0], e1 = rp[min(r0 + 64, D.n)];
  const GLOBAL T* __restrict__ x = gptr((const T*)D.x) + gptr(D.base)[slice];
  if (D.x_jstride) x += int64_t(D.st->j) * D.x_jstride;
  const GLOBAL int32_t* __restrict__ key = gptr(D.col);
  const GLOBAL T* __restrict__ val = gptr((const T*)D.val);
  constexpr int U = 4;  // entries per lane with their loads in flight together
  constexpr int MASK = (1 << CSORT_SLOT_BITS) - 1;
  for (int e = e0 + int(threadIdx.x); e < e1; e += 256 * U) {
    int k[U];
    T w[U], xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = e + 256 * u;
      k[u] = q < e1 ? key[q] : 0;  // key 0: the slice's first column, read again
      w[u] = q < e1 ? val[q] : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = x[k[u] >> CSORT_SLOT_BITS];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e + 256 * u < e1) prod[k[u] & MASK] = w[u] * xv[u];
  }
  __syncthreads();
  const int r = r0 + int(threadIdx.x >> 2), q = threadIdx.x & 3;
  T sum = 0;
  if (r < D.n) {
    const int s0 = rp[r] - e0, s1 = rp[r + 1] - e0;
    for (int k = s0 + q; k < s1; k += 4) sum += prod[k];
  }
  sum += __shfl_xor(sum, 1, 4);
  sum += __shfl_xor(sum, 2, 4);
  if (q == 0 && r < D.n) ((T*)D.y)[r] = D.r ? ((const T*)D.r)[r] - sum : sum;
}

// ell[e] = csr[src[e]] (0 for padding, src < 0)
template <typename T>
__global__ __launch_bounds__(256) void k_gather_ell(const int32_t* __restrict__ src, const double* __restrict__ csr,
                                                    T* __restrict__ ell, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n) {
    const int32_t q = src[i];
    ell[i] = q >= 0 ? T(csr[q]) : T(0);
  }
}

template <typename T>
hipError_t launch_sell(const SpmvDesc* d, int nd, int nblocks, int split, hipStream_t s) {
  if (nd <= 0 || nblocks <= 0) return hipSuccess;
  if (split)
    hipLaunchKernelGGL((k_sell4<T>), dim3(nblocks), dim3(256), 0, s, d, nd);
  else
    hipLaunchKernelGGL((k_sell<T>), dim3(nblocks), dim3(256), 0, s, d, nd);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_ell(const int32_t* src, const double* csr, T* ell, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_gather_ell<T>), dim3((n + 255) / 256), dim3(256), 0, s, src, csr, ell, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_csort(const SpmvDesc* d, int nd, int nblocks, int cap, hipStream_t s) {
  if (nd <= 0 || nblocks <= 0) return hipSuccess;
  if (cap < 1 || cap > (1 << CSORT_SLOT_BITS)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_csort<T>), dim3(nblocks), dim3(256), size_t(cap) * sizeof(T), s, d, nd);
  return hipGetLastError();
}

template hipError_t launch_csort<double>(const SpmvDesc*, int, int, int, hipStream_t);
template hipError_t launch_csort<float>(const SpmvDesc*, int, int, int, hipStream_t);
template hipError_t launch_sell<double>(const SpmvDesc*, int, int, int, hipStream_t);
template hipError_t launch_sell<float>(const SpmvDesc*, int, int, int, hipStream_t);
template hipError_t launch_gather_ell<double>(const int32_t*, const double*, double*, int64_t, hipStream_t);
template hipError_t launch_gather_ell<float>(const int32_t*, const double*, float*, int64_t, hipStream_t);

template <typename T>
hipError_t launch_spmv(const SpmvDesc* d, int nd, int nblocks, int group, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  switch (group) {
    case 4: hipLaunchKernelGGL((k_spmv<T, 4>), dim3(nblocks), dim3(256), 0, s, d, nd); break;
    case 8: hipLaunchKernelGGL((k_spmv<T, 8>), dim3(nblocks), dim3(256), 0, s, d, nd); break;
    case 16: hipLaunchKernelGGL((k_spmv<T, 16>), dim3(nblocks), dim3(256), 0, s, d, nd); break;
    case 32: hipLaunchKernelGGL((k_spmv<T, 32>), dim3(nblocks), dim3(256), 0, s, d, nd); break;
    case 64: hipLaunchKernelGGL((k_spmv<T, 64>), dim3(nblocks), dim3(256), 0, s, d, nd); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// zf[i] += sum_a w[4i+a] zc[idx[4i+a]]: coarse-to-fine barycentric transfer.
template <typename T>
__global__ __launch_bounds__(256) void k_prolong(const ProlongDesc* __restrict__ d, int nd) {
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const ProlongDesc D = d[find_desc(d, nd, b)];
  if (!slot_active(D.st, WHEN_RUNNING)) return;
  const int i = (b - D.blk0) * 256 + threadIdx.x;
  if (i >= D.n) return;
  const int4 id = ((const int4*)D.idx)[i];
  const GLOBAL T* w = gptr((const T*)D.w) + int64_t(i) * 4;
  const GLOBAL T* zc = gptr((const T*)D.zc);
  T acc = w[0] * zc[id.x] + w[1] * zc[id.y] + w[2] * zc[id.z] + w[3] * zc[id.w];
  GLOBAL T* zf = gptr((T*)D.zf);
  zf[i] += acc;
}

template <typename T>
hipError_t launch_prolong(const ProlongDesc* d, int nd, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_prolong<T>), dim3(nblocks), dim3(256), 0, s, d, nd);
  return hipGetLastError();
}

template <typename T>
__global__ void k_fill(T* p, int64_t n, T v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) p[i] = v;
}

template <typename T>
hipError_t launch_fill(T* p, int64_t n, T v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL((k_fill<T>), dim3(int(blocks)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

template <typename A, typename B>
__global__ void k_cast(const A* a, B* b, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    b[i] = B(a[i]);
}

hipError_t launch_cast_d2f(const double* a, float* b, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL((k_cast<double, float>), dim3(int(blocks)), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}
hipError_t launch_cast_f2d(const float* a, double* b, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL((k_cast<float, double>), dim3(int(blocks)), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}

template hipError_t launch_spmv<double>(const SpmvDesc*, int, int, int, hipStream_t);
template hipError_t launch_spmv<float>(const SpmvDesc*, int, int, int, hipStream_t);
template hipError_t launch_prolong<double>(const ProlongDesc*, int, int, hipStream_t);
template hipError_t launch_prolong<float>(const ProlongDesc*, int, int, hipStream_t);
template hipError_t launch_fill<double>(double*, int64_t, double, hipStream_t);
template hipError_t launch_fill<float>(float*, int64_t, float, hipStream_t);
template hipError_t launch_fill<int32_t>(int32_t*, int64_t, int32_t, hipStream_t);

}  // namespace nnms

namespace nnms {
// plain streaming copy in 16-byte units (calibration of byte counters)
__global__ __launch_bounds__(256) void k_copy16(const int4* __restrict__ a, int4* __restrict__ b, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) b[i] = a[i];
}
hipError_t launch_copy16(const void* a, void* b, int64_t bytes, hipStream_t s) {
  const int64_t n = bytes / 16;
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 256 * 16);
  hipLaunchKernelGGL(k_copy16, dim3(int(blocks)), dim3(256), 0, s, (const int4*)a, (int4*)b, n);
  return hipGetLastError();
}
}  // namespace nnms

namespace nnms {
// read-only streaming reference: every work-item sums 16-byte chunks, eight
// loads in flight, and writes one value per work-group (the achievable read
// bandwidth of the memory system for a large resident array)
typedef int ivec4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_read16(const ivec4* __restrict__ a, int64_t n, int* out) {
  // each pass of a work-group reads 8 consecutive 4 KB stretches (one per
  // load in flight), so every stretch of DRAM is streamed in order
  constexpr int U = 8;
  int acc = 0;
  const int64_t stride = int64_t(gridDim.x) * 256 * U;
  for (int64_t base = int64_t(blockIdx.x) * 256 * U; base < n; base += stride) {
    ivec4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + u * 256 + threadIdx.x;
      v[u] = i < n ? __builtin_nontemporal_load(a + i) : ivec4{0, 0, 0, 0};
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc ^= __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) out[blockIdx.x * 4 + (threadIdx.x >> 6)] = acc;
}
hipError_t launch_read16(const void* a, int64_t bytes, int* out, int grid, hipStream_t s) {
  const int64_t n = bytes / 16;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_read16, dim3(grid), dim3(256), 0, s, (const ivec4*)a, n, out);
  return hipGetLastError();
}
}  // namespace nnms
