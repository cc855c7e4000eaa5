// Right-preconditioned flexible GMRES on the device (Section 2.1, equation
// 'right-preconditioned'; GMRES as used in Section 4).  Every step of every
// batched slot runs without a host round trip: Gram-Schmidt products are
// reduced in a fixed order (partial sums per 2048-row block, then a fixed
// tree), the Givens rotations, the convergence test and the restart logic
// run in one work-group per slot, and finished slots are masked out.
//
// Per Arnoldi step j (classical Gram-Schmidt twice):
//   cast_in   r0 = V_j (or V_0 = w / beta after a restart)      -> T
//   ... V-cycle z0 = M r0 ...
//   cast_out  Z_j = z0;  spmv  w = A Z_j
//   dots1     h1 = V^T w, |w|^2
//   upd1      w -= V h1;  h2 = V^T w
//   upd2      w -= V h2;  |w|^2
//   givens    H column, rotations, |g_{j+1}| test, y = R^{-1} g at a cycle end
//   normalize V_{j+1} = w / h_{j+1,j}
//   xupd      x += Z y (cycle end);  spmv w = b - A x;  cycle: restart or stop
#include "devcommon.h"
#include "kernels.h"

namespace nnms {

constexpr int PSTRIDE = MMAX + 1;

__device__ __forceinline__ int row_of(int lb, int q) { return lb * VBLK + q * 256 + int(threadIdx.x); }

template <typename T>
__global__ __launch_bounds__(256) void k_cast_in(const KrylovDesc* __restrict__ d, int nd, int boff) {
  const int b = blockIdx.x + boff;
  const KrylovDesc D = d[find_desc(d, nd, b)];
  const KState* st = D.st;
  if (st->status != ST_RUNNING) return;
  const int lb = b - D.blk0, n = D.n;
  const bool pend = st->pending_v0 != 0;
  const double ib = pend ? 1.0 / st->beta : 0.0;
  const double* Vj = D.V + int64_t(st->j) * n;
  T* r0 = (T*)D.r0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int i = row_of(lb, q);
    if (i < n) {
      double v;
      if (pend) {
        v = D.w[i] * ib;
        D.V[i] = v;
      } else {
        v = Vj[i];
      }
      r0[i] = T(v);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_cast_out(const KrylovDesc* __restrict__ d, int nd) {
  const int b = blockIdx.x;
  const KrylovDesc D = d[find_desc(d, nd, b)];
  const KState* st = D.st;
  if (st->status != ST_RUNNING) return;
  const int lb = b - D.blk0, n = D.n;
  double* Zj = D.Z + int64_t(st->j) * n;
  const T* z0 = (const T*)D.z0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int i = row_of(lb, q);
    if (i < n) Zj[i] = double(z0[i]);
  }
}

// partial dots of w with V_0..V_j, and |w|^2
__global__ __launch_bounds__(256) void k_dots1(const KrylovDesc* __restrict__ d, int nd) {
  __shared__ double red[4][PSTRIDE];
  const int b = blockIdx.x;
  const KrylovDesc D = d[find_desc(d, nd, b)];
  const KState* st = D.st;
  if (st->status != ST_RUNNING) return;
  const int lb = b - D.blk0, n = D.n, j = st->j;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double wv[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int i = row_of(lb, q);
    wv[q] = i < n ? D.w[i] : 0.0;
  }
  for (int k = 0; k <= j; ++k) {
    const double* Vk = D.V + int64_t(k) * n;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = row_of(lb, q);
      if (i < n) s += Vk[i] * wv[q];
    }
    s = wave_sum(s);
    if (lane == 0) red[wave][k] = s;
  }
  {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) s += wv[q] * wv[q];
    s = wave_sum(s);
    if (lane == 0) red[wave][MMAX] = s;
  }
  __syncthreads();
  double* out = D.part1 + int64_t(lb) * PSTRIDE;
  for (int t = threadIdx.x; t < PSTRIDE; t += 256)
    if (t <= j || t == MMAX) out[t] = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
}

// h[k] = sum over blocks of part[b*stride + k], k <= j, in a fixed order
__device__ __forceinline__ void reduce_parts(const double* part, int stride, int nblk, int j, double* h_sh,
                                             double (*tmp)[MMAX]) {
  const int k = threadIdx.x & 63, p = threadIdx.x >> 6;
  if (k <= j) {
    double s = 0.0;
    for (int b = p; b < nblk; b += 4) s += part[int64_t(b) * stride + k];
    tmp[p][k] = s;
  }
  __syncthreads();
  if (threadIdx.x <= j) h_sh[threadIdx.x] = (tmp[0][threadIdx.x] + tmp[1][threadIdx.x]) + (tmp[2][threadIdx.x] + tmp[3][threadIdx.x]);
  __syncthreads();
}

// w -= V h1 (h1 from part1), then partial dots of the new w with V
__global__ __launch_bounds__(256) void k_upd1(const KrylovDesc* __restrict__ d, int nd) {
  __shared__ double h[MMAX];
  __shared__ double tmp[4][MMAX];
  __shared__ double red[4][MMAX];
  const int b = blockIdx.x;
  const KrylovDesc D = d[find_desc(d, nd, b)];
  KState* st = D.st;
  if (st->status != ST_RUNNING) return;
  const int lb = b - D.blk0, n = D.n, j = st->j;
  reduce_parts(D.part1, PSTRIDE, D.nblk, j, h, tmp);
  if (lb == 0 && threadIdx.x <= j) st->h1[threadIdx.x] = h[threadIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double wv[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int i = row_of(lb, q);
    wv[q] = i < n ? D.w[i] : 0.0;
  }
  for (int k = 0; k <= j; ++k) {
    const double* Vk = D.V + int64_t(k) * n;
    const double hk = h[k];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = row_of(lb, q);
      if (i < n) wv[q] -= Vk[i] * hk;
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int i = row_of(lb, q);
    if (i < n) D.w[i] = wv[q];
  }
  for (int k = 0; k <= j; ++k) {
    const double* Vk = D.V + int64_t(k) * n;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = row_of(lb, q);
      if (i < n) s += Vk[i] * wv[q];
    }
    s = wave_sum(s);
    if (lane == 0) red[wave][k] = s;
  }
  __syncthreads();
  double* out = D.part2 + int64_t(lb) * MMAX;
  if (threadIdx.x <= j) out[threadIdx.x] = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// w -= V h2 (h2 from part2); partial |w|^2
__global__ __launch_bounds__(256) void k_upd2(const KrylovDesc* __restrict__ d, int nd) {
  __shared__ double h[MMAX];
  __shared__ double tmp[4][MMAX];
  __shared__ double red[4];
  const int b = blockIdx.x;
  const KrylovDesc D = d[find_desc(d, nd, b)];
  KState* st = D.st;
  if (st->status != ST_RUNNING) return;
  const int lb = b - D.blk0, n = D.n, j = st->j;
  reduce_parts(D.part2, MMAX, D.nblk, j, h, tmp);
  if (lb == 0 && threadIdx.x <= j) st->h1[threadIdx.x] = st->h1[threadIdx.x] + h[threadIdx.x];
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int i = row_of(lb, q);
    if (i < n) {
      double wv = D.w[i];
      for (int k = 0; k <= j; ++k) wv -= D.V[int64_t(k) * n + i] * h[k];
      D.w[i] = wv;
      s += wv * wv;
    }
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) D.partn[lb] = (red[0] + red[1]) + (red[2] + red[3]);
}

// fixed-order sum of n values with one work-group
__device__ double block_sum(const double* p, int64_t stride, int n) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += p[int64_t(i) * stride];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_givens(const KrylovDesc* __restrict__ d) {
  const KrylovDesc D = d[blockIdx.x];
  KState* st = D.st;
  if (st->status != ST_RUNNING) return;
  const double hn2 = block_sum(D.partn, 1, D.nblk);
  const double wn2 = block_sum(D.part1 + MMAX, PSTRIDE, D.nblk);
  if (threadIdx.x != 0) return;
  const int j = st->j;
  double col[MMAX + 1];
  for (int k = 0; k <= j; ++k) col[k] = st->h1[k];
  const double hn = sqrt(hn2);
  col[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double c = st->cs[i], s = st->sn[i];
    const double t = c * col[i] + s * col[i + 1];
    col[i + 1] = -s * col[i] + c * col[i + 1];
    col[i] = t;
  }
  const double den = hypot(col[j], col[j + 1]);
  const double c = col[j] / den, s = col[j + 1] / den;
  st->cs[j] = c;
  st->sn[j] = s;
  col[j] = den;
  for (int k = 0; k <= j; ++k) st->R[k + j * MMAX] = col[k];
  st->g[j + 1] = -s * st->g[j];
  st->g[j] = c * st->g[j];
  st->its += 1;
  st->pending_v0 = 0;
  st->hnext = hn;
  const bool breakdown = hn <= 1e-14 * sqrt(wn2);
  const bool end = fabs(st->g[j + 1]) <= st->tol || breakdown || (j + 1 >= st->restart) || (st->its >= st->max_it);
  if (end) {
    st->cycle_end = 1;
    for (int k = j; k >= 0; --k) {
      double acc = st->g[k];
      for (int m = k + 1; m <= j; ++m) acc -= st->R[k + m * MMAX] * st->y[m];
      st->y[k] = acc / st->R[k + k * MMAX];
    }
  }
}

__global__ __launch_bounds__(256) void k_normalize(const KrylovDesc* __restrict__ d, int nd) {
  const int b = blockIdx.x;
  const KrylovDesc D = d[find_desc(d, nd, b)];
  const KState* st = D.st;
  if (st->status != ST_RUNNING || st->cycle_end) return;
  const int lb = b - D.blk0, n = D.n;
  const double hn = st->hnext;
  double* Vn = D.V + int64_t(st->j + 1) * n;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int i = row_of(lb, q);
    if (i < n) Vn[i] = D.w[i] / hn;
  }
}

__global__ __launch_bounds__(256) void k_xupd(const KrylovDesc* __restrict__ d, int nd) {
  __shared__ double y[MMAX];
  const int b = blockIdx.x;
  const KrylovDesc D = d[find_desc(d, nd, b)];
  const KState* st = D.st;
  if (st->status != ST_RUNNING || !st->cycle_end) return;
  const int lb = b - D.blk0, n = D.n, j = st->j;
  if (int(threadIdx.x) <= j) y[threadIdx.x] = st->y[threadIdx.x];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int i = row_of(lb, q);
    if (i < n) {
      double acc = 0.0;
      for (int k = 0; k <= j; ++k) acc += D.Z[int64_t(k) * n + i] * y[k];
      D.x[i] += acc;
    }
  }
}

__global__ __launch_bounds__(256) void k_cycle(const KrylovDesc* __restrict__ d) {
  const KrylovDesc D = d[blockIdx.x];
  KState* st = D.st;
  if (st->status != ST_RUNNING) return;
  double r2 = 0.0;
  if (st->cycle_end) r2 = block_sum(D.partr, 1, D.nblkr);
  if (threadIdx.x != 0) return;
  if (!st->cycle_end) {
    st->j += 1;
    return;
  }
  const double beta = sqrt(r2);
  st->cycles += 1;
  st->relres = beta / st->bnorm;
  st->cycle_end = 0;
  if (beta <= st->tol) {
    st->status = ST_CONVERGED;
  } else if (st->its >= st->max_it) {
    st->status = ST_MAXIT;
  } else {
    st->j = 0;
    st->pending_v0 = 1;
    st->beta = beta;
    st->g[0] = beta;
    for (int k = 1; k <= MMAX; ++k) st->g[k] = 0.0;
  }
}

// start of a solve: b_D = 0, w = b, x = 0, partial |b|^2
__global__ __launch_bounds__(256) void k_init(const KrylovDesc* __restrict__ d, int nd, int boff) {
  __shared__ double red[4];
  const int b = blockIdx.x + boff;
  const KrylovDesc D = d[find_desc(d, nd, b)];
  const int lb = b - D.blk0, n = D.n;
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int i = row_of(lb, q);
    if (i < n) {
      const double v = D.dmask[i] ? 0.0 : D.b[i];
      D.b[i] = v;
      D.w[i] = v;
      D.x[i] = 0.0;
      s += v * v;
    }
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) D.partn[lb] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_start(const KrylovDesc* __restrict__ d, double rtol, int restart, int max_it) {
  const KrylovDesc D = d[blockIdx.x];
  KState* st = D.st;
  const double b2 = block_sum(D.partn, 1, D.nblk);
  if (threadIdx.x != 0) return;
  const double bn = sqrt(b2);
  st->rtol = rtol;
  st->restart = restart;
  st->max_it = max_it;
  st->its = 0;
  st->cycles = 0;
  st->cycle_end = 0;
  st->j = 0;
  st->bnorm = bn;
  st->tol = rtol * bn;
  st->relres = 0.0;
  for (int k = 0; k <= MMAX; ++k) st->g[k] = 0.0;
  if (bn == 0.0) {
    st->status = ST_CONVERGED;
    st->pending_v0 = 0;
  } else {
    st->status = ST_RUNNING;
    st->pending_v0 = 1;
    st->beta = bn;
    st->g[0] = bn;
    st->relres = 1.0;
  }
}

__global__ void k_count_active(const KrylovDesc* d, int nd, int* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int c = 0;
    for (int s = 0; s < nd; ++s) c += (d[s].st->status == ST_RUNNING);
    *out = c;
  }
}

// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_krylov_cast_in(const KrylovDesc* d, int nd, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL((k_cast_in<T>), dim3(nblocks), dim3(256), 0, s, d, nd, 0);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_krylov_cast_out(const KrylovDesc* d, int nd, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL((k_cast_out<T>), dim3(nblocks), dim3(256), 0, s, d, nd);
  return hipGetLastError();
}
hipError_t launch_krylov_dots1(const KrylovDesc* d, int nd, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_dots1, dim3(nblocks), dim3(256), 0, s, d, nd);
  return hipGetLastError();
}
hipError_t launch_krylov_upd1(const KrylovDesc* d, int nd, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_upd1, dim3(nblocks), dim3(256), 0, s, d, nd);
  return hipGetLastError();
}
hipError_t launch_krylov_upd2(const KrylovDesc* d, int nd, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_upd2, dim3(nblocks), dim3(256), 0, s, d, nd);
  return hipGetLastError();
}
hipError_t launch_krylov_givens(const KrylovDesc* d, int nd, hipStream_t s) {
  hipLaunchKernelGGL(k_givens, dim3(nd), dim3(256), 0, s, d);
  return hipGetLastError();
}
hipError_t launch_krylov_normalize(const KrylovDesc* d, int nd, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_normalize, dim3(nblocks), dim3(256), 0, s, d, nd);
  return hipGetLastError();
}
hipError_t launch_krylov_xupd(const KrylovDesc* d, int nd, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_xupd, dim3(nblocks), dim3(256), 0, s, d, nd);
  return hipGetLastError();
}
hipError_t launch_krylov_cycle(const KrylovDesc* d, int nd, hipStream_t s) {
  hipLaunchKernelGGL(k_cycle, dim3(nd), dim3(256), 0, s, d);
  return hipGetLastError();
}
hipError_t launch_krylov_init_slot(const KrylovDesc* d, int nd, int boff, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_init, dim3(nblocks), dim3(256), 0, s, d, nd, boff);
  return hipGetLastError();
}
hipError_t launch_krylov_start_slot(const KrylovDesc* d1, double rtol, int restart, int max_it, hipStream_t s) {
  hipLaunchKernelGGL(k_start, dim3(1), dim3(256), 0, s, d1, rtol, restart, max_it);
  return hipGetLastError();
}
hipError_t launch_count_active(const KrylovDesc* d, int nd, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_count_active, dim3(1), dim3(64), 0, s, d, nd, out);
  return hipGetLastError();
}

template hipError_t launch_krylov_cast_in<double>(const KrylovDesc*, int, int, hipStream_t);
template hipError_t launch_krylov_cast_in<float>(const KrylovDesc*, int, int, hipStream_t);
template hipError_t launch_krylov_cast_out<double>(const KrylovDesc*, int, int, hipStream_t);
template hipError_t launch_krylov_cast_out<float>(const KrylovDesc*, int, int, hipStream_t);

}  // namespace nnms
