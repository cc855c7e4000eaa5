// Dense subdomain matrices J_p = R_p J R_p^T (Section 2.2) and their batched
// LU factorisation without pivoting (the matrices are SPD principal
// submatrices; every pivot is checked to be positive).
//
// Layout: a subdomain of n rows is padded to N = ceil(n/64) tiles per side
// (padding rows get a unit diagonal).  Tile (i, j) of the N x N grid holds
// L_ij below the diagonal and U_ij above it; the diagonal tile holds
// inv(U_ii), and N extra tiles hold inv(L_ii) -- the inverted diagonal
// blocks turn every step of the triangular solves into a 64x64
// matrix-vector product.
//
// Right-looking blocked LU, one launch triple per block column k:
//   diag   factor A_kk = L_kk U_kk in LDS, invert both triangles;
//   panel  L_ik = A_ik inv(U_kk),  U_ki = inv(L_kk) A_ki      (MFMA);
//   update A_ij -= L_ik U_kj for i, j > k                      (MFMA).
#include "devcommon.h"
#include "kernels.h"

namespace nnms {

constexpr int LDP = 65;  // LDS row pitch

template <typename F>
struct Mma;
template <>
struct Mma<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output element v of `lane` is row lane/16 + 4v, column lane%16
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct Mma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output element v of `lane` is row 4*(lane/16) + v, column lane%16
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

template <typename F>
__device__ __forceinline__ void tile_to_lds(const F* g, F (*s)[LDP]) {
  using C = typename Chunk<F>::type;
  constexpr int W = Chunk<F>::W;
  const C* gc = (const C*)g;
  for (int q = threadIdx.x; q < TILE_ELEMS / W; q += 256) {
    const int cg = q / 64, r = q % 64;
    const C v = gc[q];
    const F* e = (const F*)&v;
#pragma unroll
    for (int k = 0; k < W; ++k) s[r][cg * W + k] = e[k];
  }
}

template <typename F>
__device__ __forceinline__ void lds_to_tile(F (*s)[LDP], F* g) {
  using C = typename Chunk<F>::type;
  constexpr int W = Chunk<F>::W;
  C* gc = (C*)g;
  for (int q = threadIdx.x; q < TILE_ELEMS / W; q += 256) {
    const int cg = q / 64, r = q % 64;
    C v;
    F* e = (F*)&v;
#pragma unroll
    for (int k = 0; k < W; ++k) e[k] = s[r][cg * W + k];
    gc[q] = v;
  }
}

// ---------------------------------------------------------------------------
// extraction: thread per local row; zero fill happens before (k_fill)
// ---------------------------------------------------------------------------
template <typename F>
__global__ __launch_bounds__(256) void k_extract(const FacDesc* __restrict__ d) {
  const FacDesc D = d[blockIdx.y];
  const int k = blockIdx.x * 256 + threadIdx.x;
  const int npad = D.N * 64;
  if (k >= npad) return;
  F* fac = (F*)D.fac;
  const size_t N = D.N;
  if (k >= D.n) {  // padding: unit diagonal
    fac[(size_t(k / 64) * N + k / 64) * TILE_ELEMS + tile_off<F>(k % 64, k % 64)] = F(1);
    return;
  }
  const int g0 = D.gidx[k];
  const int g = g0 >= 0 ? g0 : -g0 - 2;
  const int s = D.rp[g], e = D.rp[g + 1];
  const int* lc = D.ext_lc + D.ext_rs[k];
  const int ti = k / 64, r = k % 64;
  for (int q = s; q < e; ++q) {
    const int c = lc[q - s];
    if (c < 0) continue;
    fac[(size_t(ti) * N + c / 64) * TILE_ELEMS + tile_off<F>(r, c % 64)] = F(D.val[q]);
  }
}

template <typename F>
hipError_t launch_extract(const FacDesc* d, int nd, int maxn, hipStream_t s) {
  if (nd <= 0 || maxn <= 0) return hipSuccess;
  const int npad = ((maxn + 63) / 64) * 64;
  hipLaunchKernelGGL((k_extract<F>), dim3((npad + 255) / 256, nd), dim3(256), 0, s, d);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// diagonal tile: LU, then inv(L_kk) (unit lower) and inv(U_kk).
// LU: work-item c < 64 keeps column c in registers; at step c it scales its
// column below the diagonal and publishes the multipliers through LDS, and
// every column to its right applies the rank-1 update.  Inverses: one
// work-item per column of inv(L) (items 0..63) and of inv(U) (items
// 64..127), each column in registers, the factor rows read from LDS as
// broadcasts; loops are unrolled so that the register columns have fixed
// indices.
// ---------------------------------------------------------------------------
template <typename F>
__global__ __launch_bounds__(256) void k_lu_diag(const FacDesc* __restrict__ d, int k, int* err) {
  const FacDesc D = d[blockIdx.x];
  if (k >= D.N) return;
  __shared__ F a[64][LDP];
  __shared__ F lbuf[64];
  const int tid = threadIdx.x;
  const size_t N = D.N;
  F* fac = (F*)D.fac;
  F* tkk = fac + (size_t(k) * N + k) * TILE_ELEMS;
  F* linv = fac + (N * N + k) * TILE_ELEMS;
  tile_to_lds<F>(tkk, a);
  __syncthreads();
  F col[64];
  if (tid < 64) {
#pragma unroll
    for (int r = 0; r < 64; ++r) col[r] = a[r][tid];
  }
#pragma unroll
  for (int c = 0; c < 64; ++c) {
    if (tid == c) {
      const F piv = col[c];
      if (!(piv > F(0) && piv < F(INFINITY))) atomicOr(err, 1);
      const F rp = F(1) / piv;
#pragma unroll
      for (int r = c + 1; r < 64; ++r) {
        col[r] *= rp;
        lbuf[r] = col[r];
      }
    }
    __syncthreads();
    if (tid > c && tid < 64) {
      const F u = col[c];
#pragma unroll
      for (int r = c + 1; r < 64; ++r) col[r] -= lbuf[r] * u;
    }
    __syncthreads();
  }
  if (tid < 64) {
#pragma unroll
    for (int r = 0; r < 64; ++r) a[r][tid] = col[r];
  }
  __syncthreads();
  F x[64];
  if (tid < 64) {  // column c of inv(L): x_r = [r==c] - sum_{q<r} L_rq x_q
    const int c = tid;
#pragma unroll
    for (int r = 0; r < 64; ++r) {
      F s = (r == c) ? F(1) : F(0);
#pragma unroll
      for (int q = 0; q < r; ++q) s -= a[r][q] * x[q];
      x[r] = (r >= c) ? s : F(0);
    }
  } else if (tid < 128) {  // column c of inv(U): x_r = ([r==c] - sum_{q>r} U_rq x_q) / U_rr
    const int c = tid - 64;
#pragma unroll
    for (int r = 63; r >= 0; --r) {
      F s = (r == c) ? F(1) : F(0);
#pragma unroll
      for (int q = r + 1; q < 64; ++q) s -= a[r][q] * x[q];
      x[r] = (r <= c) ? s / a[r][r] : F(0);
    }
  }
  __syncthreads();  // every column read the factor: reuse a for inv(U), lbuf-free
  if (tid >= 64 && tid < 128) {
#pragma unroll
    for (int r = 0; r < 64; ++r) a[r][tid - 64] = x[r];
  }
  __syncthreads();
  lds_to_tile<F>(a, tkk);
  __syncthreads();
  if (tid < 64) {
#pragma unroll
    for (int r = 0; r < 64; ++r) a[r][tid] = x[r];
  }
  __syncthreads();
  lds_to_tile<F>(a, linv);
}

// ---------------------------------------------------------------------------
// C (=|-=) A * B on 64x64 tiles with MFMA 16x16x4; wave w owns the 32x32
// quadrant (w/2, w%2) of C.  A, B staged in LDS.
// ---------------------------------------------------------------------------
template <typename F>
__device__ __forceinline__ void tile_mma(F (*As)[LDP], F (*Bs)[LDP], typename Mma<F>::acc_t (&acc)[2][2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int R0 = (wave >> 1) * 32, C0 = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll 4
  for (int kk = 0; kk < 16; ++kk) {
    const int kc = kk * 4 + lk;
    F a0 = As[R0 + lr][kc], a1 = As[R0 + 16 + lr][kc];
    F b0 = Bs[kc][C0 + lr], b1 = Bs[kc][C0 + 16 + lr];
    acc[0][0] = Mma<F>::op(a0, b0, acc[0][0]);
    acc[0][1] = Mma<F>::op(a0, b1, acc[0][1]);
    acc[1][0] = Mma<F>::op(a1, b0, acc[1][0]);
    acc[1][1] = Mma<F>::op(a1, b1, acc[1][1]);
  }
}

template <typename F>
__device__ __forceinline__ void acc_to_lds(typename Mma<F>::acc_t (&acc)[2][2], F (*Cs)[LDP]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int R0 = (wave >> 1) * 32, C0 = (wave & 1) * 32;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) Cs[R0 + rb * 16 + Mma<F>::row(lane, v)][C0 + cb * 16 + (lane & 15)] = acc[rb][cb][v];
}

template <typename F>
__device__ __forceinline__ void lds_to_acc(F (*Cs)[LDP], typename Mma<F>::acc_t (&acc)[2][2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int R0 = (wave >> 1) * 32, C0 = (wave & 1) * 32;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[rb][cb][v] = Cs[R0 + rb * 16 + Mma<F>::row(lane, v)][C0 + cb * 16 + (lane & 15)];
}

// panel: blockIdx.x < nr -> L_{k+1+x, k} = A * inv(U_kk);  else U_{k, k+1+x'} = inv(L_kk) * A
template <typename F>
__global__ __launch_bounds__(256) void k_lu_panel(const FacDesc* __restrict__ d, int k) {
  const FacDesc D = d[blockIdx.y];
  const int nr = D.N - k - 1;
  if (nr <= 0 || int(blockIdx.x) >= 2 * nr) return;
  __shared__ F As[64][LDP], Bs[64][LDP];
  const size_t N = D.N;
  F* fac = (F*)D.fac;
  F* target;
  if (int(blockIdx.x) < nr) {
    const int i = k + 1 + blockIdx.x;
    target = fac + (size_t(i) * N + k) * TILE_ELEMS;
    tile_to_lds<F>(target, As);
    tile_to_lds<F>(fac + (size_t(k) * N + k) * TILE_ELEMS, Bs);
  } else {
    const int j = k + 1 + (blockIdx.x - nr);
    target = fac + (size_t(k) * N + j) * TILE_ELEMS;
    tile_to_lds<F>(fac + (N * N + k) * TILE_ELEMS, As);
    tile_to_lds<F>(target, Bs);
  }
  __syncthreads();
  typename Mma<F>::acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = typename Mma<F>::acc_t{0, 0, 0, 0};
  tile_mma<F>(As, Bs, acc);
  __syncthreads();
  acc_to_lds<F>(acc, As);
  __syncthreads();
  lds_to_tile<F>(As, target);
}

// update: A_ij -= L_ik U_kj for all i, j in k+1..N-1
template <typename F>
__global__ __launch_bounds__(256) void k_lu_update(const FacDesc* __restrict__ d, int k) {
  const FacDesc D = d[blockIdx.y];
  const int nr = D.N - k - 1;
  if (nr <= 0 || int(blockIdx.x) >= nr * nr) return;
  __shared__ F As[64][LDP], Bs[64][LDP];
  const int i = k + 1 + blockIdx.x / nr, j = k + 1 + blockIdx.x % nr;
  const size_t N = D.N;
  F* fac = (F*)D.fac;
  F* target = fac + (size_t(i) * N + j) * TILE_ELEMS;
  typename Mma<F>::acc_t acc[2][2];
  tile_to_lds<F>(target, As);
  __syncthreads();
  lds_to_acc<F>(As, acc);
  __syncthreads();
  tile_to_lds<F>(fac + (size_t(i) * N + k) * TILE_ELEMS, As);
  tile_to_lds<F>(fac + (size_t(k) * N + j) * TILE_ELEMS, Bs);
  __syncthreads();
  // C - A B: negate A on the fly
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = -acc[a][b];
  tile_mma<F>(As, Bs, acc);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = -acc[a][b];
  __syncthreads();
  acc_to_lds<F>(acc, As);
  __syncthreads();
  lds_to_tile<F>(As, target);
}

template <typename F>
hipError_t launch_lu_step(const FacDesc* d, int nd, int k, int maxN, int* err, hipStream_t s) {
  if (nd <= 0 || k >= maxN) return hipSuccess;
  hipLaunchKernelGGL((k_lu_diag<F>), dim3(nd), dim3(256), 0, s, d, k, err);
  const int nr = maxN - k - 1;
  if (nr > 0) {
    hipLaunchKernelGGL((k_lu_panel<F>), dim3(2 * nr, nd), dim3(256), 0, s, d, k);
    hipLaunchKernelGGL((k_lu_update<F>), dim3(nr * nr, nd), dim3(256), 0, s, d, k);
  }
  return hipGetLastError();
}

template hipError_t launch_extract<double>(const FacDesc*, int, int, hipStream_t);
template hipError_t launch_extract<float>(const FacDesc*, int, int, hipStream_t);
template hipError_t launch_lu_step<double>(const FacDesc*, int, int, int, int*, hipStream_t);
template hipError_t launch_lu_step<float>(const FacDesc*, int, int, int, int*, hipStream_t);

}  // namespace nnms
