// Dense subdomain matrices J_p = R_p J R_p^T (Section 2.2) and their batched
// LU factorisation without pivoting (the matrices are SPD principal
// submatrices; every pivot is checked to be positive).
//
// Layout: a subdomain of n rows is padded to N = ceil(n/64) tiles per side
// (padding rows get a unit diagonal).  Tile (i, j) of the N x N grid holds
// L_ij below the diagonal and U_ij above it; the diagonal tile holds
// inv(U_ii), and N extra tiles hold inv(L_ii) -- the inverted diagonal
// blocks turn every step of the triangular solves into a 64x64
// matrix-vector product.  Then 2 floor(N/2) tiles hold the coupling blocks
// of the inverses of the 128 x 128 diagonal blocks of tile pairs (below).
//
// Right-looking LU blocked twice: 64-wide tile columns, grouped into blocks
// of LU_DEPTH tile columns.  For block column k0 .. k0+D-1 and each k in it:
//   diag   A_kk -= sum_{k0<=s<k} L_ks U_sk, then A_kk = L_kk U_kk in
//          registers, invert both triangles;
//   panel  A_ik -= sum_s L_is U_sk, L_ik = A_ik inv(U_kk)      (i > k),
//          A_kj -= sum_s L_ks U_sj, U_kj = inv(L_kk) A_kj      (j > k);
// then one trailing update A_ij -= sum_{s in block} L_is U_sj for every i, j
// past the block, so each trailing tile is read and written once per D tile
// columns instead of once per tile column.  Every product runs on MFMA.
#include "devcommon.h"
#include "kernels.h"

namespace nnms {

constexpr int LDP = 65;  // LDS row pitch
constexpr int LU_DEPTH = 6;  // tile columns per trailing update (of 4, 6 and 8 the fastest)

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

// whole-tile copies between global memory and LDS by a work-group of 256:
// every load of the thread is issued before the first write
template <typename F>
__device__ __forceinline__ void tile_to_lds(const GLOBAL F* g, F (*s)[LDP]) {
  using C = typename Chunk<F>::type;
  constexpr int W = Chunk<F>::W, NC = TILE_ELEMS / W / 256;
  const GLOBAL C* gc = (const GLOBAL C*)g;
  C v[NC];
#pragma unroll
  for (int u = 0; u < NC; ++u) v[u] = gc[threadIdx.x + 256 * u];
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    const int q = threadIdx.x + 256 * u, cg = q / 64, r = q % 64;
#pragma unroll
    for (int k = 0; k < W; ++k) s[r][cg * W + k] = v[u][k];
  }
}

template <typename F>
__device__ __forceinline__ void lds_to_tile(F (*s)[LDP], GLOBAL F* g) {
  using C = typename Chunk<F>::type;
  constexpr int W = Chunk<F>::W, NC = TILE_ELEMS / W / 256;
  GLOBAL C* gc = (GLOBAL C*)g;
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    const int q = threadIdx.x + 256 * u, cg = q / 64, r = q % 64;
    C v;
#pragma unroll
    for (int k = 0; k < W; ++k) v[k] = s[r][cg * W + k];
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
// C += A * B on 64x64 tiles staged in LDS, MFMA 16x16x4; wave w owns the
// 32x32 quadrant (w/2, w%2) of C.  Quadrant accumulators, here and in the
// products from global memory below, hold rows R0 + 16 rb + (MFMA row) and
// columns C0 + 2 lr + cb (lr = lane % 16, cb = 0, 1): a lane's two column
// blocks are adjacent columns, one 8- or 16-byte piece of a tile row.
// ---------------------------------------------------------------------------
template <typename F>
struct Pair;
template <>
struct Pair<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Pair<float> {
  typedef float type __attribute__((ext_vector_type(2)));
};

template <typename F>
__device__ __forceinline__ void tile_mma(F (*As)[LDP], F (*Bs)[LDP], typename Mma<F>::acc_t (&acc)[2][2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int R0 = (wave >> 1) * 32, C0 = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll 4
  for (int kk = 0; kk < 16; ++kk) {
    const int kc = kk * 4 + lk;
    F a0 = As[R0 + lr][kc], a1 = As[R0 + 16 + lr][kc];
    F b0 = Bs[kc][C0 + 2 * lr], b1 = Bs[kc][C0 + 2 * lr + 1];
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
      for (int v = 0; v < 4; ++v) Cs[R0 + rb * 16 + Mma<F>::row(lane, v)][C0 + 2 * (lane & 15) + cb] = acc[rb][cb][v];
}

// ---------------------------------------------------------------------------
// Products with operands read straight from the tiles in global memory (no
// LDS, no barriers).  Wave w owns the 32x32 quadrant (w/2, w%2) of the 64x64
// output; the accumulator holds the quadrant in MFMA output layout.
// ---------------------------------------------------------------------------
template <typename F>
__device__ __forceinline__ void acc_load(const GLOBAL F* __restrict__ T, typename Mma<F>::acc_t (&acc)[2][2]) {
  using P = typename Pair<F>::type;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int R0 = (wave >> 1) * 32, C0 = (wave & 1) * 32;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const P x = *(const GLOBAL P*)(T + tile_off<F>(R0 + rb * 16 + Mma<F>::row(lane, v), C0 + 2 * (lane & 15)));
      acc[rb][0][v] = x[0];
      acc[rb][1][v] = x[1];
    }
}

template <typename F>
__device__ __forceinline__ void acc_store(typename Mma<F>::acc_t (&acc)[2][2], GLOBAL F* __restrict__ T) {
  using P = typename Pair<F>::type;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int R0 = (wave >> 1) * 32, C0 = (wave & 1) * 32;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      P x;
      x[0] = acc[rb][0][v];
      x[1] = acc[rb][1][v];
      *(GLOBAL P*)(T + tile_off<F>(R0 + rb * 16 + Mma<F>::row(lane, v), C0 + 2 * (lane & 15))) = x;
    }
}

template <typename F>
__device__ __forceinline__ void acc_negate(typename Mma<F>::acc_t (&acc)[2][2]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = -acc[a][b];
}

// MFMA operands of 16 consecutive k of one quadrant, in NS = 4 / W
// sub-groups of 4W k: 16-byte A chunks (W consecutive k of one row) and B
// pairs (one k, the lane's two adjacent columns).  In sub-group u, step
// s = 0 .. W-1 of lane (lr, lk) takes k = 16 g + 4W u + W lk + s, so one A
// chunk serves W MFMA steps; the sum over k is the same, only the order in
// which the MFMAs add the k values differs.
template <typename F>
struct Frag {
  static constexpr int W = Chunk<F>::W, NS = 4 / W;
  typename Chunk<F>::type a[NS][2];
  typename Pair<F>::type b[NS][W];
};

// group g (0..3) of the 64-deep product Lt * Ut
template <typename F>
__device__ __forceinline__ void frag_load(Frag<F>& f, const GLOBAL F* __restrict__ Lt, const GLOBAL F* __restrict__ Ut, int g) {
  using C = typename Chunk<F>::type;
  using P = typename Pair<F>::type;
  constexpr int W = Chunk<F>::W, NS = 4 / W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int R0 = (wave >> 1) * 32, C0 = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    const GLOBAL C* la = (const GLOBAL C*)Lt + (16 / W * g + 4 * u + lk) * 64 + R0 + lr;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) f.a[u][rb] = la[16 * rb];
    const GLOBAL F* ub = Ut + tile_off<F>(16 * g + 4 * W * u + W * lk, C0 + 2 * lr);
#pragma unroll
    for (int s = 0; s < W; ++s) f.b[u][s] = *(const GLOBAL P*)(ub + W * s);
  }
}

template <typename F>
__device__ __forceinline__ void frag_mma(const Frag<F>& f, typename Mma<F>::acc_t (&acc)[2][2]) {
  constexpr int W = Chunk<F>::W, NS = 4 / W;
#pragma unroll
  for (int u = 0; u < NS; ++u)
#pragma unroll
    for (int s = 0; s < W; ++s)
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = Mma<F>::op(f.a[u][rb][s], f.b[u][s][cb], acc[rb][cb]);
}

// acc += sum_{s<depth} Ls(s) * Us(s), where Ls(s) = a + lt0 + s*lstep tiles and
// Us(s) = b + ut0 + s*ustep tiles; operand loads run one group ahead.
template <typename F>
__device__ __forceinline__ void acc_add_products(typename Mma<F>::acc_t (&acc)[2][2], const GLOBAL F* __restrict__ a,
                                                 size_t lt0, size_t lstep, const GLOBAL F* __restrict__ b, size_t ut0,
                                                 size_t ustep, int depth) {
  if (depth <= 0) return;
  const int ng = 4 * depth;
  Frag<F> f0, f1;
  frag_load<F>(f0, a + lt0 * TILE_ELEMS, b + ut0 * TILE_ELEMS, 0);
  for (int g = 0; g < ng; g += 2) {
    {
      const int h = g + 1, s = h >> 2;  // ng is even: h < ng
      frag_load<F>(f1, a + (lt0 + s * lstep) * TILE_ELEMS, b + (ut0 + s * ustep) * TILE_ELEMS, h & 3);
    }
    frag_mma<F>(f0, acc);
    if (g + 2 < ng) {
      const int h = g + 2, s = h >> 2;
      frag_load<F>(f0, a + (lt0 + s * lstep) * TILE_ELEMS, b + (ut0 + s * ustep) * TILE_ELEMS, h & 3);
    }
    frag_mma<F>(f1, acc);
  }
}

template <typename F>
__device__ __forceinline__ void acc_add_products(typename Mma<F>::acc_t (&acc)[2][2], const GLOBAL F* __restrict__ fac,
                                                 size_t lt0, size_t lstep, size_t ut0, size_t ustep, int depth) {
  acc_add_products<F>(acc, fac, lt0, lstep, fac, ut0, ustep, depth);
}

// acc = T - sum_{s<depth} Ls(s) * Us(s)
template <typename F>
__device__ __forceinline__ void acc_updated_tile(typename Mma<F>::acc_t (&acc)[2][2], const GLOBAL F* __restrict__ fac,
                                                 size_t tt, size_t lt0, size_t lstep, size_t ut0, size_t ustep,
                                                 int depth) {
  acc_load<F>(fac + tt * TILE_ELEMS, acc);
  acc_negate<F>(acc);
  acc_add_products<F>(acc, fac, lt0, lstep, ut0, ustep, depth);
  acc_negate<F>(acc);
}

// ---------------------------------------------------------------------------
// diagonal tile: pending in-block updates, LU, then inv(L_kk) (unit lower)
// and inv(U_kk), all in LDS.  Everything here is on the critical path of the
// factorisation (one work-group per subdomain), so the kernel is built for
// latency and small code:
//   LU in four 16-column steps: one wave factors the 16-wide panel (lane r
//   keeps row r's 16 entries in registers; pivot-row values come by scalar
//   broadcast), one wave solves U12 = inv(L11) A12 (a work-item per column),
//   and the four waves update the trailing block with MFMA (K = 16);
//   inverses: the 16x16 diagonal blocks by column-parallel substitution,
//   then the off-diagonal blocks one block diagonal at a time,
//   X_ij = -X_ii sum_m L_im X_mj (and likewise for U), on MFMA.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bcast(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ double bcast(double x, int l) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane(int(v), l), hi = __builtin_amdgcn_readlane(int(v >> 32), l);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

// acc -= (or +=) A(r0.., k0..k0+15) * B(k0.., c0..), 16x16 output, K = 16, operands in LDS
template <typename F, bool SUB>
__device__ __forceinline__ void mma16(F (*A)[LDP], int ar, int ak, F (*B)[LDP], int bk, int bc,
                                      typename Mma<F>::acc_t& acc) {
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const F av = A[ar + lr][ak + 4 * kk + lk];
    acc = Mma<F>::op(SUB ? -av : av, B[bk + 4 * kk + lk][bc + lr], acc);
  }
}

template <typename F>
__device__ __forceinline__ void acc16_load(F (*C)[LDP], int r0, int c0, typename Mma<F>::acc_t& acc) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int v = 0; v < 4; ++v) acc[v] = C[r0 + Mma<F>::row(lane, v)][c0 + (lane & 15)];
}

template <typename F>
__device__ __forceinline__ void acc16_store(typename Mma<F>::acc_t acc, F (*C)[LDP], int r0, int c0, F scale) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int v = 0; v < 4; ++v) C[r0 + Mma<F>::row(lane, v)][c0 + (lane & 15)] = scale * acc[v];
}

template <typename F>
__global__ __launch_bounds__(256) void k_lu_diag(const FacDesc* __restrict__ d, int k0, int k, int* err) {
  const FacDesc D = d[blockIdx.x];
  if (k >= D.N) return;
  __shared__ F a[64][LDP];  // A, then L (strictly lower) and U
  __shared__ F X[64][LDP];  // inv(L)
  __shared__ F Y[64][LDP];  // inv(U)
  __shared__ F T[4][16][LDP];  // per-wave 16x16 product scratch
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const size_t N = D.N;
  GLOBAL F* fac = gptr((F*)D.fac);
  GLOBAL F* tkk = fac + (size_t(k) * N + k) * TILE_ELEMS;
  GLOBAL F* linv = fac + (N * N + k) * TILE_ELEMS;
  if (k > k0) {  // pending updates of this block column
    typename Mma<F>::acc_t acc[2][2];
    acc_updated_tile<F>(acc, fac, size_t(k) * N + k, size_t(k) * N + k0, 1, size_t(k0) * N + k, N, k - k0);
    acc_to_lds<F>(acc, a);
  } else {
    tile_to_lds<F>(tkk, a);
  }
  for (int q = tid; q < 64 * 64; q += 256) X[q >> 6][q & 63] = F(0), Y[q >> 6][q & 63] = F(0);
  __syncthreads();

  for (int p = 0; p < 4; ++p) {
    const int c0 = 16 * p;
    if (wave == 0) {  // panel rows c0..63, columns c0..c0+15
      F pr[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) pr[q] = a[lane][c0 + q];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        const int j = c0 + jj;
        const F piv = bcast(pr[jj], j);
        if (lane == 0 && !(piv > F(0) && piv < F(INFINITY))) atomicOr(err, 1);
        const F rp = F(1) / piv;
        const bool below = lane > j;
        if (below) pr[jj] *= rp;
#pragma unroll
        for (int q = jj + 1; q < 16; ++q) {
          const F u = bcast(pr[q], j);
          if (below) pr[q] -= pr[jj] * u;
        }
      }
      if (lane >= c0) {
#pragma unroll
        for (int q = 0; q < 16; ++q) a[lane][c0 + q] = pr[q];
      }
    }
    __syncthreads();
    if (p == 3) break;
    const int nc = 48 - c0;  // columns right of the panel
    if (wave == 1 && lane < nc) {  // U12 = inv(L11) A12, one column per work-item
      const int q = c0 + 16 + lane;
      F x[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        F s = a[c0 + r][q];
#pragma unroll
        for (int m = 0; m < r; ++m) s -= a[c0 + r][c0 + m] * x[m];
        x[r] = s;
      }
#pragma unroll
      for (int r = 1; r < 16; ++r) a[c0 + r][q] = x[r];
    }
    __syncthreads();
    const int nb = 3 - p;  // trailing blocks per side
    for (int jb = wave; jb < nb * nb; jb += 4) {  // A22 -= L21 U12
      const int r0 = c0 + 16 + 16 * (jb / nb), cc = c0 + 16 + 16 * (jb % nb);
      typename Mma<F>::acc_t acc;
      acc16_load<F>(a, r0, cc, acc);
      mma16<F, true>(a, r0, c0, a, c0, cc, acc);
      acc16_store<F>(acc, a, r0, cc, F(1));
    }
    __syncthreads();
  }

  // diagonal 16x16 blocks of inv(L) (wave 0) and inv(U) (wave 1): lane = 16 b + c
  if (wave < 2) {
    const int b = lane >> 4, c = lane & 15, o = 16 * b;
    F x[16];
    if (wave == 0) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        F s = (r == c) ? F(1) : F(0);
#pragma unroll
        for (int m = 0; m < r; ++m) s -= a[o + r][o + m] * x[m];
        x[r] = (r >= c) ? s : F(0);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) X[o + r][o + c] = x[r];
    } else {
#pragma unroll
      for (int r = 15; r >= 0; --r) {
        F s = (r == c) ? F(1) : F(0);
#pragma unroll
        for (int m = r + 1; m < 16; ++m) s -= a[o + r][o + m] * x[m];
        x[r] = (r <= c) ? s / a[o + r][o + r] : F(0);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) Y[o + r][o + c] = x[r];
    }
  }
  __syncthreads();
  // off-diagonal blocks, block diagonal dd: 4 - dd blocks of each inverse
  for (int dd = 1; dd < 4; ++dd) {
    for (int job = wave; job < 2 * (4 - dd); job += 4) {
      const bool lower = job < 4 - dd;
      const int t = lower ? job : job - (4 - dd);
      typename Mma<F>::acc_t acc = {0, 0, 0, 0};
      if (lower) {  // X_ij, i = t + dd, j = t: T = sum_{m=j}^{i-1} L_im X_mj, X_ij = -X_ii T
        const int i = t + dd, j = t;
        for (int m = j; m < i; ++m) mma16<F, false>(a, 16 * i, 16 * m, X, 16 * m, 16 * j, acc);
        acc16_store<F>(acc, T[wave], 0, 0, F(1));
        acc = typename Mma<F>::acc_t{0, 0, 0, 0};
        mma16<F, false>(X, 16 * i, 16 * i, T[wave], 0, 0, acc);
        acc16_store<F>(acc, X, 16 * i, 16 * j, F(-1));
      } else {  // Y_ij, i = t, j = t + dd: T = sum_{m=i+1}^{j} U_im Y_mj, Y_ij = -Y_ii T
        const int i = t, j = t + dd;
        for (int m = i + 1; m <= j; ++m) mma16<F, false>(a, 16 * i, 16 * m, Y, 16 * m, 16 * j, acc);
        acc16_store<F>(acc, T[wave], 0, 0, F(1));
        acc = typename Mma<F>::acc_t{0, 0, 0, 0};
        mma16<F, false>(Y, 16 * i, 16 * i, T[wave], 0, 0, acc);
        acc16_store<F>(acc, Y, 16 * i, 16 * j, F(-1));
      }
    }
    __syncthreads();
  }
  lds_to_tile<F>(Y, tkk);
  lds_to_tile<F>(X, linv);
}

// ---------------------------------------------------------------------------
// trailing update past block column k0 .. k0+depth-1:
// A_ij -= sum_{s<depth} L_{i,k0+s} U_{k0+s,j} for all i, j >= k0+depth.
// A work-group covers 2x2 tiles; each wave owns one whole 64x64 tile (4x4
// MFMA blocks), the wave pairs that share a tile row or column fetch the
// same L or U operands through L1.
// ---------------------------------------------------------------------------
// Operands of one k-group of the whole-tile product, read as 16-byte chunks
// (W values).  Inside every 16x16 MFMA block the order of k and of the
// output columns is permuted so that one chunk feeds W MFMAs: in group g
// (4W consecutive k) a lane (lr = lane % 16, lk = lane / 16) takes in step
// s = 0 .. W-1 the k index 4W g + W lk + s, and output block cb holds the
// columns 16W (cb / W) + W lr + cb % W.  So the lane's A chunk (row
// 16 rb + lr, W consecutive k) serves its W steps and its B chunk (one k,
// W consecutive columns) serves W output blocks: 8 loads per 16W MFMAs.
// The sum over k is the same; only the order in which the MFMAs add the
// k values changes.
template <typename F>
struct FragC {
  using C = typename Chunk<F>::type;
  static constexpr int W = Chunk<F>::W;
  C a[4];          // block row rb
  C b[W][4 / W];   // step s, column chunk c
};

// chunk offsets of a lane inside a tile: A (row 16 rb + lr, k chunk 4g + lk),
// B (k row 4W g + W lk + s, column chunk 16 c + lr)
template <typename F>
__device__ __forceinline__ void fragc_load(FragC<F>& f, const GLOBAL typename Chunk<F>::type* __restrict__ Lt,
                                          const GLOBAL typename Chunk<F>::type* __restrict__ Ut, int g, int acb,
                                          int bcb) {
  constexpr int W = Chunk<F>::W;
  const GLOBAL typename Chunk<F>::type* la = Lt + acb + 256 * g;
  const GLOBAL typename Chunk<F>::type* ub = Ut + bcb + 4 * W * g;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) f.a[rb] = la[16 * rb];
#pragma unroll
  for (int s = 0; s < W; ++s)
#pragma unroll
    for (int c = 0; c < 4 / W; ++c) f.b[s][c] = ub[1024 * c + s];
}

template <typename F>
__device__ __forceinline__ void fragc_mma(const FragC<F>& f, typename Mma<F>::acc_t (&acc)[4][4]) {
  constexpr int W = Chunk<F>::W;
#pragma unroll
  for (int s = 0; s < W; ++s)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = Mma<F>::op(f.a[rb][s], f.b[s][cb / W][cb % W], acc[rb][cb]);
}

// whole-tile accumulator of a wave (the trailing update's layout: block
// (rb, cb) holds rows 16 rb + MFMA row and columns 16W (cb / W) + W lr + cb % W)
template <typename F>
__device__ __forceinline__ void acc4_load(const GLOBAL F* __restrict__ T, typename Mma<F>::acc_t (&acc)[4][4]) {
  using C = typename Chunk<F>::type;
  constexpr int W = Chunk<F>::W;
  const int lane = threadIdx.x & 63, lr = lane & 15;
  const GLOBAL C* Tc = (const GLOBAL C*)T;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int c = 0; c < 4 / W; ++c) {
        const C x = Tc[(16 * c + lr) * 64 + 16 * rb + Mma<F>::row(lane, v)];
#pragma unroll
        for (int w = 0; w < W; ++w) acc[rb][W * c + w][v] = x[w];
      }
}

template <typename F>
__device__ __forceinline__ void acc4_to_lds(typename Mma<F>::acc_t (&acc)[4][4], F (*Cs)[LDP], F scale) {
  constexpr int W = Chunk<F>::W;
  const int lane = threadIdx.x & 63, lr = lane & 15;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) Cs[16 * rb + Mma<F>::row(lane, v)][16 * W * (cb / W) + W * lr + cb % W] = scale * acc[rb][cb][v];
}

// acc += sum_{s<depth} L0(s) * U0(s) for a whole tile, L0(s) = L0 + s tiles,
// U0(s) = U0 + s*ustride tiles (16-byte chunk pointers); the loads of the
// next k-group are issued before the products of the current one (the last
// pass reloads group ng-1, which is in bounds and unused)
template <typename F>
__device__ __forceinline__ void acc4_add_products(typename Mma<F>::acc_t (&acc)[4][4],
                                                  const GLOBAL typename Chunk<F>::type* __restrict__ L0,
                                                  const GLOBAL typename Chunk<F>::type* __restrict__ U0, size_t ustride,
                                                  int depth) {
  constexpr int W = Chunk<F>::W, TC = TILE_ELEMS / W, GPT = 16 / W;  // k-groups per tile
  if (depth <= 0) return;
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
  const int acb = lk * 64 + lr, bcb = lr * 64 + W * lk;
  const int ng = GPT * depth;  // even: GPT is 4 or 8
  FragC<F> f0, f1;
  fragc_load<F>(f0, L0, U0, 0, acb, bcb);
  for (int g = 0; g < ng; g += 2) {
    {
      const int h = g + 1, s = h / GPT;
      fragc_load<F>(f1, L0 + size_t(s) * TC, U0 + size_t(s) * ustride * TC, h % GPT, acb, bcb);
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the products
    fragc_mma<F>(f0, acc);
    __builtin_amdgcn_sched_barrier(0);
    {
      const int h = min(g + 2, ng - 1), s = h / GPT;
      fragc_load<F>(f0, L0 + size_t(s) * TC, U0 + size_t(s) * ustride * TC, h % GPT, acb, bcb);
    }
    __builtin_amdgcn_sched_barrier(0);
    fragc_mma<F>(f1, acc);
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <typename F>
__global__ __launch_bounds__(256, 2) void k_lu_trail(const FacDesc* __restrict__ d, int k0, int depth) {
  using C = typename Chunk<F>::type;
  constexpr int W = Chunk<F>::W;
  constexpr int TC = TILE_ELEMS / W;  // chunks per tile
  // XCD-aware order: each XCD takes a contiguous range of (subdomain,
  // super-tile) work items, so the panels one subdomain's super-tiles share
  // stay in one XCD's L2 instead of being fetched by all eight
  const int gx = int(gridDim.x);
  const int lin = xcd_block(int(blockIdx.y) * gx + int(blockIdx.x), gx * int(gridDim.y));
  const int bx = lin % gx;
  const FacDesc D = d[lin / gx];
  const int nr = D.N - k0 - depth;
  if (nr <= 0) return;
  const int ns = (nr + 1) >> 1;  // 2x2 super-tiles per side
  if (bx >= ns * ns) return;
  // wave-uniform: keeps the tile base addresses in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int ti = 2 * (bx / ns) + (wave >> 1), tj = 2 * (bx % ns) + (wave & 1);
  if (ti >= nr || tj >= nr) return;  // no barriers below: a wave may leave alone
  const size_t N = D.N;
  const size_t i = k0 + depth + ti, j = k0 + depth + tj;
  GLOBAL C* fac = gptr((C*)D.fac);
  GLOBAL C* Ct = fac + (i * N + j) * TC;
  const int lr = lane & 15;
  typename Mma<F>::acc_t acc[4][4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = typename Mma<F>::acc_t{0, 0, 0, 0};
  // L_{i,k0+s} = L0 + s tiles, U_{k0+s,j} = U0 + s*N tiles
  acc4_add_products<F>(acc, fac + (i * N + k0) * TC, fac + (size_t(k0) * N + j) * TC, N, depth);
  // C -= acc: output (16 rb + row(lane, v), 16W c + W lr + w) is element w
  // of chunk (16 c + lr) * 64 + row of the tile
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int c = 0; c < 4 / W; ++c) {
        GLOBAL C* e = Ct + (16 * c + lr) * 64 + 16 * rb + Mma<F>::row(lane, v);
        C x = *e;
#pragma unroll
        for (int w = 0; w < W; ++w) x[w] -= acc[rb][W * c + w][v];
        *e = x;
      }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// operand halves of a quadrant k-group (see Frag): 16-byte A chunks, B pairs
template <typename F>
struct FragA {
  typename Chunk<F>::type a[4 / Chunk<F>::W][2];
};
template <typename F>
struct FragB {
  typename Pair<F>::type b[4 / Chunk<F>::W][Chunk<F>::W];
};

template <typename F>
__device__ __forceinline__ void fraga_load(FragA<F>& f, const GLOBAL F* __restrict__ At, int g) {
  using C = typename Chunk<F>::type;
  constexpr int W = Chunk<F>::W, NS = 4 / W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int R0 = (wave >> 1) * 32, lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    const GLOBAL C* la = (const GLOBAL C*)At + (16 / W * g + 4 * u + lk) * 64 + R0 + lr;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) f.a[u][rb] = la[16 * rb];
  }
}

template <typename F>
__device__ __forceinline__ void fragb_load(FragB<F>& f, const GLOBAL F* __restrict__ Bt, int g) {
  using P = typename Pair<F>::type;
  constexpr int W = Chunk<F>::W, NS = 4 / W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int C0 = (wave & 1) * 32, lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    const GLOBAL F* ub = Bt + tile_off<F>(16 * g + 4 * W * u + W * lk, C0 + 2 * lr);
#pragma unroll
    for (int s = 0; s < W; ++s) f.b[u][s] = *(const GLOBAL P*)(ub + W * s);
  }
}

// acc += As * B (As in LDS, B a tile in global memory) or acc += A * Bs (A
// in global memory, Bs in LDS): one tile product per quadrant, the global
// operand's next k-group loaded before the current one's products
template <typename F, bool LDS_A>
__device__ __forceinline__ void acc_add_product_half_lds(typename Mma<F>::acc_t (&acc)[2][2], F (*S)[LDP],
                                                         const GLOBAL F* __restrict__ G) {
  constexpr int W = Chunk<F>::W, NS = 4 / W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int R0 = (wave >> 1) * 32, C0 = (wave & 1) * 32, lr = lane & 15, lk = lane >> 4;
  FragA<F> a0, a1;
  FragB<F> b0, b1;
  if (LDS_A)
    fragb_load<F>(b0, G, 0);
  else
    fraga_load<F>(a0, G, 0);
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    FragA<F>& ac = (g & 1) ? a1 : a0;
    FragA<F>& an = (g & 1) ? a0 : a1;
    FragB<F>& bc = (g & 1) ? b1 : b0;
    FragB<F>& bn = (g & 1) ? b0 : b1;
    if (g + 1 < 4) {
      if (LDS_A)
        fragb_load<F>(bn, G, g + 1);
      else
        fraga_load<F>(an, G, g + 1);
    }
#pragma unroll
    for (int u = 0; u < NS; ++u)
#pragma unroll
      for (int s = 0; s < W; ++s) {
        const int k = 16 * g + 4 * W * u + W * lk + s;
        F av[2], bv[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          av[q] = LDS_A ? S[R0 + 16 * q + lr][k] : ac.a[u][q][s];
          bv[q] = LDS_A ? bc.b[u][s][q] : S[k][C0 + 2 * lr + q];
        }
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = Mma<F>::op(av[rb], bv[cb], acc[rb][cb]);
      }
  }
}

// panel of tile column k: blockIdx.x < nr -> L_{k+1+x, k}, else U_{k, k+1+x'};
// pending in-block updates fused in front of the product with the inverse.
// FP64: only the updated tile goes through LDS and the inverse (the same
// tile for the whole panel, so mostly an L2 hit) is read from global
// memory, which leaves room for four work-groups per CU; FP32: both tiles
// in LDS (four work-groups per CU already fit).
template <typename F>
__global__ __launch_bounds__(256) void k_lu_panel(const FacDesc* __restrict__ d, int k0, int k) {
  constexpr bool ONE_TILE = sizeof(F) == 8;
  // XCD-aware order: the panel tiles of one subdomain (which share the
  // diagonal tile's inverse and the pending-update operands) run on one XCD
  const int gx = int(gridDim.x);
  const int lin = xcd_block(int(blockIdx.y) * gx + int(blockIdx.x), gx * int(gridDim.y));
  const int bx = lin % gx;
  const FacDesc D = d[lin / gx];
  const int nr = D.N - k - 1;
  if (nr <= 0 || bx >= 2 * nr) return;
  __shared__ F Ts[64][LDP];
  __shared__ F Is[ONE_TILE ? 1 : 64][LDP];  // the inverse (FP32)
  const size_t N = D.N;
  GLOBAL F* fac = gptr((F*)D.fac);
  typename Mma<F>::acc_t acc[2][2];
  const bool lower = bx < nr;
  size_t target;
  if (lower) {  // L_ik = (A_ik - sum_s L_is U_sk) inv(U_kk)
    const size_t i = k + 1 + bx;
    target = i * N + k;
    acc_updated_tile<F>(acc, fac, target, i * N + k0, 1, size_t(k0) * N + k, N, k - k0);
  } else {  // U_kj = inv(L_kk) (A_kj - sum_s L_ks U_sj)
    const size_t j = k + 1 + (bx - nr);
    target = size_t(k) * N + j;
    acc_updated_tile<F>(acc, fac, target, size_t(k) * N + k0, 1, size_t(k0) * N + j, N, k - k0);
  }
  acc_to_lds<F>(acc, Ts);
  const GLOBAL F* inv = fac + (lower ? size_t(k) * N + k : N * N + k) * TILE_ELEMS;  // inv(U_kk) / inv(L_kk)
  if (!ONE_TILE) tile_to_lds<F>(inv, Is);
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = typename Mma<F>::acc_t{0, 0, 0, 0};
  if (ONE_TILE) {
    if (lower)
      acc_add_product_half_lds<F, true>(acc, Ts, inv);  // A_ik inv(U_kk)
    else
      acc_add_product_half_lds<F, false>(acc, Ts, inv);  // inv(L_kk) A_kj
  } else {
    if (lower)
      tile_mma<F>(Ts, Is, acc);
    else
      tile_mma<F>(Is, Ts, acc);
  }
  acc_store<F>(acc, fac + target * TILE_ELEMS);
}

// ---------------------------------------------------------------------------
// Coupling tiles of the 128 x 128 block inverses of tile pairs (a, b) =
// (2p, 2p+1), used by the two-block triangular-solve work items:
//   X_L = -inv(L_bb) L_ba inv(L_aa)   (tile N*N + N + p)
//   X_U = -inv(U_aa) U_ab inv(U_bb)   (tile N*N + N + N/2 + p)
// so that inv([L_aa 0; L_ba L_bb]) = [inv(L_aa) 0; X_L inv(L_bb)] and
// inv([U_aa U_ab; 0 U_bb]) = [inv(U_aa) X_U; 0 inv(U_bb)].
// blockIdx.x < npmax: X_L of pair x, else X_U of pair x - npmax.
// ---------------------------------------------------------------------------
template <typename F>
__global__ __launch_bounds__(256) void k_lu_pairs(const FacDesc* __restrict__ d, int npmax) {
  const FacDesc D = d[blockIdx.y];
  const int N = D.N, np = N / 2;
  const bool lower = int(blockIdx.x) < npmax;
  const int p = lower ? int(blockIdx.x) : int(blockIdx.x) - npmax;
  if (p >= np) return;
  const size_t a = 2 * size_t(p), b = a + 1, n = size_t(N), NN = n * n;
  __shared__ F As[64][LDP], Bs[64][LDP];
  GLOBAL F* fac = gptr((F*)D.fac);
  // X = -(T1 T2) T3
  const size_t t1 = lower ? NN + b : a * n + a;
  const size_t t2 = lower ? b * n + a : a * n + b;
  const size_t t3 = lower ? NN + a : b * n + b;
  const size_t out = lower ? NN + n + p : NN + n + np + p;
  typename Mma<F>::acc_t acc[2][2];
  tile_to_lds<F>(fac + t1 * TILE_ELEMS, As);
  tile_to_lds<F>(fac + t2 * TILE_ELEMS, Bs);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[u][v] = typename Mma<F>::acc_t{0, 0, 0, 0};
  tile_mma<F>(As, Bs, acc);
  __syncthreads();
  acc_to_lds<F>(acc, As);
  tile_to_lds<F>(fac + t3 * TILE_ELEMS, Bs);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[u][v] = typename Mma<F>::acc_t{0, 0, 0, 0};
  tile_mma<F>(As, Bs, acc);
  acc_negate<F>(acc);
  acc_store<F>(acc, fac + out * TILE_ELEMS);
}

// LDS reserved, unused, by an FP32 launch of the trailing update and of the
// inverse panels so that one work-group runs per CU: their waves share
// operands through the CU's L1, and further resident work-groups evict
// them (fine-level FP32 LU 11.4 ms with three per CU, 10.0 with two, 9.8
// with one; in FP64 two per CU stay the faster).  `static_lds`: what the
// kernel declares itself.
template <typename F>
constexpr size_t one_per_cu_lds(size_t static_lds) {
  return sizeof(F) == 4 ? size_t(96 * 1024) - static_lds : 0;
}

template <typename F>
hipError_t launch_lu(const FacDesc* d, int nd, int maxN, int* err, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  for (int k0 = 0; k0 < maxN; k0 += LU_DEPTH) {
    const int depth = maxN - k0 < LU_DEPTH ? maxN - k0 : LU_DEPTH;
    for (int k = k0; k < k0 + depth; ++k) {
      hipLaunchKernelGGL((k_lu_diag<F>), dim3(nd), dim3(256), 0, s, d, k0, k, err);
      const int nr = maxN - k - 1;
      if (nr > 0) hipLaunchKernelGGL((k_lu_panel<F>), dim3(2 * nr, nd), dim3(256), 0, s, d, k0, k);
    }
    const int nt = maxN - k0 - depth, ns = (nt + 1) / 2;
    if (nt > 0)
      hipLaunchKernelGGL((k_lu_trail<F>), dim3(ns * ns, nd), dim3(256), one_per_cu_lds<F>(0), s, d, k0, depth);
  }
  const int npmax = maxN / 2;
  if (npmax > 0) hipLaunchKernelGGL((k_lu_pairs<F>), dim3(2 * npmax, nd), dim3(256), 0, s, d, npmax);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Inverse panels.  With the owned rows last (local rows nv .. n-1), the
// owned columns of J^{-1} are X = U^{-1} L^{-1} E_o, E_o = [0; I]: column c
// of E_o is the unit vector of local row nv + c.  In 64 x 64 tiles (X has
// the factor's tile rows i and tile columns j over the owned columns):
//   forward   Y_ij = inv(L_ii) (E_ij - sum_{m0(j) <= m < i} L_im Y_mj),
//             where Y_mj = 0 for m < m0(j) = floor((nv + 64 j) / 64) (the
//             unit vectors of column tile j start in tile row m0(j));
//   backward  X_ij = inv(U_ii) (Y_ij - sum_{m > i} U_im X_mj),  i = N-1 .. 0.
// X overwrites Y in place; tile (i, j) of X sits at tile j N + i.  Padding
// rows (unit diagonal in the factor, no unit vector) and padding columns
// stay zero.
//
// The tile rows are taken in blocks of four, one launch per block (the
// forward from tile row nv / 64 down, the backward from N - 1 up).  A
// work-group owns one tile column j of one subdomain, and wave t the whole
// tile of the block's row t (the layout of the trailing update):
//   phase 1: the products with the rows already final (outside the block),
//            every wave reading the same X (or Y) tiles, through L1;
//   phase 2: the block row by row, nearest the final rows first: the row's
//            wave puts its tile in LDS, the work-group multiplies it by the
//            diagonal inverse and stores it, and the waves of the later rows
//            add its products (their tiles hold minus the right-hand side).
// ---------------------------------------------------------------------------
constexpr int XINV_ROWS = 4;

// acc += A * Bs for a whole tile: A in global memory (16-byte chunks), Bs in LDS
template <typename F>
__device__ __forceinline__ void acc4_add_product_lds(typename Mma<F>::acc_t (&acc)[4][4], const GLOBAL F* __restrict__ A,
                                                     F (*Bs)[LDP]) {
  using C = typename Chunk<F>::type;
  constexpr int W = Chunk<F>::W, GPT = 16 / W;
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
  const GLOBAL C* Ac = (const GLOBAL C*)A + lk * 64 + lr;
  C a0[4], a1[4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) a0[rb] = Ac[16 * rb];
#pragma unroll
  for (int g = 0; g < GPT; ++g) {
    C(&cur)[4] = (g & 1) ? a1 : a0;
    C(&nxt)[4] = (g & 1) ? a0 : a1;
    if (g + 1 < GPT) {
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) nxt[rb] = Ac[256 * (g + 1) + 16 * rb];
    }
#pragma unroll
    for (int s = 0; s < W; ++s) {
      const int k = 4 * W * g + W * lk + s;
      F b[4];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) b[cb] = Bs[k][16 * W * (cb / W) + W * lr + cb % W];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = Mma<F>::op(cur[rb][s], b[cb], acc[rb][cb]);
    }
  }
}

template <typename F>
__global__ __launch_bounds__(256, 2) void k_xinv(const FacDesc* __restrict__ d, int blk, int fwd) {
  using C = typename Chunk<F>::type;
  constexpr int W = Chunk<F>::W, TC = TILE_ELEMS / W;
  // XCD-aware order: the tile columns of one subdomain (which share its
  // factor's tile rows) run on one XCD
  const int gx = int(gridDim.x);
  const int lin = xcd_block(int(blockIdx.y) * gx + int(blockIdx.x), gx * int(gridDim.y));
  const FacDesc D = d[lin / gx];
  const int j = lin % gx;
  if (!D.X || j >= D.No) return;
  const int N = D.N;
  // rows of the block this work-group forms: r(t) = r0 + dir t, t < nr
  int r0, dir, nr, m0 = 0;
  if (fwd) {
    const int i0 = D.nv / 64 + XINV_ROWS * blk;
    m0 = (D.nv + 64 * j) / 64;
    r0 = max(i0, m0);  // Y_rj = 0 above tile row m0(j)
    nr = min(i0 + XINV_ROWS, N) - r0;
    dir = 1;
  } else {
    const int i0 = N - 1 - XINV_ROWS * blk;
    r0 = i0;
    nr = min(XINV_ROWS, i0 + 1);
    // Without overlap rows (the coarsest level: X is the whole inverse,
    // symmetric, and its tile rows are its tile columns) only the lower
    // triangle is kept, and X_ij, i >= j, reads only X_mj, m > i: the
    // upper tiles are not formed.
    if (D.nv == 0) nr = min(nr, i0 - j + 1);
    dir = -1;
  }
  if (nr <= 0) return;
  __shared__ F As[64][LDP], Bs[64][LDP];
  const size_t n = size_t(N), NN = n * n, col = size_t(j) * n;
  const GLOBAL F* fac = gptr((const F*)D.fac);
  GLOBAL F* X = gptr((F*)D.X);
  // wave-uniform: keeps the tile base addresses in scalar registers
  const int t = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int lr = lane & 15;
  const bool mine = t < nr;  // this wave holds row r(t) of the block
  const int r = r0 + dir * t;
  typename Mma<F>::acc_t acc[4][4];
  // phase 1: acc = -(right-hand side of row r) + products with the final rows
  int m1 = 0, depth = 0;
  if (fwd) {
    // -E: E(r, c) = 1 where 64 i + r = nv + 64 j + c, for owned columns 64 j + c < n - nv
    const int off = D.nv + 64 * j - 64 * r, nown = D.n - D.nv;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rr = 16 * rb + Mma<F>::row(lane, v), c = 16 * W * (cb / W) + W * lr + cb % W;
          acc[rb][cb][v] = (rr == c + off && 64 * j + c < nown) ? F(-1) : F(0);
        }
    m1 = m0, depth = r0 - m0;  // final rows m0(j) .. r0 - 1 (none when the block starts at m0(j))
  } else {
    if (mine) {
      acc4_load<F>(X + (col + r) * TILE_ELEMS, acc);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = -acc[rb][cb];
    }
    m1 = r0 + 1, depth = N - 1 - r0;  // final rows r0 + 1 .. N - 1
  }
  // L_{r, m1 + s} / U_{r, m1 + s} times Y_{m1 + s, j} / X_{m1 + s, j}
  if (mine) acc4_add_products<F>(acc, (const GLOBAL C*)fac + (size_t(r) * n + m1) * TC, (const GLOBAL C*)X + (col + m1) * TC, 1, depth);
  // phase 2: the block row by row
  for (int q = 0; q < nr; ++q) {
    const int rq = r0 + dir * q;
    if (q > 0) __syncthreads();  // the previous row's products have read Bs
    if (t == q) acc4_to_lds<F>(acc, Bs, F(-1));  // rhs - products
    tile_to_lds<F>(fac + (fwd ? NN + rq : size_t(rq) * n + rq) * TILE_ELEMS, As);  // inv(L_qq) / inv(U_qq)
    __syncthreads();
    typename Mma<F>::acc_t x[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) x[u][v] = typename Mma<F>::acc_t{0, 0, 0, 0};
    tile_mma<F>(As, Bs, x);
    acc_store<F>(x, X + (col + rq) * TILE_ELEMS);
    if (q + 1 < nr) {
      __syncthreads();  // tile_mma has read Bs
      acc_to_lds<F>(x, Bs);
      __syncthreads();
      // later rows hold -(rhs - products): add L_{r, rq} x / U_{r, rq} x
      if (mine && t > q) acc4_add_product_lds<F>(acc, fac + (size_t(r) * n + rq) * TILE_ELEMS, Bs);
    }
  }
}

template <typename F>
hipError_t launch_xinv(const FacDesc* d, int nd, int maxNo, int fsteps, int bsteps, hipStream_t s) {
  if (nd <= 0 || maxNo <= 0) return hipSuccess;
  constexpr int R = XINV_ROWS;
  const size_t lds = one_per_cu_lds<F>(2 * 64 * LDP * sizeof(F));  // beside its two LDS tiles
  for (int k = 0; k < (fsteps + R - 1) / R; ++k) hipLaunchKernelGGL((k_xinv<F>), dim3(maxNo, nd), dim3(256), lds, s, d, k, 1);
  for (int k = 0; k < (bsteps + R - 1) / R; ++k) hipLaunchKernelGGL((k_xinv<F>), dim3(maxNo, nd), dim3(256), lds, s, d, k, 0);
  return hipGetLastError();
}

// Packed symmetric form of the panels (what the smoother reads): the overlap
// rows X_v in tile rows of 64 local rows (zero past nv), then the lower
// triangle of X_oo = J^{-1}[o, o] in tile rows of 64 owned rows, by columns
// (X_oo is symmetric: its upper triangle is the transpose of the lower one,
// so the smoother reads 0.68 of the full panels on the benchmark's
// subdomains).  One work-group per packed tile; every element comes from
// the full panels' tile row (local row) / 64.
template <typename F>
__global__ __launch_bounds__(256) void k_xpack(const FacDesc* __restrict__ d) {
  const FacDesc D = d[blockIdx.y];
  if (!D.X) return;
  const int No = D.No, Nv = (D.nv + 63) / 64, nown = D.n - D.nv;
  int t = int(blockIdx.x), a, b, row0, rows;  // destination tile (a, b): local rows row0 .. row0 + rows - 1
  if (t < Nv * No) {
    b = t / Nv, a = t % Nv;
    row0 = 64 * a, rows = min(64, D.nv - 64 * a);
  } else {
    t -= Nv * No;
    if (t >= No * (No + 1) / 2) return;
    b = 0;
    while (t >= No - b) t -= No - b, ++b;  // column b holds tiles a = b .. No-1
    a = b + t;
    row0 = D.nv + 64 * a, rows = min(64, nown - 64 * a);
  }
  const GLOBAL F* X = gptr((const F*)D.X);
  GLOBAL F* out = gptr((F*)D.Xs) + size_t(blockIdx.x) * TILE_ELEMS;
  const size_t N = size_t(D.N);
  for (int e = threadIdx.x; e < TILE_ELEMS; e += 256) {
    const int r = e % 64, c = e / 64;
    F v = F(0);
    if (r < rows) {
      const int lr = row0 + r;
      v = X[(size_t(b) * N + lr / 64) * TILE_ELEMS + tile_off<F>(lr % 64, c)];
    }
    out[tile_off<F>(r, c)] = v;
  }
}

template <typename F>
hipError_t launch_xpack(const FacDesc* d, int nd, int maxPacked, hipStream_t s) {
  if (nd <= 0 || maxPacked <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_xpack<F>), dim3(maxPacked, nd), dim3(256), 0, s, d);
  return hipGetLastError();
}

template hipError_t launch_extract<double>(const FacDesc*, int, int, hipStream_t);
template hipError_t launch_extract<float>(const FacDesc*, int, int, hipStream_t);
template hipError_t launch_lu<double>(const FacDesc*, int, int, int*, hipStream_t);
template hipError_t launch_lu<float>(const FacDesc*, int, int, int*, hipStream_t);
template hipError_t launch_xinv<double>(const FacDesc*, int, int, int, int, hipStream_t);
template hipError_t launch_xinv<float>(const FacDesc*, int, int, int, int, hipStream_t);
template hipError_t launch_xpack<double>(const FacDesc*, int, int, hipStream_t);
template hipError_t launch_xpack<float>(const FacDesc*, int, int, hipStream_t);

}  // namespace nnms
