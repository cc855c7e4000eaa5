// One application of the restricted additive Schwarz smoother
//   z (+)= sum_p (R^0_p)^T  J_p^{-1}  R^delta_p r        (Section 2.2)
// with J_p = L_p U_p factored into dense 64x64 tiles.
//
// Work unit = a group of K consecutive 64-row blocks of one triangular sweep
// of one subdomain.  For the forward sweep and a group with rows i:
//   y_i = inv(L_ii) (r[S_p]_i - sum_{j<i} L_ij y_j)
// the blocks j of earlier groups come from other work-groups; the blocks
// inside the group are substituted in order inside the work-group.  The
// backward sweep x_i = inv(U_ii) (y_i - sum_{j>i} U_ij x_j) mirrors it.  The
// gather r[S_p] is fused into the forward groups and the restricted scatter
// (owned rows only) into the backward groups.  A group waits only for the
// blocks it reads (no grid-wide barrier), so groups of all subdomains of all
// batched systems stream their tiles concurrently; K trades hand-offs
// between work-groups (latency) against parallelism.
//
// Work items are handed out in dependency order from an atomic ticket: a
// work-group only ever waits on tickets drawn before its own, by
// work-groups that are already running, so the schedule cannot deadlock;
// every wait is additionally bounded.
//
// Hand-off: every block result is published as tagged 64-bit words through
// device-coherent (agent-scope) relaxed atomic stores; each word carries the
// launch's tag (forward or backward) next to 32 bits of the value, so a
// consumer polls the data itself: one memory round trip per hand-off, with
// no separate flag, no store drain and no L2 write-back or invalidate (which
// is what an agent-scope release / acquire pair costs on this GPU).  The
// yx workspace holds 16 bytes per value: one word (FP32) or the low and high
// halves of the FP64 bit pattern in two words.
#include "devcommon.h"
#include "kernels.h"

namespace nnms {

constexpr int SPIN_LIMIT = 1 << 22;

// Epochs.  A launch tags its results with its epoch e (2e forward, 2e + 1
// backward).  The epoch lives in word 1 of the launch's counter array and is
// read by every work-group when it starts; it is set before the launch, by
// the seeding kernel when the counter array is created or by the last
// work-group of the previous launch on the same counter array (launches on
// one counter array are stream-ordered), from the device-wide counter below.
// So every launch has one epoch for all its work-groups, whatever runs on
// other streams meanwhile, and no two launches share one (until the 31-bit
// counter wraps): results left in a workspace by any earlier launch never
// carry a current tag.
__device__ int32_t g_ras_epoch = 0;

__device__ __forceinline__ int32_t fresh_epoch() {
  int32_t e = (atomicAdd(&g_ras_epoch, 1) + 1) & 0x7fffffff;
  return e ? e : 1;  // tag 0 never matches: zeroed words and torn FP64 halves read as 0
}

__global__ void k_ras_seed(int32_t* counter) {
  if (threadIdx.x == 0) {
    __hip_atomic_store(counter, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(counter + 1, fresh_epoch(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(counter + 2, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(counter + 3, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

hipError_t launch_ras_seed(int32_t* counter, hipStream_t s) {
  hipLaunchKernelGGL(k_ras_seed, dim3(1), dim3(64), 0, s, counter);
  return hipGetLastError();
}

// the last work-group of a launch: ticket back to 0, the next launch's epoch
__device__ __forceinline__ void finish_launch(int32_t* counter) {
  __hip_atomic_store(counter, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(counter + 1, fresh_epoch(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


__device__ __forceinline__ uint64_t ld64(const uint64_t* p) {
  return __hip_atomic_load(gptr(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(gptr(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename F>
struct Tagged;
template <>
struct Tagged<float> {
  static __device__ __forceinline__ void put(uint64_t* p, float v, uint32_t tag) {
    st64(p, (uint64_t(tag) << 32) | uint64_t(__float_as_uint(v)));
  }
  // returns the word's tag; v receives the value
  static __device__ __forceinline__ uint32_t get(const uint64_t* p, float& v) {
    const uint64_t w = ld64(p);
    v = __uint_as_float(uint32_t(w));
    return uint32_t(w >> 32);
  }
};
template <>
struct Tagged<double> {
  static __device__ __forceinline__ void put(uint64_t* p, double v, uint32_t tag) {
    const uint64_t b = uint64_t(__double_as_longlong(v));
    st64(p, (uint64_t(tag) << 32) | (b & 0xffffffffull));
    st64(p + 1, (uint64_t(tag) << 32) | (b >> 32));
  }
  // returns the tag if both halves carry the same one, else 0
  static __device__ __forceinline__ uint32_t get(const uint64_t* p, double& v) {
    const uint64_t lo = ld64(p), hi = ld64(p + 1);
    v = __longlong_as_double((long long)((hi << 32) | (lo & 0xffffffffull)));
    const uint32_t t0 = uint32_t(lo >> 32), t1 = uint32_t(hi >> 32);
    return t0 == t1 ? t0 : 0u;
  }
};

// waves per SIMD the register allocation must allow: FP64 takes the whole
// register file (the four prefetched tiles alone are 128 VGPRs; one work-group
// per CU is also the launch shape that streams fastest), FP32 two
template <typename F, int K>
struct RasWaves {
  static constexpr int value = sizeof(F) == 8 ? 1 : 2;
};

template <typename F, typename V, int K>
__global__ __launch_bounds__(256, (RasWaves<F, K>::value)) void k_ras(RasLaunch P, int32_t* err) {
  using C = typename Chunk<F>::type;
  constexpr int W = Chunk<F>::W;
  constexpr int NQ = 16 / W;  // 16-byte chunks per lane per tile
  __shared__ F red[4][64];
  __shared__ __align__(16) F vsh[64];
  __shared__ __align__(16) F ysh[K][64];
  __shared__ F bsh[K][64];
  __shared__ __align__(16) F ywv[4][2][64];  // per-wave staging of fetched result blocks
  __shared__ int s_task;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int epoch = __hip_atomic_load(P.counter + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t tag_fwd = 2u * uint32_t(epoch), tag_bwd = tag_fwd + 1u;

  // this lane's value of block j, waiting until the whole wave sees `tag`
  // (or `tag2`, when nonzero) on its words
  auto fetch = [&](const uint64_t* yx, int j, uint32_t tag, uint32_t tag2) -> F {
    const uint64_t* p = yx + (size_t(j) * 64 + lane) * 2;
    F v;
    int spins = 0;
    for (;;) {
      const uint32_t t = Tagged<F>::get(p, v);
      if (__all(t == tag || (tag2 != 0u && t == tag2))) break;
      __builtin_amdgcn_s_sleep(1);
      if (++spins > SPIN_LIMIT) {
        if (lane == 0) atomicOr(err, 2);
        break;
      }
    }
    return v;
  };

  for (;;) {
    if (tid == 0) s_task = atomicAdd(P.counter, 1);
    __syncthreads();
    const int t = s_task;
    __syncthreads();
    if (t >= P.ntasks) {
      if (tid == 0 && t == P.ntasks + int(gridDim.x) - 1) {
        finish_launch(P.counter);
      }
      return;
    }
    const int code = gptr(P.tasks)[t];
    const int sub = code >> 16, dir = (code >> 15) & 1, I = code & 0x7fff;
    const SubDesc S = P.subs[sub];
    if (!slot_active(S.st, WHEN_RUNNING)) continue;
    const int N = S.N;
    const int i0 = I * K;
    const int nr = min(K, N - i0);  // blocks in this group
    const F* __restrict__ fac = (const F*)S.fac;
    uint64_t* yx = (uint64_t*)S.yx;
    const size_t NN = size_t(N) * N;

    auto load_tile = [&](size_t tix, C (&reg)[NQ]) {
      const GLOBAL C* base = gptr((const C*)(fac + tix * TILE_ELEMS));
#pragma unroll
      for (int q = 0; q < NQ; ++q) reg[q] = __builtin_nontemporal_load(base + (wave + 4 * q) * 64 + lane);
    };
    // acc += tile . y, y in LDS
    auto gemv_lds = [&](const C (&A)[NQ], const F* y, F& acc) {
      const C* yc = (const C*)y;
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc += chunk_dot(A[q], yc[wave + 4 * q]);
    };
    // reduce acc over the 4 waves into out[64] (minus it from minuend)
    auto reduce_into = [&](F acc, F* out, const F* minuend) {
      red[wave][lane] = acc;
      __syncthreads();
      if (wave == 0) {
        const F s = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
        out[lane] = minuend ? minuend[lane] - s : s;
      }
      __syncthreads();
    };

    F acc[K];
#pragma unroll
    for (int r = 0; r < K; ++r) acc[r] = 0;
    const bool fwd = dir == 0;
    const int i1 = i0 + nr - 1;
    const uint32_t tag_in = fwd ? tag_fwd : tag_bwd;  // tag of the blocks this group reads

    // right-hand sides of the group's rows: gathered r[S_p] (forward) or y (backward)
    if (fwd) {
      if (wave < nr) {
        const int g = gptr(S.gidx)[(i0 + wave) * 64 + lane];
        const int gg = g >= 0 ? g : -g - 2;
        bsh[wave][lane] = (g != -1) ? F(gptr((const V*)S.rin)[gg]) : F(0);
      }
    } else {
      // the last forward block is published (forward or already backward
      // tag): every forward group of this subdomain is complete
      (void)fetch(yx, N - 1, tag_fwd, tag_bwd);
      if (wave < nr) bsh[wave][lane] = fetch(yx, i0 + wave, tag_fwd, 0u);
    }
    // scatter indices of the group's rows (backward), loaded now: the
    // scatter follows the publication of each block result
    int gz[K];
#pragma unroll
    for (int r = 0; r < K; ++r) gz[r] = (!fwd && r < nr) ? gptr(S.gidx)[(i0 + r) * 64 + lane] : -1;

    // Off-diagonal stream: M tiles (blocks of other groups, in the order the
    // chain produces them), rows of the group innermost; then the first
    // in-group tile.  Two tiles and their two result blocks per round trip.
    const int M = (fwd ? i0 : (N - 1 - i1)) * nr;
    const size_t first_in = fwd ? NN + i0 : size_t(i1) * N + i1;  // inv(L_i0) / inv(U_i1)
    auto col_of = [&](int k) -> int {
      const int jj = k / nr;
      return fwd ? jj : N - 1 - jj;
    };
    auto tile_of = [&](int k) -> size_t {
      if (k >= M) return first_in;
      const int r = k % nr;
      return size_t(i0 + r) * N + col_of(k);
    };
    auto add_row = [&](int r, F d) {
#pragma unroll
      for (int kk = 0; kk < K; ++kk) acc[kk] += (kk == r) ? d : F(0);
    };
    // ring of four register tiles: the loads of tiles k+2 .. k+5 are in
    // flight while tiles k, k+1 are applied (128 KB per work-group in FP64)
    C R0[NQ], R1[NQ], R2[NQ], R3[NQ];
    load_tile(tile_of(0), R0);
    if (M >= 1) load_tile(tile_of(1), R1);
    if (M >= 2) load_tile(tile_of(2), R2);
    if (M >= 3) load_tile(tile_of(3), R3);
    // applies tiles k (Ra) and k+1 (Rb, when k+1 < M) and refills them with
    // tiles k+4, k+5 (tile M is the first in-group tile, also kept)
    auto pair = [&](int k, C (&Ra)[NQ], C (&Rb)[NQ]) {
      const bool two = k + 1 < M;
      const int j0 = col_of(k), j1 = two ? col_of(k + 1) : j0;
      // fetch both result blocks in one polling loop
      const uint64_t* p0 = yx + (size_t(j0) * 64 + lane) * 2;
      const uint64_t* p1 = yx + (size_t(j1) * 64 + lane) * 2;
      F y0, y1;
      {
        int spins = 0;
        for (;;) {
          const uint32_t t0 = Tagged<F>::get(p0, y0);
          const uint32_t t1 = Tagged<F>::get(p1, y1);
          if (__all(t0 == tag_in && t1 == tag_in)) break;
          __builtin_amdgcn_s_sleep(1);
          if (++spins > SPIN_LIMIT) {
            if (lane == 0) atomicOr(err, 2);
            break;
          }
        }
      }
      // stage both blocks in this wave's LDS slice; chunks are read back as broadcasts
      ywv[wave][0][lane] = y0;
      ywv[wave][1][lane] = y1;
      __builtin_amdgcn_wave_barrier();
      F d0 = 0;
      gemv_lds(Ra, ywv[wave][0], d0);
      add_row(k % nr, d0);
      // keep the refill of a tile's registers after their last use, so the
      // compiler does not double-buffer them (register pressure = occupancy)
      __builtin_amdgcn_sched_barrier(0);
      if (k + 4 <= M) load_tile(tile_of(k + 4), Ra);
      if (two) {
        F d1 = 0;
        gemv_lds(Rb, ywv[wave][1], d1);
        add_row((k + 1) % nr, d1);
        __builtin_amdgcn_sched_barrier(0);
        if (k + 5 <= M) load_tile(tile_of(k + 5), Rb);
      }
      __builtin_amdgcn_wave_barrier();
    };
    for (int k = 0; k < M; k += 4) {
      pair(k, R0, R1);
      if (k + 2 < M) pair(k + 2, R2, R3);
    }
    // the first in-group tile is in register tile M mod 4; from here on R0
    // is the current tile (A) and R1 the prefetched one (B)
    switch (M & 3) {
      case 1:
#pragma unroll
        for (int q = 0; q < NQ; ++q) R0[q] = R1[q];
        break;
      case 2:
#pragma unroll
        for (int q = 0; q < NQ; ++q) R0[q] = R2[q];
        break;
      case 3:
#pragma unroll
        for (int q = 0; q < NQ; ++q) R0[q] = R3[q];
        break;
      default:
        break;
    }
    C(&A)[NQ] = R0;
    C(&B)[NQ] = R1;
    __syncthreads();  // bsh visible

    if (fwd) {
      // in-group substitution, rows i0 .. i1; A holds inv(L_i0)
#pragma unroll
      for (int r = 0; r < K; ++r) {
        if (r < nr) {
#pragma unroll
          for (int q = 0; q < r; ++q) {  // A = L(i0+r, i0+q)
            if (q + 1 < r)
              load_tile(size_t(i0 + r) * N + i0 + q + 1, B);
            else
              load_tile(NN + i0 + r, B);
            F d = 0;
            gemv_lds(A, ysh[q], d);
            acc[r] += d;
#pragma unroll
            for (int c = 0; c < NQ; ++c) A[c] = B[c];
          }
          // A = inv(L_{i0+r}); v = b - acc
          reduce_into(acc[r], vsh, bsh[r]);
          if (r + 1 < nr) load_tile(size_t(i0 + r + 1) * N + i0, B);  // next row's first in-group tile
          F a2 = 0;
          gemv_lds(A, vsh, a2);
          reduce_into(a2, ysh[r], nullptr);
          if (wave == 0) Tagged<F>::put(yx + (size_t(i0 + r) * 64 + lane) * 2, ysh[r][lane], tag_fwd);
          if (r + 1 < nr) {
#pragma unroll
            for (int c = 0; c < NQ; ++c) A[c] = B[c];
          }
        }
      }
    } else {
      // in-group back substitution, rows i1 down to i0; A holds inv(U_i1)
#pragma unroll
      for (int rr = 0; rr < K; ++rr) {
        const int r = nr - 1 - rr;
        if (r >= 0) {
          F ar = 0;
#pragma unroll
          for (int kk = 0; kk < K; ++kk)
            if (kk == r) ar = acc[kk];
          // A = U(i0+r, i0+q) for q = nr-1 .. r+1, then inv(U_{i0+r})
          for (int q = nr - 1; q > r; --q) {
            if (q - 1 > r)
              load_tile(size_t(i0 + r) * N + i0 + q - 1, B);
            else
              load_tile(size_t(i0 + r) * N + i0 + r, B);
            F d = 0;
            gemv_lds(A, ysh[q], d);
            ar += d;
#pragma unroll
            for (int c = 0; c < NQ; ++c) A[c] = B[c];
          }
          reduce_into(ar, vsh, bsh[r]);
          if (r - 1 >= 0) load_tile(size_t(i0 + r - 1) * N + i1, B);  // next row's first in-group tile
          F a2 = 0;
          gemv_lds(A, vsh, a2);
          reduce_into(a2, ysh[r], nullptr);
          if (wave == 0) {
            const F out = ysh[r][lane];
            // publish first: later blocks of the chain wait for it
            Tagged<F>::put(yx + (size_t(i0 + r) * 64 + lane) * 2, out, tag_bwd);
            int g = -1;
#pragma unroll
            for (int kk = 0; kk < K; ++kk)
              if (kk == r) g = gz[kk];
            if (g >= 0) {
              GLOBAL V* z = gptr((V*)S.zout);
              z[g] = P.add ? V(z[g] + V(out)) : V(out);
            }
          }
          if (r - 1 >= 0) {
#pragma unroll
            for (int c = 0; c < NQ; ++c) A[c] = B[c];
          }
        }
      }
    }
  }
}


// Work items of two blocks (K = 2) with the pair's 128 x 128 triangular
// inverse precomputed: for rows a = 2p, b = 2p + 1
//   forward   y_a = inv(L_aa) v_a,   y_b = X_L v_a + inv(L_bb) v_b,
//             X_L = -inv(L_bb) L_ba inv(L_aa)
//   backward  x_a = inv(U_aa) s_a + X_U s_b,   x_b = inv(U_bb) s_b,
//             X_U = -inv(U_aa) U_ab inv(U_bb)
// (v, s: right-hand side minus the off-pair products), so both blocks come
// out of one step with three resident tiles instead of one block after the
// other: the chain of hand-offs between work-groups halves, and so does the
// number of work items.  A last single block (odd N) uses its inverse alone.
template <typename F, typename V>
__global__ __launch_bounds__(256, (RasWaves<F, 2>::value)) void k_ras2(RasLaunch P, int32_t* err) {
  using C = typename Chunk<F>::type;
  constexpr int W = Chunk<F>::W;
  constexpr int NQ = 16 / W;  // 16-byte chunks per lane per tile
  __shared__ F red[4][2][64];
  __shared__ __align__(16) F vsh[2][64];
  __shared__ F ysh[2][64];
  __shared__ F bsh[2][64];
  __shared__ __align__(16) F ywv[4][2][64];  // per-wave staging of fetched result blocks
  __shared__ int s_task;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int epoch = __hip_atomic_load(P.counter + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t tag_fwd = 2u * uint32_t(epoch), tag_bwd = tag_fwd + 1u;

  auto fetch = [&](const uint64_t* yx, int j, uint32_t tag, uint32_t tag2) -> F {
    const uint64_t* p = yx + (size_t(j) * 64 + lane) * 2;
    F v;
    int spins = 0;
    for (;;) {
      const uint32_t t = Tagged<F>::get(p, v);
      if (__all(t == tag || (tag2 != 0u && t == tag2))) break;
      __builtin_amdgcn_s_sleep(1);
      if (++spins > SPIN_LIMIT) {
        if (lane == 0) atomicOr(err, 2);
        break;
      }
    }
    return v;
  };

  for (;;) {
    if (tid == 0) s_task = atomicAdd(P.counter, 1);
    __syncthreads();
    const int t = s_task;
    __syncthreads();
    if (t >= P.ntasks) {
      if (tid == 0 && t == P.ntasks + int(gridDim.x) - 1) {
        finish_launch(P.counter);
      }
      return;
    }
    const int code = gptr(P.tasks)[t];
    const int sub = code >> 16, dir = (code >> 15) & 1, I = code & 0x7fff;
    const SubDesc S = P.subs[sub];
    if (!slot_active(S.st, WHEN_RUNNING)) continue;
    const int N = S.N, NP = N / 2;
    const int a = 2 * I;
    const int nr = min(2, N - a);  // 2: a pair, 1: the last single block
    const int b = a + nr - 1;
    const F* __restrict__ fac = (const F*)S.fac;
    uint64_t* yx = (uint64_t*)S.yx;
    const size_t NN = size_t(N) * N;
    const bool fwd = dir == 0;
    const uint32_t tag_in = fwd ? tag_fwd : tag_bwd;

    auto load_tile = [&](size_t tix, C (&reg)[NQ]) {
      const GLOBAL C* base = gptr((const C*)(fac + tix * TILE_ELEMS));
#pragma unroll
      for (int q = 0; q < NQ; ++q) reg[q] = __builtin_nontemporal_load(base + (wave + 4 * q) * 64 + lane);
    };
    // acc += tile . y, y in LDS
    auto gemv_lds = [&](const C (&A)[NQ], const F* y, F& acc) {
      const C* yc = (const C*)y;
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc += chunk_dot(A[q], yc[wave + 4 * q]);
    };
    // reduces the two rows' partial sums over the four waves: out[r] =
    // minuend[r] - sum (or the sum); wave r writes row r
    auto reduce2 = [&](F acc0, F acc1, F (*out)[64], F (*minuend)[64]) {
      red[wave][0][lane] = acc0;
      red[wave][1][lane] = acc1;
      __syncthreads();
      if (wave < nr) {
        const F s = (red[0][wave][lane] + red[1][wave][lane]) + (red[2][wave][lane] + red[3][wave][lane]);
        out[wave][lane] = minuend ? minuend[wave][lane] - s : s;
      }
      __syncthreads();
    };

    F acc0 = 0, acc1 = 0;
    // right-hand sides of the rows: gathered r[S_p] (forward) or y (backward)
    if (fwd) {
      if (wave < nr) {
        const int g = gptr(S.gidx)[(a + wave) * 64 + lane];
        const int gg = g >= 0 ? g : -g - 2;
        bsh[wave][lane] = (g != -1) ? F(gptr((const V*)S.rin)[gg]) : F(0);
      }
    } else {
      // the last forward block is published (forward or already backward
      // tag): every forward work item of this subdomain is complete
      (void)fetch(yx, N - 1, tag_fwd, tag_bwd);
      if (wave < nr) bsh[wave][lane] = fetch(yx, a + wave, tag_fwd, 0u);
    }
    // scatter index of this wave's row (backward), loaded now: the scatter
    // follows the publication of the block result
    const int gz = (!fwd && wave < nr) ? gptr(S.gidx)[(a + wave) * 64 + lane] : -1;

    // the pair's inverse tiles, loaded first and kept in registers for the
    // whole item (they are needed right after the last wait, on the chain's
    // critical path): forward inv(L_aa), X_L, inv(L_bb), backward inv(U_aa),
    // X_U, inv(U_bb); a single block has its inverse only
    C D0[NQ], D1[NQ], D2[NQ];
    load_tile(fwd ? NN + a : size_t(a) * N + a, D0);
    if (nr == 2) {
      load_tile(fwd ? NN + N + I : NN + N + NP + I, D1);
      load_tile(fwd ? NN + b : size_t(b) * N + b, D2);
    }
    // stream positions: the M off-pair tiles (blocks of other work items in
    // the order the chain produces them, the pair's rows innermost)
    const int M = (fwd ? a : N - 1 - b) * nr;
    auto col_of = [&](int k) -> int {
      const int jj = k / nr;
      return fwd ? jj : N - 1 - jj;
    };
    auto tile_of = [&](int k) -> size_t { return size_t(a + k % nr) * N + col_of(k); };
    // ring of four register tiles: the loads of positions k+2 .. k+5 are in
    // flight while k, k+1 are applied (128 KB per work-group in FP64)
    C R0[NQ], R1[NQ], R2[NQ], R3[NQ];
    if (M >= 1) load_tile(tile_of(0), R0);
    if (M >= 2) load_tile(tile_of(1), R1);
    if (M >= 3) load_tile(tile_of(2), R2);
    if (M >= 4) load_tile(tile_of(3), R3);
    // polls result blocks j0 and j1 until the whole wave sees the tag on
    // both, and stages them in this wave's LDS slice (chunks are read back
    // as broadcasts)
    auto poll2 = [&](int j0, int j1) {
      const uint64_t* p0 = yx + (size_t(j0) * 64 + lane) * 2;
      const uint64_t* p1 = yx + (size_t(j1) * 64 + lane) * 2;
      F y0, y1;
      int spins = 0;
      for (;;) {
        const uint32_t t0 = Tagged<F>::get(p0, y0);
        const uint32_t t1 = Tagged<F>::get(p1, y1);
        if (__all(t0 == tag_in && t1 == tag_in)) break;
        __builtin_amdgcn_s_sleep(1);
        if (++spins > SPIN_LIMIT) {
          if (lane == 0) atomicOr(err, 2);
          break;
        }
      }
      ywv[wave][0][lane] = y0;
      ywv[wave][1][lane] = y1;
      __builtin_amdgcn_wave_barrier();
    };
    const int ncols = M / nr;
    // applies positions k (Ra) and k+1 (Rb, when k+1 < M) and refills them
    // with positions k+4, k+5.  A pair's positions k, k+1 are its two rows
    // of one column jj = k/2; the blocks of columns jj and jj+1 are polled
    // together at even jj, so that the row's last two columns (published
    // together by the previous pair) cost one wait, not two.  A single
    // block's positions k, k+1 are two columns, polled together.
    auto pair = [&](int k, C (&Ra)[NQ], C (&Rb)[NQ]) {
      const bool two = k + 1 < M;
      const F* ya;
      const F* yb;
      if (nr == 2) {
        const int jj = k >> 1;
        if ((jj & 1) == 0) poll2(col_of(k), jj + 1 < ncols ? col_of(k + 2) : col_of(k));
        ya = yb = ywv[wave][jj & 1];
      } else {
        poll2(col_of(k), two ? col_of(k + 1) : col_of(k));
        ya = ywv[wave][0];
        yb = ywv[wave][1];
      }
      F d0 = 0;
      gemv_lds(Ra, ya, d0);
      if (nr == 1 || (k & 1) == 0)
        acc0 += d0;
      else
        acc1 += d0;
      // keep the refill of a tile's registers after their last use, so the
      // compiler does not double-buffer them (register pressure = occupancy)
      __builtin_amdgcn_sched_barrier(0);
      if (k + 4 < M) load_tile(tile_of(k + 4), Ra);
      if (two) {
        F d1 = 0;
        gemv_lds(Rb, yb, d1);
        if (nr == 1 || ((k + 1) & 1) == 0)
          acc0 += d1;
        else
          acc1 += d1;
        __builtin_amdgcn_sched_barrier(0);
        if (k + 5 < M) load_tile(tile_of(k + 5), Rb);
      }
      __builtin_amdgcn_wave_barrier();
    };
    for (int k = 0; k < M; k += 4) {
      pair(k, R0, R1);
      if (k + 2 < M) pair(k + 2, R2, R3);
    }
    __syncthreads();  // bsh visible
    reduce2(acc0, acc1, vsh, bsh);
    // the pair's block inverse applied to both rows
    auto pair_step = [&](const C (&T0)[NQ], const C (&T1)[NQ], const C (&T2)[NQ]) {
      F o0 = 0, o1 = 0;
      if (nr == 1) {
        gemv_lds(T0, vsh[0], o0);
      } else if (fwd) {
        gemv_lds(T0, vsh[0], o0);  // inv(L_aa) v_a
        gemv_lds(T1, vsh[0], o1);  // X_L v_a
        gemv_lds(T2, vsh[1], o1);  // + inv(L_bb) v_b
      } else {
        gemv_lds(T0, vsh[0], o0);  // inv(U_aa) s_a
        gemv_lds(T1, vsh[1], o0);  // + X_U s_b
        gemv_lds(T2, vsh[1], o1);  // inv(U_bb) s_b
      }
      reduce2(o0, o1, ysh, nullptr);
    };
    pair_step(D0, D1, D2);
    if (wave < nr) {
      const int i = a + wave;
      const F out = ysh[wave][lane];
      // publish first: later blocks of the chain wait for it
      Tagged<F>::put(yx + (size_t(i) * 64 + lane) * 2, out, fwd ? tag_fwd : tag_bwd);
      if (gz >= 0) {
        GLOBAL V* z = gptr((V*)S.zout);
        z[gz] = P.add ? V(z[gz] + V(out)) : V(out);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Inverse panels: z_o = X_p^T r[S_p], X_p = J_p^{-1} E_o, from the packed
// symmetric form (overlap rows X_v, then the lower triangle of the owned
// block X_oo by columns), every stored tile read once.  Two kinds of work
// item per owned tile column b of subdomain p:
//   overlap part: X_v(t, b), t < Nv;
//   owned part:   X_oo(a, b), a >= b.
// A tile is split by rows: wave w holds rows 16 w .. 16 w + 15, lane l row
// 16 w + l % 16 and the 16-byte column chunks l / 16, l / 16 + 4, ...  Each
// item accumulates z_b += T^T y per column over its tiles (y: the tile's
// rows of r[S_p]); the 64 row partials of every column are added through LDS
// at the end and stored as the column part Cv_b or Co_b.  The owned part also
// forms, for a > b and by symmetry X_oo(b, a) = X_oo(a, b)^T, the
// contribution of the owned rows of tile b to z_a: T y_b, whose rows are
// complete inside a wave (the four lanes of a row add their chunks by two
// exchanges), stored as P_{b,a}.  A second launch adds
//   z_a = Cv_a + Co_a + sum_{b < a} P_{b,a}
// in that fixed order, so a batch gives every system the bits it gets
// alone.  No work-group waits for another.  The rows of r[S_p] are gathered
// into LDS first (YL: overlap rows, zero past nv, then owned rows, zero past
// no), or read per tile when they do not fit.  Partials of subdomain p at
// S.part: Cv_b at 64 b, Co_b at 64 (No + b), P_{b,a} at 128 No + 64 pair(b, a),
// pair(b, a) = b (No - 1) - b (b - 1) / 2 + (a - b - 1).
// ---------------------------------------------------------------------------
__device__ __forceinline__ size_t xpair(int b, int a, int No) {
  return size_t(b) * (No - 1) - size_t(b) * (b - 1) / 2 + (a - b - 1);
}

template <typename F, typename V, bool YL>
__global__ __launch_bounds__(256, 2) void k_xapply(RasLaunch P) {
  using C = typename Chunk<F>::type;
  constexpr int W = Chunk<F>::W;
  constexpr int NQ = 16 / W;  // 16-byte chunks per lane per tile
  extern __shared__ __align__(16) unsigned char xsh[];
  F* ysh = (F*)xsh;  // the gathered rows the item reads, then the column reduction
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row = 16 * wave + (lane & 15), cgrp = lane >> 4;  // this lane's tile row and first chunk
  const int code = gptr(P.tasks)[blockIdx.x];
  const int sub = code >> 16, owned = (code >> 15) & 1, b = code & 0x7fff;
  const SubDesc S = P.subs[sub];
  if (!slot_active(S.st, WHEN_RUNNING)) return;
  const int nv = S.nv, no = S.no;
  const int Nv = (nv + 63) / 64, No = (no + 63) / 64;
  const int NT = owned ? No - b : Nv;
  // the item's tiles are contiguous: X_v column b, or X_oo column b from the diagonal down
  const size_t first = owned ? size_t(Nv) * No + size_t(b) * No - size_t(b) * (b - 1) / 2 : size_t(b) * Nv;
  const GLOBAL C* base = gptr((const C*)S.fac) + first * (TILE_ELEMS / W);
  const GLOBAL int32_t* gidx = gptr(S.gidx);
  const GLOBAL V* rin = gptr((const V*)S.rin);
  GLOBAL F* part = gptr((F*)S.part);
  // rows of a tile past nv (overlap part) or no (owned part) hold zeros: not read
  auto load_tile = [&](int k, C (&reg)[NQ]) {
    const GLOBAL C* t = base + size_t(k) * (TILE_ELEMS / W);
    const bool live = row < (owned ? no - 64 * (b + k) : nv - 64 * k);
#pragma unroll
    for (int q = 0; q < NQ; ++q) reg[q] = live ? __builtin_nontemporal_load(t + (cgrp + 4 * q) * 64 + row) : C{};
  };
  // row e of the item's tiles: overlap row e (< nv), or owned row 64 b + e (< no)
  auto gathered = [&](int e) -> F {
    int lr;
    if (owned)
      lr = 64 * b + e < no ? nv + 64 * b + e : -1;
    else
      lr = e < nv ? e : -1;
    if (lr < 0) return F(0);
    const int g = gidx[lr];
    return g == -1 ? F(0) : F(rin[g >= 0 ? g : -g - 2]);
  };
  C R0[NQ], R1[NQ], R2[NQ], R3[NQ];
  load_tile(0, R0);
  if (NT > 1) load_tile(1, R1);
  if (NT > 2) load_tile(2, R2);
  if (NT > 3) load_tile(3, R3);
  if (YL) {
    for (int e = tid; e < NT * 64; e += 256) ysh[e] = gathered(e);
    __syncthreads();
  }
  // y_b under this lane's chunks (the owned part's row products)
  C yb[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (!owned) {
      yb[q] = C{};
    } else if (YL) {
      yb[q] = ((const C*)ysh)[cgrp + 4 * q];
    } else {
#pragma unroll
      for (int w = 0; w < W; ++w) yb[q][w] = gathered((cgrp + 4 * q) * W + w);
    }
  }
  C acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = C{};
  GLOBAL F* pp = part + 128 * No + row;
  auto apply = [&](const C (&R)[NQ], int k) {
    const F y = YL ? ysh[k * 64 + row] : gathered(k * 64 + row);
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] += R[q] * y;
    if (owned && k > 0) {
      F racc = F(0);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const C p = R[q] * yb[q];
#pragma unroll
        for (int w = 0; w < W; ++w) racc += p[w];
      }
      racc += __shfl_xor(racc, 16, 64);
      racc += __shfl_xor(racc, 32, 64);
      if (cgrp == 0) pp[64 * xpair(b, b + k, No)] = racc;
    }
  };
  for (int k = 0; k < NT; k += 4) {
    apply(R0, k);
    // refill a ring slot only after its last use (no double buffering)
    __builtin_amdgcn_sched_barrier(0);
    if (k + 4 < NT) load_tile(k + 4, R0);
    if (k + 1 < NT) {
      apply(R1, k + 1);
      __builtin_amdgcn_sched_barrier(0);
      if (k + 5 < NT) load_tile(k + 5, R1);
    }
    if (k + 2 < NT) {
      apply(R2, k + 2);
      __builtin_amdgcn_sched_barrier(0);
      if (k + 6 < NT) load_tile(k + 6, R2);
    }
    if (k + 3 < NT) {
      apply(R3, k + 3);
      __builtin_amdgcn_sched_barrier(0);
      if (k + 7 < NT) load_tile(k + 7, R3);
    }
  }
  __syncthreads();  // every read of the gathered values is done
  F(*red)[65] = (F(*)[65])xsh;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int k = 0; k < W; ++k) red[(cgrp + 4 * q) * W + k][row] = acc[q][k];
  __syncthreads();
  if (tid < 64) {
    F sum = 0;
    for (int r = 0; r < 64; ++r) sum += red[tid][r];
    part[64 * (owned ? No + b : b) + tid] = sum;
  }
}

// z_a = Cv_a + Co_a + sum_{b < a} P_{b,a}, scattered to the owned rows
// (one wave per task, four tasks per work-group; the owned parts' codes
// only; Cv_a only where there are overlap rows).  The partials are loaded
// in batches of XRED_BATCH before they are added, in the order above.
constexpr int XRED_BATCH = 16;

template <typename F, typename V>
__global__ __launch_bounds__(256) void k_xreduce(RasLaunch P) {
  const int task = 4 * int(blockIdx.x) + int(threadIdx.x >> 6);
  if (task >= P.ntasks) return;
  const int code = gptr(P.tasks)[task];
  if (!((code >> 15) & 1)) return;
  const int sub = code >> 16, a = code & 0x7fff;
  const SubDesc S = P.subs[sub];
  if (!slot_active(S.st, WHEN_RUNNING)) return;
  const int lane = threadIdx.x & 63, No = (S.no + 63) / 64;
  const GLOBAL F* part = gptr((const F*)S.part);
  const GLOBAL F* pp = part + 128 * No + lane;
  F sum = S.nv > 0 ? part[64 * a + lane] : F(0);
  sum += part[64 * (No + a) + lane];
  for (int b0 = 0; b0 < a; b0 += XRED_BATCH) {
    F v[XRED_BATCH];
#pragma unroll
    for (int u = 0; u < XRED_BATCH; ++u) v[u] = b0 + u < a ? pp[64 * xpair(b0 + u, a, No)] : F(0);
#pragma unroll
    for (int u = 0; u < XRED_BATCH; ++u)
      if (b0 + u < a) sum += v[u];
  }
  const int oc = 64 * a + lane;  // owned row index; local row nv + oc
  if (oc < S.no) {
    const int g = gptr(S.gidx)[S.nv + oc];
    GLOBAL V* z = gptr((V*)S.zout);
    z[g] = P.add ? V(z[g] + V(sum)) : V(sum);
  }
}

// LDS of an inverse-panel work-group holding the gathered vector (else only
// the column reduction)
constexpr size_t XAPPLY_MAX_LDS = 65536;

template <typename F, typename V>
static hipError_t launch_xapply(const RasLaunch& p, hipStream_t s) {
  // gathered rows: at most N tiles per work item; column reduction: 64 x 65
  const size_t red = 64 * 65 * sizeof(F), ylds = size_t(p.max_tiles + 1) * 64 * sizeof(F);
  if (ylds <= XAPPLY_MAX_LDS)
    hipLaunchKernelGGL((k_xapply<F, V, true>), dim3(p.ntasks), dim3(256), ylds > red ? ylds : red, s, p);
  else
    hipLaunchKernelGGL((k_xapply<F, V, false>), dim3(p.ntasks), dim3(256), red, s, p);
  hipLaunchKernelGGL((k_xreduce<F, V>), dim3((p.ntasks + 3) / 4), dim3(256), 0, s, p);
  return hipGetLastError();
}

template <typename F, typename V>
hipError_t launch_ras(const RasLaunch& p, int grid, hipStream_t s) {
  if (p.ntasks <= 0) return hipSuccess;
  if (p.group == 0) return launch_xapply<F, V>(p, s);
  if (grid > p.ntasks) grid = p.ntasks;
  if (grid < 1) grid = 1;
  switch (p.group) {
    case 1: hipLaunchKernelGGL((k_ras<F, V, 1>), dim3(grid), dim3(256), 0, s, p, p.counter + 2); break;
    case 2: hipLaunchKernelGGL((k_ras2<F, V>), dim3(grid), dim3(256), 0, s, p, p.counter + 2); break;
    case 4: hipLaunchKernelGGL((k_ras<F, V, 4>), dim3(grid), dim3(256), 0, s, p, p.counter + 2); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_ras<double, double>(const RasLaunch&, int, hipStream_t);
template hipError_t launch_ras<float, float>(const RasLaunch&, int, hipStream_t);
template hipError_t launch_ras<double, float>(const RasLaunch&, int, hipStream_t);

}  // namespace nnms
