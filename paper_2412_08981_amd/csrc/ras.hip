// One application of the restricted additive Schwarz smoother
//   z (+)= sum_p (R^0_p)^T  J_p^{-1}  R^delta_p r        (Section 2.2)
// with J_p = L_p U_p factored into dense 64x64 tiles.
//
// Work unit = one 64-row block of one triangular sweep of one subdomain:
//   forward  y_i = inv(L_ii) (r[S_p]_i - sum_{j<i} L_ij y_j)
//   backward x_i = inv(U_ii) (y_i     - sum_{j>i} U_ij x_j)
// The gather r[S_p] is fused into the forward blocks and the restricted
// scatter (owned rows only) into the backward blocks.  A block waits only
// for the blocks it reads, through per-block flags (no grid-wide barrier),
// so blocks of all subdomains of all batched systems stream their tiles
// concurrently.  Work items are handed out in dependency order from an
// atomic ticket: a work-group only ever waits on tickets drawn before its
// own, by work-groups that are already running, so the schedule cannot
// deadlock; every wait is additionally bounded.
//
// Block results and flags travel through device-coherent (agent-scope)
// relaxed atomic loads and stores; a block's results are complete (the
// wave's stores acknowledged) before its flag is stored.  This avoids a
// full L2 write-back / invalidate per block, which is what an agent-scope
// release / acquire pair costs on this GPU.
#include "devcommon.h"
#include "kernels.h"

namespace nnms {

constexpr int SPIN_LIMIT = 1 << 22;

template <typename F>
__device__ __forceinline__ F ld_coh(const F* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename F>
__device__ __forceinline__ void st_coh(F* p, F v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// all memory operations of this wave issued so far are complete
__device__ __forceinline__ void wave_drain() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <typename F, typename V>
__global__ __launch_bounds__(256) void k_ras(RasLaunch P, int32_t* err) {
  using C = typename Chunk<F>::type;
  constexpr int W = Chunk<F>::W;
  constexpr int NQ = 16 / W;  // 16-byte chunks per lane per tile
  __shared__ F red[4][64];
  __shared__ __align__(16) F vsh[64];
  __shared__ int s_task;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int epoch = atomic_load_acq(P.counter + 1) + 1;

  auto spin = [&](const int32_t* fl) {
    int spins = 0;
    while (atomic_load_rlx(fl) != epoch) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > SPIN_LIMIT) {
        if (lane == 0) atomicOr(err, 2);
        break;
      }
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  };

  for (;;) {
    if (tid == 0) s_task = atomicAdd(P.counter, 1);
    __syncthreads();
    const int t = s_task;
    __syncthreads();
    if (t >= P.ntasks) {
      if (tid == 0 && t == P.ntasks + int(gridDim.x) - 1) {
        __hip_atomic_store(P.counter, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        atomic_store_rel(P.counter + 1, epoch);
      }
      return;
    }
    const int code = P.tasks[t];
    const int sub = code >> 16, dir = (code >> 15) & 1, i = code & 0x7fff;
    const SubDesc S = P.subs[sub];
    if (!slot_active(S.st, WHEN_RUNNING)) continue;
    const int N = S.N;
    const F* __restrict__ fac = (const F*)S.fac;
    F* yx = (F*)S.yx;
    const size_t NN = size_t(N) * N;
    const int32_t* fwd_flags = P.flags + S.flag0;
    const int32_t* bwd_flags = fwd_flags + N;

    auto load_tile = [&](size_t tix, C (&reg)[NQ]) {
      const C* base = (const C*)(fac + tix * TILE_ELEMS);
#pragma unroll
      for (int q = 0; q < NQ; ++q) reg[q] = __builtin_nontemporal_load(base + (wave + 4 * q) * 64 + lane);
    };
    // acc += tile . y (y distributed one value per lane)
    auto gemv = [&](const C (&A)[NQ], F yl, F& acc) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        C yv;
        F* e = (F*)&yv;
        const int c0 = (wave + 4 * q) * W;
#pragma unroll
        for (int k = 0; k < W; ++k) e[k] = __shfl(yl, c0 + k, 64);
        acc += chunk_dot(A[q], yv);
      }
    };

    F acc = 0, bval = 0;
    C A[NQ], B[NQ];
    if (dir == 0) {
      if (wave == 0) {
        const int g = S.gidx[i * 64 + lane];
        const int gg = g >= 0 ? g : -g - 2;
        bval = (g != -1) ? F(((const V*)S.rin)[gg]) : F(0);
      }
      load_tile(i > 0 ? size_t(i) * N : NN + i, A);
      int ready = -1;  // forward blocks known to be complete: 0..ready
      for (int j = 0; j < i; ++j) {
        if (j > ready) {
          if (atomic_load_rlx(fwd_flags + i - 1) == epoch) {
            ready = i - 1;
          } else {
            spin(fwd_flags + j);
            ready = j;
          }
          __atomic_signal_fence(__ATOMIC_SEQ_CST);
        }
        const F yl = ld_coh(yx + j * 64 + lane);
        load_tile(j + 1 < i ? size_t(i) * N + j + 1 : NN + i, B);
        gemv(A, yl, acc);
#pragma unroll
        for (int q = 0; q < NQ; ++q) A[q] = B[q];
      }
    } else {
      spin(fwd_flags + N - 1);  // every forward block of this subdomain is complete
      if (wave == 0) bval = ld_coh(yx + i * 64 + lane);
      load_tile(size_t(i) * N + (i < N - 1 ? N - 1 : i), A);
      int ready = N;  // backward blocks known to be complete: ready..N-1
      for (int j = N - 1; j > i; --j) {
        if (j < ready) {
          if (atomic_load_rlx(bwd_flags + i + 1) == epoch) {
            ready = i + 1;
          } else {
            spin(bwd_flags + j);
            ready = j;
          }
          __atomic_signal_fence(__ATOMIC_SEQ_CST);
        }
        const F yl = ld_coh(yx + j * 64 + lane);
        load_tile(size_t(i) * N + (j - 1 > i ? j - 1 : i), B);
        gemv(A, yl, acc);
#pragma unroll
        for (int q = 0; q < NQ; ++q) A[q] = B[q];
      }
    }
    red[wave][lane] = acc;
    __syncthreads();
    if (wave == 0) vsh[lane] = bval - ((red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]));
    __syncthreads();
    {
      const C* vc = (const C*)vsh;
      F acc2 = 0;
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc2 += chunk_dot(A[q], vc[wave + 4 * q]);
      red[wave][lane] = acc2;
    }
    __syncthreads();
    if (wave == 0) {
      const F out = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
      st_coh(yx + i * 64 + lane, out);
      if (dir == 1) {
        const int g = S.gidx[i * 64 + lane];
        if (g >= 0) {
          V* z = (V*)S.zout;
          z[g] = P.add ? V(z[g] + V(out)) : V(out);
        }
      }
      wave_drain();
      if (lane == 0) __hip_atomic_store(P.flags + S.flag0 + dir * N + i, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <typename F, typename V>
hipError_t launch_ras(const RasLaunch& p, int grid, hipStream_t s) {
  if (p.ntasks <= 0) return hipSuccess;
  if (grid > p.ntasks) grid = p.ntasks;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((k_ras<F, V>), dim3(grid), dim3(256), 0, s, p, p.counter + 2);
  return hipGetLastError();
}

template hipError_t launch_ras<double, double>(const RasLaunch&, int, hipStream_t);
template hipError_t launch_ras<float, float>(const RasLaunch&, int, hipStream_t);
template hipError_t launch_ras<double, float>(const RasLaunch&, int, hipStream_t);

}  // namespace nnms
