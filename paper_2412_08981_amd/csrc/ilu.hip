// ILU(k) subdomain solver of the RAS smoother (Section 4 of the paper runs
// the smoother with incomplete LU subdomain solves in place of exact ones).
//
// Every subdomain is one work-group, and every row is handled by a group of
// G lanes of one wave (G = 4..32, chosen from the longest row).  The
// factorisation is the i-k-j form of Gaussian elimination restricted to the
// ILU pattern: a row eliminates its lower entries in ascending column order
// with rows already finished; the rows of one forward level depend only on
// earlier levels, so a level is processed in parallel and levels are
// separated by a work-group barrier.  The apply gathers the subdomain's part
// of the residual into LDS, runs the unit-lower forward and the upper
// backward solve level by level in LDS (partial sums of a row added in a
// fixed order, so results are deterministic) and scatters the owned rows.
#include "devcommon.h"
#include "kernels.h"

namespace nnms {

// one 16-byte schedule entry through a global-address-space pointer
__device__ __forceinline__ int4 meta_at(const int32_t* m, int q) {
  const GLOBAL int32_t* p = gptr(m) + 4 * q;
  return make_int4(p[0], p[1], p[2], p[3]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_ilu_extract(const int32_t* __restrict__ asrc, const double* __restrict__ a,
                                                     T* __restrict__ val, int64_t n) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int32_t s = gptr(asrc)[e];
  gptr(val)[e] = s >= 0 ? T(gptr(a)[s]) : T(0);
}

// Row i of the factorisation by a group of G lanes of one wave: the row's
// values and columns are staged in the group's LDS slice (at most 4G
// entries); for every lower entry k in ascending order the multiplier
// l = a_ik / u_kk is formed and the lanes take row k's upper entries j in
// turn (at most 2G of them), find j in row i by binary search and update
// a_ij -= l u_kj (distinct j, distinct targets).  Every a_ij receives its
// updates in ascending k, the same operations in the same order as the
// textbook i-k-j loop.  The rows k are final, so their loads do not wait
// for the eliminations: the diagonal and end of every row k are fetched
// for all steps at once, and the upper entries of four steps at a time.
// A column is found in row i through the group's window map (position of
// every column of row i, indexed by column - first column) when the row
// spans fewer than WIN columns, else by binary search.
template <typename T, int G>
__global__ __launch_bounds__(256) void k_ilu_factor(const IluDesc* __restrict__ d, int* __restrict__ err) {
  constexpr int NE = 4 * G;  // entries per row that a group can stage
  constexpr int CH = 4;      // elimination steps whose row data is loaded together
  constexpr int WIN = 64 * G;  // columns a row may span to use the window map (32 KiB of maps)
  __shared__ T svals[256 / G][NE];
  __shared__ int32_t scols[256 / G][NE];
  __shared__ int32_t sdk[256 / G][NE], sbk[256 / G][NE];
  __shared__ int16_t smap[256 / G][WIN];
  const IluDesc D = d[blockIdx.x];
  const GLOBAL int32_t* rp = gptr(D.rp);
  const GLOBAL int32_t* col = gptr(D.col);
  const GLOBAL int32_t* dpos = gptr(D.dpos);
  GLOBAL T* val = gptr((T*)D.val);
  const int grp = int(threadIdx.x) / G, lane = int(threadIdx.x) % G, ngrp = int(blockDim.x) / G;
  T* rv = svals[grp];
  int32_t* rc = scols[grp];
  int32_t* kd = sdk[grp];
  int32_t* kb = sbk[grp];
  int16_t* wmap = smap[grp];
  for (int t = lane; t < WIN; t += G) wmap[t] = -1;
  for (int lv = 0; lv < D.nfl; ++lv) {
    const int r0 = gptr(D.flev)[lv], r1 = gptr(D.flev)[lv + 1];
    for (int q = r0 + grp; q < r1; q += ngrp) {  // uniform within a group
      const int4 m = meta_at(D.fmeta, q);
      const int a = m.y, len = m.w - m.y, di = m.z - m.y;
      for (int t = lane; t < len; t += G) rv[t] = val[a + t], rc[t] = col[a + t];
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const int c0 = rc[0];
      const bool windowed = rc[len - 1] - c0 < WIN;  // uniform within a group
      if (windowed)
        for (int t = lane; t < len; t += G) wmap[rc[t] - c0] = int16_t(t);
      for (int e = lane; e < di; e += G) {
        const int k = rc[e];
        kd[e] = dpos[k], kb[e] = rp[k + 1];
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      for (int e0 = 0; e0 < di; e0 += CH) {
        T ukk[CH], fv[CH][2];
        int fc[CH][2];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int e = e0 + c;
          ukk[c] = T(1), fc[c][0] = fc[c][1] = -1, fv[c][0] = fv[c][1] = T(0);
          if (e < di) {
            const int dk = kd[e], bk = kb[e];
            const int f0 = dk + 1 + lane, f1 = f0 + G;
            ukk[c] = val[dk];
            if (f0 < bk) fc[c][0] = col[f0], fv[c][0] = val[f0];
            if (f1 < bk) fc[c][1] = col[f1], fv[c][1] = val[f1];
          }
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int e = e0 + c;
          if (e >= di) break;  // uniform within a group
          const T l = rv[e] / ukk[c];
#pragma unroll
          for (int x = 0; x < 2; ++x) {
            const int j = fc[c][x];
            if (j < 0) continue;
            if (windowed) {
              // j > k = rc[e] >= c0; a hit lies after e
              const int w = j - c0;
              const int pos = w < WIN ? int(wmap[w]) : -1;
              if (pos > e) rv[pos] -= l * fv[c][x];
            } else {
              int lo = e + 1, hi = len;
              while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (rc[mid] < j)
                  lo = mid + 1;
                else
                  hi = mid;
              }
              if (lo < len && rc[lo] == j) rv[lo] -= l * fv[c][x];
            }
          }
          if (lane == 0) rv[e] = l;
          __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
          __builtin_amdgcn_wave_barrier();
        }
      }
      for (int t = lane; t < len; t += G) val[a + t] = rv[t];
      if (windowed)
        for (int t = lane; t < len; t += G) wmap[rc[t] - c0] = -1;
      if (lane == 0 && !(rv[di] > T(0))) *err = 1;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
  }
}

// G lanes per row: lane l of a row's group takes entries l, l + G, ... and
// the group adds its partial sums in a fixed order, so a level's rows issue
// all their loads at once instead of one dependent chain per row.  Groups of
// up to 16 lanes are a quad, half row or row of the wave's DPP lanes, and
// add with DPP moves inside the ALU (swap within pairs, then pairs of a
// quad, then mirrored quads of a half row, then mirrored half rows) instead
// of LDS-routed shuffles; 32-lane groups use the shuffles.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
constexpr int DPP_QUAD_1032 = 0xB1;     // quad_perm(1, 0, 3, 2)
constexpr int DPP_QUAD_2301 = 0x4E;     // quad_perm(2, 3, 0, 1)
constexpr int DPP_HALF_MIRROR = 0x141;  // lane i <-> 7 - i within 8 lanes
constexpr int DPP_ROW_MIRROR = 0x140;   // lane i <-> 15 - i within 16 lanes

template <typename T, int G>
__device__ __forceinline__ T group_sum(T v) {
  if constexpr (G <= 16) {
    v += dpp_move<DPP_QUAD_1032>(v);
    v += dpp_move<DPP_QUAD_2301>(v);
    if constexpr (G >= 8) v += dpp_move<DPP_HALF_MIRROR>(v);
    if constexpr (G >= 16) v += dpp_move<DPP_ROW_MIRROR>(v);
    return v;
  } else {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
    return v;
  }
}

// Work-group barrier that orders LDS only: the apply's global memory is
// read-only until the final scatter, so loads issued before the barrier
// (the next level's factor entries) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The (at most two per lane) entries of one row's lower (FWD) or upper part
// that a lane of the row's group takes: entries e0 = first + lane and
// e1 = e0 + G; the host picks G with 2G >= the longest such part.
template <typename T, int G, bool FWD>
struct IluRow {
  int i = -1, c0 = -1, c1 = -1;
  T v0 = 0, v1 = 0, diag = 1;
  // m: forward {row, first, diagonal, end}, the lower part is [y, z);
  // backward {row, diagonal + 1, end, diagonal}, the upper part [y, z)
  __device__ __forceinline__ void load(const IluDesc& D, const int4 m, int lane) {
    i = m.x;
    const int first = m.y, end = m.z;
    const int e0 = first + lane, e1 = e0 + G;
    const GLOBAL T* val = gptr((const T*)D.val);
    c0 = e0 < end ? gptr(D.col)[e0] : -1;
    v0 = e0 < end ? val[e0] : T(0);
    c1 = e1 < end ? gptr(D.col)[e1] : -1;
    v1 = e1 < end ? val[e1] : T(0);
    if (!FWD) diag = val[m.w];
  }
  // y_i -= sum (forward) or y_i = (y_i - sum) / u_ii (backward), the partial
  // sums of the group added by a fixed xor tree
  __device__ __forceinline__ void apply(T* y, int lane) const {
    T s = c0 >= 0 ? v0 * y[c0] : T(0);
    if (c1 >= 0) s += v1 * y[c1];
    s = group_sum<T, G>(s);
    if (lane == 0) y[i] = FWD ? y[i] - s : (y[i] - s) / diag;
  }
};

// One sweep over the levels of one triangular factor.  The group's first
// row of a level is prefetched in two stages: its schedule entry two levels
// ahead and its factor entries one level ahead, both issued before the
// barrier that ends the current level, so no load of the critical path
// waits for another one between two barriers.
template <typename T, int G, bool FWD>
__device__ __forceinline__ void ilu_sweep(const IluDesc& D, T* y, int grp, int lane, int ngrp) {
  const int nl = FWD ? D.nfl : D.nbl;
  const GLOBAL int32_t* lev = gptr(FWD ? D.flev : D.blev);
  const int32_t* meta = FWD ? D.fmeta : D.bmeta;
  IluRow<T, G, FWD> cur;
  int4 mnext = make_int4(-1, 0, 0, 0);
  if (nl > 0 && lev[0] + grp < lev[1]) cur.load(D, meta_at(meta, lev[0] + grp), lane);
  if (nl > 1 && lev[1] + grp < lev[2]) mnext = meta_at(meta, lev[1] + grp);
  for (int lv = 0; lv < nl; ++lv) {
    const int r0 = lev[lv], r1 = lev[lv + 1];
    if (r0 + grp < r1) cur.apply(y, lane);  // uniform within a group
    for (int q = r0 + grp + ngrp; q < r1; q += ngrp) {
      IluRow<T, G, FWD> more;
      more.load(D, meta_at(meta, q), lane);
      more.apply(y, lane);
    }
    if (lv + 1 < nl && lev[lv + 1] + grp < lev[lv + 2]) cur.load(D, mnext, lane);
    if (lv + 2 < nl && lev[lv + 2] + grp < lev[lv + 3]) mnext = meta_at(meta, lev[lv + 2] + grp);
    lds_barrier();
  }
}

template <typename T, int G>
__global__ __launch_bounds__(256) void k_ilu_apply(const IluDesc* __restrict__ d, int add) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* y = reinterpret_cast<T*>(lds_raw);
  const IluDesc D = d[blockIdx.x];
  if (!slot_active(D.st, WHEN_RUNNING)) return;
  const GLOBAL int32_t* gid = gptr(D.gid);
  const GLOBAL T* rin = gptr((const T*)D.rin);
  const int grp = int(threadIdx.x) / G, lane = int(threadIdx.x) % G, ngrp = int(blockDim.x) / G;
  for (int i = threadIdx.x; i < D.n; i += blockDim.x) {
    const int g = gid[i];
    y[i] = rin[g >= 0 ? g : -g - 2];
  }
  __syncthreads();
  ilu_sweep<T, G, true>(D, y, grp, lane, ngrp);
  ilu_sweep<T, G, false>(D, y, grp, lane, ngrp);
  GLOBAL T* z = gptr((T*)D.zout);
  for (int i = threadIdx.x; i < D.n; i += blockDim.x) {
    const int g = gid[i];
    if (g >= 0) z[g] = add ? z[g] + y[i] : y[i];
  }
}

template <typename T>
hipError_t launch_ilu_extract(const int32_t* asrc, const double* a, T* val, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_ilu_extract<T><<<dim3(unsigned((n + 255) / 256)), dim3(256), 0, s>>>(asrc, a, val, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ilu_factor(const IluDesc* d, int nd, int lanes, int* err, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  switch (lanes) {
    case 4: k_ilu_factor<T, 4><<<dim3(nd), dim3(256), 0, s>>>(d, err); break;
    case 8: k_ilu_factor<T, 8><<<dim3(nd), dim3(256), 0, s>>>(d, err); break;
    case 16: k_ilu_factor<T, 16><<<dim3(nd), dim3(256), 0, s>>>(d, err); break;
    case 32: k_ilu_factor<T, 32><<<dim3(nd), dim3(256), 0, s>>>(d, err); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ilu_apply(const IluDesc* d, int nd, int maxn, int lanes, int add, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  const size_t lds = size_t(maxn) * sizeof(T);
  if (lds > ILU_MAX_LDS) return hipErrorInvalidValue;
  switch (lanes) {
    case 4: k_ilu_apply<T, 4><<<dim3(nd), dim3(256), lds, s>>>(d, add); break;
    case 8: k_ilu_apply<T, 8><<<dim3(nd), dim3(256), lds, s>>>(d, add); break;
    case 16: k_ilu_apply<T, 16><<<dim3(nd), dim3(256), lds, s>>>(d, add); break;
    case 32: k_ilu_apply<T, 32><<<dim3(nd), dim3(256), lds, s>>>(d, add); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_ilu_extract<double>(const int32_t*, const double*, double*, int64_t, hipStream_t);
template hipError_t launch_ilu_extract<float>(const int32_t*, const double*, float*, int64_t, hipStream_t);
template hipError_t launch_ilu_factor<double>(const IluDesc*, int, int, int*, hipStream_t);
template hipError_t launch_ilu_factor<float>(const IluDesc*, int, int, int*, hipStream_t);
template hipError_t launch_ilu_apply<double>(const IluDesc*, int, int, int, int, hipStream_t);
template hipError_t launch_ilu_apply<float>(const IluDesc*, int, int, int, int, hipStream_t);

}  // namespace nnms
