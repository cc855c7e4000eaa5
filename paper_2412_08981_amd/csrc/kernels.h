// Host-callable launchers of the HIP kernels.  Every launcher enqueues on
// `stream` and returns the hipError_t of the launch.
#pragma once
#include <hip/hip_runtime.h>

#include "devtypes.h"

namespace nnms {

// sparse.hip
template <typename T>
hipError_t launch_spmv(const SpmvDesc* d, int nd, int nblocks, int group, hipStream_t s);
// sliced-ELL matrices: split = 0, four slices per block (nblocks =
// ceil(rows / 256) per descriptor); split = 1, one slice per block with its
// steps split over the four waves (nblocks = ceil(rows / 64))
template <typename T>
hipError_t launch_sell(const SpmvDesc* d, int nd, int nblocks, int split, hipStream_t s);
// column-sorted slices (d.col = keys, d.base = slice bases, d.rp = the CSR
// row pointers): one 64-row slice per block (nblocks = ceil(rows / 64) per
// descriptor), cap = the most entries of one slice over the descriptors
template <typename T>
hipError_t launch_csort(const SpmvDesc* d, int nd, int nblocks, int cap, hipStream_t s);
template <typename T>
hipError_t launch_gather_ell(const int32_t* src, const double* csr, T* ell, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_prolong(const ProlongDesc* d, int nd, int nblocks, hipStream_t s);
template <typename T>
hipError_t launch_fill(T* p, int64_t n, T v, hipStream_t s);
hipError_t launch_cast_d2f(const double* a, float* b, int64_t n, hipStream_t s);
hipError_t launch_cast_f2d(const float* a, double* b, int64_t n, hipStream_t s);
hipError_t launch_copy16(const void* a, void* b, int64_t bytes, hipStream_t s);
hipError_t launch_read16(const void* a, int64_t bytes, int* out, int grid, hipStream_t s);

// ras.hip: one restricted additive Schwarz application (all subdomains of
// all slots), forward and backward block triangular solves with gather and
// scatter fused.  F = factor precision, V = vector precision.
template <typename F, typename V>
hipError_t launch_ras(const RasLaunch& p, int grid, hipStream_t s);
// readies a counter array of launch_ras (4 words): ticket and error words
// zeroed, the epoch of its next launch set; every launch leaves the next one's
hipError_t launch_ras_seed(int32_t* counter, hipStream_t s);

// lu.hip
template <typename F>
hipError_t launch_extract(const FacDesc* d, int nd, int maxn, hipStream_t s);
// complete blocked LU of every subdomain (maxN = largest tile count)
template <typename F>
hipError_t launch_lu(const FacDesc* d, int nd, int maxN, int* err, hipStream_t s);
// inverse panels X_p = J_p^{-1} E_o of every subdomain with d.X set, from its
// LU factors: block forward substitution over fsteps tile rows, then block
// back substitution over bsteps tile rows, four tile rows per launch (X
// zero-filled before)
template <typename F>
hipError_t launch_xinv(const FacDesc* d, int nd, int maxNo, int fsteps, int bsteps, hipStream_t s);
// packed symmetric form d.Xs of every subdomain's panels d.X (maxPacked =
// most packed tiles of a subdomain)
template <typename F>
hipError_t launch_xpack(const FacDesc* d, int nd, int maxPacked, hipStream_t s);

// ilu.hip: values of the ILU pattern from the level's FP64 CSR values (0 on
// fill), the factorisation (err set on a non-positive pivot) and the
// smoother application z = B^{-1} r (add = 0) or z += B^{-1} r (add = 1);
// maxn = the largest subdomain of the launch, lanes (4, 8, 16 or 32) per row
// of the triangular solves
template <typename T>
hipError_t launch_ilu_extract(const int32_t* asrc, const double* a, T* val, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_ilu_factor(const IluDesc* d, int nd, int lanes, int* err, hipStream_t s);
template <typename T>
hipError_t launch_ilu_apply(const IluDesc* d, int nd, int maxn, int lanes, int add, hipStream_t s);

// assemble.hip
hipError_t launch_assemble(const AsmDesc& a, const KappaDev& k, double f, hipStream_t s);

// krylov.hip (T = precision of the level-0 preconditioner vectors)
template <typename T>
hipError_t launch_krylov_cast_in(const KrylovDesc* d, int nd, int nblocks, hipStream_t s);
template <typename T>
hipError_t launch_krylov_cast_out(const KrylovDesc* d, int nd, int nblocks, hipStream_t s);
hipError_t launch_krylov_dots1(const KrylovDesc* d, int nd, int nblocks, hipStream_t s);
hipError_t launch_krylov_upd1(const KrylovDesc* d, int nd, int nblocks, hipStream_t s);
hipError_t launch_krylov_upd2(const KrylovDesc* d, int nd, int nblocks, hipStream_t s);
hipError_t launch_krylov_givens(const KrylovDesc* d, int nd, hipStream_t s);
hipError_t launch_krylov_normalize(const KrylovDesc* d, int nd, int nblocks, hipStream_t s);
hipError_t launch_krylov_xupd(const KrylovDesc* d, int nd, int nblocks, hipStream_t s);
hipError_t launch_krylov_cycle(const KrylovDesc* d, int nd, hipStream_t s);
hipError_t launch_krylov_init_slot(const KrylovDesc* d, int nd, int boff, int nblocks, hipStream_t s);
hipError_t launch_krylov_start_slot(const KrylovDesc* d1, double rtol, int restart, int max_it, hipStream_t s);
hipError_t launch_count_active(const KrylovDesc* d, int nd, int* out, hipStream_t s);

}  // namespace nnms
