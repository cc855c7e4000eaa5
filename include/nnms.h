/*
 * nnms.h -- C ABI of the non-nested multilevel smoothed Schwarz solver.
 *
 * Method: C. Ma, "A non-nested unstructured mesh perspective on highly
 * parallel multilevel smoothed Schwarz preconditioner for linear parametric
 * PDEs" (arXiv 2412.08981).  The library solves the P1 discretisation of
 * -div(kappa grad u) = f on a tetrahedral mesh with homogeneous Dirichlet
 * data (Section 2.1, equation 'discretized'), right-preconditioned
 * (equation 'right-preconditioned') by the V-cycle of Algorithm 2
 * (Section 3.3): on every level but the coarsest, a restricted additive
 * Schwarz smoother (Section 2.2) over overlapping subdomains with exact
 * dense subdomain LU solves; between independently meshed (non-nested)
 * levels, barycentric interpolation P_l (a fine vertex located in a coarse
 * tetrahedron) and its transpose; a direct solve on the coarsest level.  The
 * outer Krylov method is flexible GMRES (Section 4 uses GMRES).
 *
 * Conventions shared by every call
 *  - Every call returns nnms_status; no exception crosses the ABI.  After a
 *    non-OK status, nnms_last_error() returns a thread-local message.
 *  - Handles are owned by the library and released by the matching
 *    *_destroy call.  Caller buffers are only accessed during the call; the
 *    library keeps no caller pointer.
 *  - Pointers named *_host are host memory; pointers documented as device
 *    memory must be HIP device pointers on the handle's device.
 *  - Device work is ordered on the hipStream_t passed as `stream` (NULL is
 *    the null stream).  Calls that return results to the host synchronise
 *    that stream before returning.
 *  - A handle must not be used by two host threads at once; different
 *    handles may.
 *  - Indices are 0-based.  Vertex-indexed vectors have one entry per mesh
 *    vertex; entries at Dirichlet vertices of right-hand sides are ignored
 *    (treated as 0) and solutions are 0 there.
 */
#ifndef NNMS_H
#define NNMS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NNMS_MAX_LEVELS 8
#define NNMS_MAX_RESTART 64

typedef enum {
  NNMS_OK = 0,
  NNMS_ERR_INVALID_ARG = 1,    /* a null pointer, a size out of range, a bad option */
  NNMS_ERR_BAD_MESH = 2,       /* vertex index out of range or tetrahedron volume <= 0 */
  NNMS_ERR_POINT_LOCATION = 3, /* a fine vertex lies outside the next coarser mesh */
  NNMS_ERR_OUT_OF_MEMORY = 4,  /* host or device allocation failed */
  NNMS_ERR_BUDGET = 5,         /* request exceeds the memory budget given to the call */
  NNMS_ERR_SINGULAR = 6,       /* a non-positive or non-finite pivot in a factorisation */
  NNMS_ERR_NOT_CONVERGED = 7,  /* iteration limit reached; x and info are still filled */
  NNMS_ERR_DEVICE = 8,         /* a HIP runtime error */
  NNMS_ERR_IN_USE = 9          /* the handle still has dependants (e.g. live systems) */
} nnms_status;

typedef enum { NNMS_FP64 = 0, NNMS_MIXED = 1 } nnms_precision;
/* Transfer between levels: barycentric P1 interpolation (each fine vertex
 * located in a coarse tetrahedron) or the moving-least-squares interpolation
 * of Section 3.2. */
typedef enum { NNMS_TRANSFER_BARYCENTRIC = 0, NNMS_TRANSFER_MLS = 1 } nnms_transfer;
/* Subdomain solver of the smoother: exact dense LU, or ILU(k) with level of
 * fill k (Section 4 runs ILU(2) on the finest level and ILU(0) on coarser
 * ones).  The coarsest level is always solved directly. */
typedef enum { NNMS_SUBSOLVER_LU = 0, NNMS_SUBSOLVER_ILU = 1 } nnms_subsolver;
typedef enum { NNMS_APPLY_SWEEPS = 0, NNMS_APPLY_INVERSE = 1 } nnms_dense_apply;

typedef struct nnms_mesh nnms_mesh;
typedef struct nnms_hierarchy nnms_hierarchy;
typedef struct nnms_system nnms_system;
typedef struct nnms_batch nnms_batch;

/* Device allocator supplied by the caller (e.g. a framework's caching
 * allocator).  alloc returns a device pointer aligned to 256 bytes or NULL;
 * free releases it.  When no allocator is given the library calls hipMalloc
 * and hipFree. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} nnms_allocator;

const char* nnms_last_error(void);
/* Bytes of device memory currently held by the library (all handles). */
int64_t nnms_device_bytes_in_use(void);

/* ---------------------------------------------------------------------------
 * Meshes (Section 2.1: the mesh perspective M = (K, N) with one unknown per
 * vertex, N = (1, 0, 0, 0)).
 *
 * xyz_host        nv*3 doubles, vertex coordinates (x, y, z per vertex).
 * tets_host       nt*4 int32 vertex ids; every tetrahedron must have a
 *                 positive signed volume det[x1-x0, x2-x0, x3-x0] / 6.
 * dirichlet_host  nv bytes, nonzero marks a homogeneous Dirichlet vertex;
 *                 NULL marks the vertices lying on the faces of the
 *                 bounding box (coordinate equal to the min or max).
 * Errors: NNMS_ERR_INVALID_ARG (nv < 4, nt < 1, null pointers),
 *         NNMS_ERR_BAD_MESH (index out of range, volume <= 0).
 * ------------------------------------------------------------------------- */
nnms_status nnms_mesh_create(int64_t nv, const double* xyz_host, int64_t nt, const int32_t* tets_host,
                             const uint8_t* dirichlet_host, nnms_mesh** out);
void nnms_mesh_destroy(nnms_mesh* m);

/* ---------------------------------------------------------------------------
 * setup(hierarchy): everything that depends on the meshes only and is reused
 * across parameters (Section 1 and Section 2.1: the mesh perspective is a
 * reusable object; the hierarchy M_0..M_{L-1} of Algorithm 2).
 *
 * Per smoothed level l < L-1: the CSR pattern of the vertex graph (Dirichlet
 * rows hold only their diagonal, Dirichlet columns are dropped from the
 * other rows), a partition of the interior vertices into nparts[l] owned
 * sets by recursive coordinate bisection and their extension by `overlap`
 * layers (Section 2.2), and the interpolation P_l from level l+1 to level
 * l with its transpose (the restriction).  The coarsest level gets one dense
 * "subdomain" holding all of its interior vertices (the direct solve).
 *
 * levels      L mesh handles, finest first (1 <= L <= NNMS_MAX_LEVELS).
 * opts        nparts[l]: power of two >= 1 for l < L-1 (0 selects
 *             max(2, 2^floor(log2(nv_l/1500))));  overlap >= 0;  its >= 1;
 *             precision NNMS_FP64 or NNMS_MIXED;
 *             transfer NNMS_TRANSFER_BARYCENTRIC (default) or
 *             NNMS_TRANSFER_MLS: the row of P_l for a fine vertex x* is
 *             the weighted least-squares fit of a linear polynomial to the
 *             coarse vertices within rho of x* (Section 3.2, the loss with
 *             w = 1 - 6r^2 + 8r^3 - 3r^4 and its stationary-point system),
 *             evaluated at x*; rho starts at mls_alpha (default 1.0) times
 *             the mean coarse edge length and grows by 1.25 until the
 *             neighbourhood has full rank (Theorem 1).  The neighbourhood
 *             is not clipped to a subdomain: the whole coarse level is
 *             resident on the device; with mls_restrict = 1 the residual
 *             goes down by the second MLS interpolation of Algorithm 2, from
 *             the fine to the coarse nodes (scale from the mean fine edge
 *             length), instead of P_l^T;
 *             subsolver NNMS_SUBSOLVER_LU (default: dense LU of every
 *             overlapping subdomain matrix) or NNMS_SUBSOLVER_ILU: ILU(k)
 *             of A[S_p, S_p] in natural ordering with k = ilu_fill[l]
 *             (defaults 2 on level 0, 0 elsewhere), factorised on the
 *             device at every assembly and applied by level-scheduled
 *             triangular solves; a subdomain may hold at most 8192 rows
 *             (FP64) or 16384 (mixed) with ILU, and a row of its ILU
 *             pattern at most 128 entries (64 below and 64 above the
 *             diagonal): NNMS_ERR_INVALID_ARG otherwise (lower the fill).
 * alloc       device allocator or NULL (hipMalloc).
 * stream      stream for the uploads.
 * Errors: NNMS_ERR_INVALID_ARG, NNMS_ERR_POINT_LOCATION (a fine vertex
 *         outside the coarse mesh, or no full-rank MLS neighbourhood),
 *         NNMS_ERR_OUT_OF_MEMORY, NNMS_ERR_DEVICE.
 *             mls_clip = 1: the paper's clipped neighbourhood (Section 3.2):
 *             both levels of a transfer are split across the same
 *             nparts[l] processors by coordinate bisection of their interior
 *             vertices with `overlap` layers; a target vertex owned by p
 *             takes its MLS neighbourhood only from the nodes of the source
 *             elements touching p's overlapping subdomain (boundary nodes
 *             included), rho grown until that neighbourhood has full rank;
 *             ncomp = 3 (multi-field problems by field splitting, Section
 *             3.2, equations field-split and interpolation split): P1 linear
 *             elasticity (Section 4.2's stress law) with the three
 *             displacement components of vertex v as unknowns 3v, 3v+1, 3v+2
 *             (all three Dirichlet on a Dirichlet vertex).  Every component
 *             is a field with one unknown per vertex: the pattern couples all
 *             components of neighbouring vertices, a subdomain holds all
 *             components of its vertices (the vertex partition), and the
 *             interpolation sum_f R_f^T P_l R~_f moves each component with the
 *             scalar P_l (barycentric or MLS).  nparts[l] = 0 then selects
 *             max(2, 2^floor(log2(3 nv_l / 1500))).
 *             dense_apply (levels with dense LU, the coarsest included):
 *             NNMS_APPLY_SWEEPS (default) applies R^0_p J_p^{-1} by the
 *             blocked forward and backward sweeps over the LU factors;
 *             NNMS_APPLY_INVERSE stores, at every assembly, the owned
 *             columns of the inverse, X_p = J_p^{-1} E_o (n_p x n_o, from
 *             the same LU factors by block forward and back substitution;
 *             on the coarsest level the whole inverse), kept as its
 *             overlap rows and the lower triangle of its symmetric owned
 *             block, and applies z_o = X_p^T r[S_p] (J_p is symmetric, so
 *             X_p^T holds the owned rows of J_p^{-1}): the same operator up
 *             to rounding, read as independent 64-column panels instead of
 *             chains of dependent blocks, for about twice the numeric
 *             setup.
 * nnms_hierarchy_setup_host builds the same structure without touching any
 * GPU (inspection and host tests); such a handle cannot be assembled.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t nparts[NNMS_MAX_LEVELS];
  int32_t overlap;
  int32_t its;
  int32_t precision;
  int32_t transfer;  /* nnms_transfer */
  double mls_alpha;  /* MLS initial scale / mean coarse edge length (> 0) */
  int32_t subsolver; /* nnms_subsolver of every smoothed level */
  int32_t ilu_fill[NNMS_MAX_LEVELS]; /* ILU level of fill per smoothed level (>= 0) */
  int32_t mls_restrict; /* with MLS: 1 = restrict by the MLS interpolation from
                           the fine to the coarse nodes, 0 = by P_l^T */
  int32_t ncomp;        /* unknowns per vertex: 1 = -div(kappa grad u) = f (default);
                           3 = P1 linear elasticity, see below */
  int32_t mls_clip;     /* with MLS: 1 = clip every neighbourhood to the overlapping
                           subdomain of the target's processor, see below */
  int32_t dense_apply;  /* nnms_dense_apply of the dense-LU levels, see below */
} nnms_setup_opts;

/* Geometry-preserving coarsening (Algorithm 1, Section 3.1): `rounds`
 * times (the paper's M, 8 in 3D), take a maximal independent set of the
 * interior (non-Dirichlet) vertices and remove every vertex of it by
 * contracting it onto the neighbour whose new elements have the best
 * smallest quality q = sqrt(2) 6V / l_rms^3 (at least 0.02, else the vertex
 * stays).  The MIS is Luby's with priorities splitmix64(seed + 2^40 round +
 * v).  Boundary vertices, their positions and the boundary surface are
 * kept; surviving vertices keep their positions, in ascending old id, with
 * their Dirichlet flags.  *out is a new mesh (nnms_mesh_destroy);
 * *removed (may be NULL) receives the number of removed vertices.
 * Errors: NNMS_ERR_INVALID_ARG (null mesh or output, rounds < 0). */
nnms_status nnms_mesh_coarsen(const nnms_mesh* fine, int32_t rounds, uint64_t seed, nnms_mesh** out,
                              int64_t* removed);
/* Read-back of a mesh: xyz_host[nv*3], tets_host[nt*4], dirichlet_host[nv]
 * (each may be NULL); *nv / *nt receive the counts. */
nnms_status nnms_mesh_read(const nnms_mesh* m, int64_t* nv, int64_t* nt, double* xyz_host, int32_t* tets_host,
                           uint8_t* dirichlet_host);

nnms_status nnms_setup_opts_default(nnms_setup_opts* o);
nnms_status nnms_hierarchy_setup(const nnms_mesh* const* levels, int32_t L, const nnms_setup_opts* opts,
                                 const nnms_allocator* alloc, void* stream, nnms_hierarchy** out);
nnms_status nnms_hierarchy_setup_host(const nnms_mesh* const* levels, int32_t L, const nnms_setup_opts* opts,
                                      nnms_hierarchy** out);
/* NNMS_ERR_IN_USE while systems assembled on it are alive. */
nnms_status nnms_hierarchy_destroy(nnms_hierarchy* h);

typedef struct {
  int64_t nv;           /* vertices */
  int64_t nt;           /* tetrahedra */
  int64_t ninterior;    /* non-Dirichlet vertices */
  int64_t nnz;          /* CSR entries of the level operator */
  int32_t nparts;       /* subdomains (1 on the coarsest level) */
  int32_t max_block;    /* largest subdomain size */
  int32_t min_block;    /* smallest subdomain size */
  int32_t transfer;     /* nnms_transfer of P_l (smoothed levels) */
  int64_t s_total;      /* sum of subdomain sizes */
  int64_t factor_elems; /* dense factor entries stored, incl. 64-padding (the
                           inverse panels of NNMS_APPLY_INVERSE not counted) */
  int64_t p_nnz;        /* entries of P_l (0 on the coarsest level) */
  int32_t subsolver;    /* nnms_subsolver of the level's smoother */
  int32_t mls_restrict; /* 1: the restriction is the fine-to-coarse MLS operator */
  int64_t ilu_nnz;      /* entries of all ILU patterns of the level (0 without ILU) */
  int64_t r_nnz;        /* entries of the restriction (P_l^T or the MLS operator) */
  int32_t ncomp;        /* unknowns per vertex */
  int32_t dense_apply;  /* nnms_dense_apply of a dense level */
  int64_t ndof;         /* unknowns of the level = ncomp * nv: the length of the
                           level's vectors and the rows of every per-row array
                           below (CSR, owner, P_l, ...) */
} nnms_level_info;

nnms_status nnms_hierarchy_level_info(const nnms_hierarchy* h, int32_t level, nnms_level_info* out);
/* CSR pattern of level `level`: row_ptr_host[nv+1], col_host[nnz]. */
nnms_status nnms_hierarchy_csr(const nnms_hierarchy* h, int32_t level, int32_t* row_ptr_host, int32_t* col_host);
/* Owner of every vertex (-1 for Dirichlet), and the overlapping sets S_p in
 * ascending vertex order: s_ptr_host[nparts+1], s_idx_host[s_total]. */
nnms_status nnms_hierarchy_partition(const nnms_hierarchy* h, int32_t level, int32_t* owner_host,
                                     int64_t* s_ptr_host, int32_t* s_idx_host);
/* P_level as 4 entries per fine vertex: idx_host[nv*4] coarse vertex ids,
 * w_host[nv*4] barycentric weights (0 for Dirichlet rows and columns).
 * Barycentric transfer only (NNMS_ERR_INVALID_ARG for MLS). */
nnms_status nnms_hierarchy_transfer(const nnms_hierarchy* h, int32_t level, int32_t* idx_host, double* w_host);
/* P_level as CSR over the fine vertices, either transfer: row_ptr_host[nv+1],
 * col_host[p_nnz], w_host[p_nnz] (p_nnz from nnms_hierarchy_level_info;
 * Dirichlet rows empty, Dirichlet coarse columns left out, columns ascending
 * within a row for MLS, in tetrahedron-vertex order for barycentric). */
nnms_status nnms_hierarchy_transfer_csr(const nnms_hierarchy* h, int32_t level, int32_t* row_ptr_host,
                                        int32_t* col_host, double* w_host);
/* The restriction of level `level` as CSR over the coarse vertices:
 * row_ptr_host[nv_{l+1}+1], col_host[r_nnz], w_host[r_nnz] (P_l^T, or the
 * fine-to-coarse MLS operator with mls_restrict). */
nnms_status nnms_hierarchy_restriction_csr(const nnms_hierarchy* h, int32_t level, int32_t* row_ptr_host,
                                           int32_t* col_host, double* w_host);
/* ILU levels: the ILU(k) pattern of every subdomain in local numbering (the
 * subdomain's rows in the order of nnms_hierarchy_partition's S_p), rows of
 * all subdomains concatenated: row_ptr_host[s_total+1] entry offsets,
 * col_host[ilu_nnz] local columns, ascending within a row.
 * NNMS_ERR_INVALID_ARG on a level without ILU. */
nnms_status nnms_hierarchy_ilu_pattern(const nnms_hierarchy* h, int32_t level, int32_t* row_ptr_host,
                                       int32_t* col_host);

/* ---------------------------------------------------------------------------
 * assemble(mesh, kappa): numeric setup for one parameter (Section 2.1: the
 * parameters mu of a parametric problem enter the coefficients, and the mesh
 * hierarchy is reused across them).  On the device: kappa of every
 * tetrahedron, P1 stiffness of every level (coarse levels rediscretised, as
 * Algorithm 2 provides the Jacobian of every level), the load vector on the
 * finest level, extraction of the overlapping subdomain matrices
 * J_p = R_p J R_p^T (Section 2.2) and their factorisation without pivoting
 * (the matrices are SPD), plus the coarsest dense FP64 LU.
 *
 * kappa (host memory; nothing is kept after the call):
 *   kind 0  constant `value` (> 0);
 *   kind 1  log-Gaussian, log kappa(x) = sum_k mu[k] exp(-|x - centres[k]|^2
 *           / width) at every tetrahedron's centroid, ncentres <= 64,
 *           width > 0;
 *   kind 2  given per tetrahedron: per_tet[l] holds nt_l doubles, the value
 *           on every tetrahedron of level l, for every level l of the
 *           hierarchy (finite and > 0; coarse levels carry their own values,
 *           e.g. the field at their own centroids).
 * rhs, the source term f of the load vector b_i = int f phi_i on the finest
 * level (host memory):
 *   kind 0  constant `value`: b_i = f sum_{T at i} |T| / 4;
 *   kind 1  one value per tetrahedron of the finest level (values[nt_0]),
 *           f constant on each: b_i = sum_{T at i} f_T |T| / 4;
 *   kind 2  P1 nodal values of the finest level (values[nv_0]), f taken as
 *           its interpolant sum_j f_j phi_j and integrated exactly with the
 *           element mass matrix |T| (1 + delta_ab) / 20: b_i =
 *           sum_{T at i} |T| / 20 (f_i + sum_{a in T} f_a).
 *   Values must be finite.  Entries of Dirichlet vertices are 0.
 *   ncomp = 3 (linear elasticity, E_T = kappa_T, Poisson's ratio from the
 *   options): f is a body force, every component loaded as above: kind 0
 *   takes vector[0..2], kind 1 three values per tetrahedron (x, y, z), kind 2
 *   the nodal values in the unknowns' order (3v + c).
 * Errors: NNMS_ERR_INVALID_ARG (a bad kind, size or value: before any device
 *         work), NNMS_ERR_BUDGET, NNMS_ERR_SINGULAR, NNMS_ERR_OUT_OF_MEMORY,
 *         NNMS_ERR_DEVICE.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t kind;
  int32_t ncentres;
  double value;
  const double* centres; /* kind 1: ncentres*3 */
  const double* mu;      /* kind 1: ncentres */
  double width;          /* kind 1 */
  const double* const* per_tet; /* kind 2: one array per level, nt_l doubles each */
} nnms_kappa;

typedef struct {
  int32_t kind;
  int32_t reserved;
  double value;          /* kind 0 */
  const double* values;  /* kind 1: nt_0 * ncomp doubles; kind 2: ndof_0 doubles */
  double vector[3];      /* kind 0 with ncomp = 3: the constant body force */
} nnms_rhs;

/* restart_cap  Krylov basis columns kept with the system for its solves
 *              (1..NNMS_MAX_RESTART; 0 = NNMS_MAX_RESTART); a solve or batch
 *              asking for a larger restart gives NNMS_ERR_INVALID_ARG.
 * max_device_bytes  > 0: the device memory this assembly may take; the
 *              assembly is refused with NNMS_ERR_BUDGET, before any device
 *              work, when nnms_hierarchy_system_bytes(h, restart_cap) (the
 *              peak of any assembly of h) exceeds it.  0: no limit. */
/* poisson_ratio  ncomp = 3: nu in [0, 0.5); the Lame coefficients are
 *              mu = E / (2 (1 + nu)), lambda = E nu / ((1 + nu)(1 - 2 nu)). */
typedef struct {
  const nnms_kappa* kappa; /* required */
  const nnms_rhs* rhs;     /* NULL: f = 1 (every component for ncomp = 3) */
  int32_t restart_cap;
  int32_t reserved;
  int64_t max_device_bytes;
  double poisson_ratio;
} nnms_assemble_opts;

nnms_status nnms_assemble_ex(nnms_hierarchy* h, const nnms_assemble_opts* opts, void* stream, nnms_system** out);
/* The same with a constant load f (each component for ncomp = 3, Poisson's
 * ratio 0.3), restart_cap NNMS_MAX_RESTART and no budget. */
nnms_status nnms_assemble(nnms_hierarchy* h, const nnms_kappa* kappa, double f, void* stream, nnms_system** out);
nnms_status nnms_system_destroy(nnms_system* s);
/* Device bytes held by one assembled system (values, factors, workspace). */
int64_t nnms_system_device_bytes(const nnms_system* s);
/* Device bytes an assembly of h with restart_cap = restart (0: NNMS_MAX_RESTART)
 * takes at its peak: what the system keeps (nnms_system_device_bytes) plus
 * what the assembly holds only while it runs (element matrices of the
 * largest level, per-tetrahedron kappa and load arrays, descriptors, and
 * with NNMS_APPLY_INVERSE the full panels of every level before packing), for
 * admission decisions; -1 for a null handle or a restart out of range.  The
 * solve plans a system's first solve and operator calls build add a few KiB
 * to a few MiB (descriptors, task lists), recycled through a per-process
 * cache of at most 64 MiB. */
int64_t nnms_hierarchy_system_bytes(const nnms_hierarchy* h, int32_t restart);

/* Read-back for checks: the load vector (nv_0 doubles) and the FP64 CSR
 * values of a level (nnz doubles, order of nnms_hierarchy_csr). */
nnms_status nnms_system_rhs(const nnms_system* s, double* b_host);
nnms_status nnms_system_matrix(const nnms_system* s, int32_t level, double* val_host);

/* Read-back of the stored dense factor of subdomain `part` of `level` (the
 * coarsest level has one part), for checks.  The subdomain is padded to N
 * tiles of 64 per side.  lu_host (may be NULL) receives the (N*64)^2 tile
 * grid row-major as stored: L_ij below the diagonal tiles, U_ij above them,
 * inv(U_ii) in the diagonal tiles.  invl_host (may be NULL) receives the N
 * tiles inv(L_ii), each 64x64 row-major.  *N_host receives N.
 * Row and column k < |S_p| of the factor is vertex (unknown) k of the local
 * order: on a smoothed level the members of S_p that the part does not own,
 * ascending, then the ones it owns, ascending (the restricted solve keeps
 * only x_o = inv(U_oo) y_o, so its backward sweep runs over the owned rows
 * alone); on the coarsest level S order.  The padding rows follow. */
nnms_status nnms_system_factor(const nnms_system* s, int32_t level, int32_t part, double* lu_host, double* invl_host,
                               int32_t* N_host);

/* Read-back of the pair coupling tiles of the same factor: for tile pairs
 * (a, b) = (2p, 2p+1), p < floor(N/2), the off-diagonal blocks of the
 * inverses of the 128 x 128 diagonal blocks,
 *   xl_host[p] = -inv(L_bb) L_ba inv(L_aa),  xu_host[p] = -inv(U_aa) U_ab inv(U_bb),
 * each 64x64 row-major (either may be NULL); *npairs_host receives
 * floor(N/2).  The two-block triangular-solve work items apply them. */
nnms_status nnms_system_factor_pairs(const nnms_system* s, int32_t level, int32_t part, double* xl_host, double* xu_host,
                                     int32_t* npairs_host);
/* Both dense read-backs give NNMS_ERR_INVALID_ARG on an ILU level. */

/* Read-back of the inverse panels of subdomain `part` of `level`
 * (NNMS_APPLY_INVERSE levels only, else NNMS_ERR_INVALID_ARG), for checks:
 * X_p = J_p^{-1} E_o, the owned columns of the inverse of the subdomain
 * matrix in the factor's local order, unpacked from the stored form (the
 * overlap rows and the lower triangle of the symmetric owned block; its
 * upper triangle is the transpose).  x_host (may be NULL: sizes only)
 * receives the (N*64) x (No*64) matrix row-major, FP32 panels widened;
 * row k < |S_p| is local row k, column c < n_o is owned row c (local row
 * |S_p| - n_o + c); padding rows and columns are zero.  *N_out and *No_out
 * (either may be NULL) receive N and No = ceil(n_o / 64). */
nnms_status nnms_system_inverse_panels(const nnms_system* s, int32_t level, int32_t part, double* x_host,
                                       int32_t* N_out, int32_t* No_out);

/* Read-back of the ILU factors of an ILU level: val_host[ilu_nnz] in the
 * order of nnms_hierarchy_ilu_pattern, L's multipliers (unit diagonal not
 * stored) below the diagonal, U on and above it; FP32 factors of mixed
 * precision are widened. */
nnms_status nnms_system_ilu_values(const nnms_system* s, int32_t level, double* val_host);

/* ---------------------------------------------------------------------------
 * Operator applications, one call each, host vectors in and out (FP64 at
 * the boundary; the level's working precision inside):
 *   nnms_apply_operator   y = A_l x                        (Section 2.1)
 *   nnms_apply_smoother   z = B_l^{-1} r, restricted additive Schwarz
 *                         (Section 2.2); on the coarsest level the direct
 *                         solve A_{L-1}^{-1} r
 *   nnms_apply_prolong    z_l = P_l z_{l+1}   (level = l, x has nv_{l+1})
 *   nnms_apply_restrict   r_{l+1} = P_l^T r_l
 *   nnms_apply_vcycle     z = M r, one V-cycle of Algorithm 2
 * ------------------------------------------------------------------------- */
nnms_status nnms_apply_operator(nnms_system* s, int32_t level, const double* x_host, double* y_host, void* stream);
nnms_status nnms_apply_smoother(nnms_system* s, int32_t level, const double* r_host, double* z_host, void* stream);
nnms_status nnms_apply_prolong(nnms_system* s, int32_t level, const double* x_host, double* y_host, void* stream);
nnms_status nnms_apply_restrict(nnms_system* s, int32_t level, const double* x_host, double* y_host, void* stream);
nnms_status nnms_apply_vcycle(nnms_system* s, const double* r_host, double* z_host, void* stream);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid allocation): nnms_apply_smoother on device vectors,
 * allocating nothing.  The launch's tables (ticket, epoch and error words,
 * subdomain or ILU descriptors, task list) go to a static array of
 * NNMS_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends, instead
 * of library-allocated memory; the level vectors and hand-off workspace
 * are the system's own (allocated by its assembly).  Results are bitwise
 * those of nnms_apply_smoother.
 *
 * r_dev, z_dev  device pointers, nv_level doubles each (r read, z written;
 *               z is 0 at Dirichlet unknowns).
 * Errors: NNMS_ERR_INVALID_ARG (null pointers, bad level, the calling
 *         thread's current device is not the system's, or the level's
 *         tables exceed the array: e.g. about 16,000 subdomains on one
 *         level), NNMS_ERR_DEVICE (a HIP error or a triangular-solve wait
 *         limit reached; the error word is cleared for later calls).
 * Every call on one GPU shares that GPU's array and leaves it with the last
 * call's tables: calls that overlap on one GPU (other streams or host
 * threads) race and must be serialised by the caller.  The call synchronises
 * `stream` to read the launch's error word.
 * ------------------------------------------------------------------------- */
#define NNMS_NOALLOC_SCRATCH_BYTES (1 << 20)
nnms_status nnms_apply_smoother_noalloc(nnms_system* s, int32_t level, const double* r_dev, double* z_dev,
                                        void* stream);

/* ---------------------------------------------------------------------------
 * Measurement: run one kernel of the solve path `reps` times back to back on
 * the stream it is launched on, bracketed by HIP events, on the system's
 * current level vectors; *ms_host receives the mean milliseconds per
 * launch.  kind: 0 smoother (restricted additive Schwarz apply, or the
 * coarsest direct solve), 1 level operator residual t = r - A z,
 * 2 prolongation, 3 restriction, 4 a plain 16-byte streaming copy of the
 * level's factor storage into a temporary buffer (a reference of known
 * size for hardware byte counters), 5 a read-only streaming pass over the
 * level's factor storage (the achievable read bandwidth), 6 the level's
 * numeric factorisation (zero fill of the tile storage, extraction of the
 * dense subdomain matrices, blocked LU), redone in place from the same
 * matrix values, which reproduces the same factors.  reps >= 1.
 * ------------------------------------------------------------------------- */
nnms_status nnms_time_kernel(nnms_system* s, int32_t kind, int32_t level, int32_t reps, double* ms_host);

/* ---------------------------------------------------------------------------
 * Launch-shape tuning, per hierarchy (used by every solve plan created after
 * it is set).  A batch keeps every system's own lanes-per-row and
 * blocks-per-work-item choices (they fix the summation order, so a system
 * gives the same bits alone and in any batch: one launch per distinct
 * choice) and takes each smoother launch's work-group count from the first
 * system of its launch (it changes no arithmetic).
 *   spmv_lanes[l]  lanes of a wave per CSR row of level l's operator (4..64),
 *                  or the operator in sliced ELL layout (64-row slices, one
 *                  lane per row, slices column-major): 0 = one wave per
 *                  slice, 1 = the slice's entries split over the four waves
 *                  of a work-group and the four partial sums of a row added
 *                  in a fixed order
 *   pt_lanes[l]    the same choice for P_l^T (4..64, 0 or 1), or 2: P_l^T in
 *                  column-sorted slices (64 rows per slice, the slice's
 *                  entries stored in fine-column order so that the gathers
 *                  of a wave read runs of consecutive fine entries; the
 *                  products regrouped by row in LDS and each row summed by
 *                  four lanes in a fixed order); accepted where every slice
 *                  holds at most 4096 entries spanning fewer than 2^19
 *                  columns, else nnms_hierarchy_set_tuning returns
 *                  NNMS_ERR_INVALID_ARG
 *   ras_groups[l]  work-groups of the persistent triangular-solve kernel on
 *                  level l (0 = 4 per compute unit)
 *   ras_blocks[l]  64-row blocks per work item of that kernel (1, 2 or 4);
 *                  only work items hand results to each other.  With 4 the
 *                  blocks of a work item are substituted one after the other
 *                  by one work-group (the same sums as 1); with 2 the pair's
 *                  precomputed 128 x 128 block inverse gives both blocks in
 *                  one step (other rounding)
 *   krylov_lanes   the same choice for the outer FP64 operator
 * nnms_autotune times the candidates of every entry on the system's own
 * data with HIP events (reps launches each), keeps the fastest, stores the
 * result in the system's hierarchy and in *out (may be NULL).
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t spmv_lanes[NNMS_MAX_LEVELS];
  int32_t pt_lanes[NNMS_MAX_LEVELS];
  int32_t ras_groups[NNMS_MAX_LEVELS];
  int32_t ras_blocks[NNMS_MAX_LEVELS];
  int32_t krylov_lanes;
  int32_t tuned; /* 1 after nnms_autotune or a tuning that was set */
} nnms_tuning;

nnms_status nnms_hierarchy_get_tuning(const nnms_hierarchy* h, nnms_tuning* out);
nnms_status nnms_hierarchy_set_tuning(nnms_hierarchy* h, const nnms_tuning* t);
nnms_status nnms_autotune(nnms_system* s, int32_t reps, nnms_tuning* out);

/* ---------------------------------------------------------------------------
 * solve(b) -> x, iterations: right-preconditioned flexible GMRES(restart)
 * with classical Gram-Schmidt applied twice, x0 = 0, stopping when the true
 * residual satisfies ||b - A x||_2 <= rtol ||b||_2 (checked at the end of
 * every cycle).  iterations counts Arnoldi steps over all cycles.
 *
 * b, x: nv_0 doubles, host memory unless flags & NNMS_DEVICE_PTRS.
 * restart in [1, NNMS_MAX_RESTART]; rtol > 0; max_it >= 1.
 * ||b|| = 0 gives x = 0 and iterations = 0.
 * NNMS_ERR_NOT_CONVERGED: max_it reached; x holds the last iterate and info
 * is filled.
 * nnms_solve replays each Arnoldi step from one HIP graph, captured on the
 * system's first solve (unless NNMS_NO_GRAPH): first as many steps back to
 * back as the system's previous solve took (at most 64), with one host
 * read of the running count after them, then one step at a time while the
 * slot still iterates.  Steps after convergence change nothing, so x and
 * info do not depend on earlier solves.
 * ------------------------------------------------------------------------- */
#define NNMS_DEVICE_PTRS 1
#define NNMS_NO_GRAPH 2

typedef struct {
  int32_t restart;
  int32_t max_it;
  double rtol;
  int32_t flags;
  int32_t reserved;
} nnms_solve_opts;

typedef struct {
  int32_t iterations;
  int32_t cycles;
  int32_t status;   /* nnms_status of this right-hand side (NOT_CONVERGED while running) */
  int32_t running;  /* 1 while the slot is still iterating, else 0 */
  double relres;    /* true ||b - A x|| / ||b|| at the last cycle end */
} nnms_solve_info;

nnms_status nnms_solve_opts_default(nnms_solve_opts* o);
nnms_status nnms_solve(nnms_system* s, const double* b, double* x, const nnms_solve_opts* opts,
                       nnms_solve_info* info, void* stream);

/* ---------------------------------------------------------------------------
 * Batched solves: several assembled systems (any mix of hierarchies with
 * the same number of levels and precision) advance together, one Arnoldi
 * step per launch sequence, each with its own Krylov basis, rotations and
 * convergence test; a finished system is masked out while the others go
 * on.  Each system's arithmetic is independent of its batch neighbours, so
 * its result is the same alone and in any batch.
 *
 * nnms_batch_create   bind systems to the slots of a batch (nb >= 1).  A
 *                     slot keeps its system's solve state: a freshly
 *                     assembled system is idle, and a system still
 *                     iterating in another batch continues from where it
 *                     is (this is how a serving loop re-forms its batch
 *                     when requests join or leave).  A system must not be
 *                     stepped by two batches at the same time.
 * nnms_batch_start    begin solving in `slot` with right-hand side b
 *                     (device pointer, nv_0 doubles; copied after the work
 *                     enqueued so far on the stream given to
 *                     nnms_batch_create).
 * nnms_batch_step     run up to `iterations` Arnoldi steps on every active
 *                     slot (replayed from a captured HIP graph unless
 *                     NNMS_NO_GRAPH); *active_host receives the number of
 *                     slots still iterating.
 * nnms_batch_result   copy slot's solution to x (device pointer) and info;
 *                     the copy follows the work enqueued so far on the stream
 *                     given to nnms_batch_create, and that stream's later
 *                     work follows the copy.
 * nnms_batch_destroy  wait for the batch's own stream (not the device) and
 *                     drop it; its stream, pinned word and small device
 *                     buffers are kept by the library for later batches
 *                     (at most 64 MiB of device buffers per process).
 * ------------------------------------------------------------------------- */
nnms_status nnms_batch_create(nnms_system* const* systems, int32_t nb, const nnms_solve_opts* opts, void* stream,
                              nnms_batch** out);
nnms_status nnms_batch_start(nnms_batch* bt, int32_t slot, const double* b_device);
nnms_status nnms_batch_step(nnms_batch* bt, int32_t iterations, int32_t* active_host);
nnms_status nnms_batch_result(nnms_batch* bt, int32_t slot, double* x_device, nnms_solve_info* info);
nnms_status nnms_batch_destroy(nnms_batch* bt);

/* All-in-one batched solve (host or device vectors per opts->flags). */
nnms_status nnms_solve_batch(nnms_system* const* systems, int32_t nb, const double* const* b, double* const* x,
                             const nnms_solve_opts* opts, nnms_solve_info* infos, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* NNMS_H */
