// Plain-old-data descriptors shared by the host driver and the HIP kernels.
// Every batched kernel receives an array of descriptors (one per solve slot
// or per subdomain) so that one launch serves any mix of systems.
#pragma once
#include <cstdint>

#include "nnms.h"

namespace nnms {

constexpr int MMAX = NNMS_MAX_RESTART;
constexpr int VBLK = 2048;   // rows per block of the Krylov vector kernels (256 threads x 8)
constexpr int MAXC = 64;     // kappa centres
constexpr int TILE = 64;     // dense factor tile edge
constexpr int TILE_ELEMS = TILE * TILE;

enum When : int32_t { WHEN_RUNNING = 0, WHEN_CYCLE_END = 1 };
enum SlotStatus : int32_t { ST_RUNNING = 0, ST_CONVERGED = 1, ST_MAXIT = 2, ST_IDLE = 3 };

// Per-slot FGMRES state, resident on the device.
struct KState {
  int32_t status;
  int32_t j;           // current Arnoldi column
  int32_t its;         // Arnoldi steps so far (all cycles)
  int32_t cycles;
  int32_t cycle_end;   // this step ends a cycle
  int32_t pending_v0;  // V[:,0] still has to be formed from w / beta
  int32_t restart;
  int32_t max_it;
  double rtol, bnorm, tol, beta, hnext, relres;
  double g[MMAX + 1], cs[MMAX], sn[MMAX], y[MMAX], h1[MMAX + 1];
  double R[MMAX * MMAX];  // column-major upper triangle, R[k + j*MMAX]
};

// A CSR matrix in column-sorted slices (the restriction P^T): rows in slices
// of 64; the entries of a slice are those of its rows, stored in column
// order (ties in row order), each keyed by
//   (column - the slice's smallest column) << CSORT_SLOT_BITS | p,
// p its position in the slice's row-major (CSR) order.
constexpr int CSORT_SLOT_BITS = 12;  // at most 4096 entries per slice
constexpr int64_t CSORT_MAX_SPAN = int64_t(1) << (31 - CSORT_SLOT_BITS);  // columns a slice may span

struct SpmvDesc {
  const int32_t* rp;
  const int32_t* col;  // column ids, or the keys of the column-sorted slices
  const void* val;
  const void* x;
  const void* r;       // optional: y = r - A x
  void* y;
  double* nrm;         // optional: per-block partial sums of y^2 (FP64 only)
  const KState* st;    // null: always active
  const int32_t* base; // column-sorted slices: each slice's smallest column
  int64_t x_jstride;   // x += state.j * x_jstride
  int32_t n;
  int32_t blk0;        // first block of this descriptor
  int32_t when;
  int32_t cap;         // column-sorted slices: most entries in one slice
};

struct ProlongDesc {
  const int32_t* idx;  // n*4 coarse ids
  const void* w;       // n*4 weights
  const void* zc;
  void* zf;            // zf += P zc
  const KState* st;
  int32_t n;
  int32_t blk0;
};

// One overlapping subdomain of one system, for the triangular-solve kernel
// (sweeps) or the inverse-panel kernel (fac = the packed symmetric panels:
// X_v, Nv x No tiles column-major, then the lower triangle of X_oo by
// columns; the owned rows are local rows nv .. nv + no - 1).
struct SubDesc {
  const void* fac;      // N*N tiles (L below, U above, inv(U_ii) on the diagonal) + N tiles inv(L_ii)
  const int32_t* gidx;  // N*64 encoded global ids: >=0 owned, <=-2 overlap (-g-2), -1 padding
  void* yx;             // N*64 workspace (forward result, then solution)
  const void* rin;      // level residual vector
  void* zout;           // level correction vector
  const KState* st;     // null: always active
  void* part;           // inverse panels: column parts and pair partials (F)
  int32_t N;
  int32_t nv;           // local rows before the owned ones (inverse panels)
  int32_t no;           // owned rows (inverse panels)
  int32_t pad;
};

struct RasLaunch {
  const SubDesc* subs;
  const int32_t* tasks;  // (sub << 16) | (dir << 15) | work item (group of K blocks);
                         // inverse panels (group 0): (sub << 16) | tile column
  int32_t* counter;      // [0] ticket, [1] this launch's epoch, [2] error bits
  int32_t ntasks;
  int32_t add;           // z += x (1) or z = x (0)
  int32_t group;         // 64-row blocks per work item (1, 2 or 4); 0: inverse panels
  int32_t max_tiles;     // largest N among the subdomains
};

// One subdomain's ILU(k) factor for the factorisation and apply kernels.
// Row indices are local (0..n-1); entry indices point into the level's
// concatenated pattern arrays (col, val).
struct IluDesc {
  const int32_t* rp;     // n+1: first entry of every row
  const int32_t* dpos;   // n: entry of every row's diagonal
  const int32_t* col;    // local column of every entry (the level's array)
  const int32_t* fmeta;  // 4n, by forward level: {row, first entry, diagonal entry, end}
  const int32_t* flev;   // nfl+1: level boundaries in fmeta
  const int32_t* bmeta;  // 4n, by backward level: {row, diagonal + 1, end, diagonal entry}
  const int32_t* blev;   // nbl+1
  const int32_t* gid;    // n: global id (>= 0 owned, -g-2 overlap)
  void* val;             // factor values of every entry (the level's array)
  const void* rin;       // level residual vector
  void* zout;            // level correction vector
  const KState* st;      // null: always active
  int32_t n, nfl, nbl, pad;
};
// LDS of one apply work-group: the subdomain's vector
constexpr size_t ILU_MAX_LDS = 65536;

// Dense-factor work of one subdomain (extraction and LU).
struct FacDesc {
  void* fac;
  const int32_t* gidx;    // as in SubDesc
  const int32_t* ext_rs;  // start of every local row in ext_lc (n+1 entries)
  const int32_t* ext_lc;
  const int32_t* rp;      // level CSR
  const double* val;      // level FP64 values
  int32_t n;
  int32_t N;
  void* X;                // inverse panels (null: sweeps only), N x No tiles, column-major tile order
  void* Xs;               // their packed symmetric form (overlap rows, lower triangle of the owned block)
  int32_t nv;             // local rows before the owned ones
  int32_t No;             // tile columns of X: ceil(owned rows / 64)
};

struct KrylovDesc {
  double* V;        // n x (restart+1), column-major
  double* Z;        // n x restart
  double* w;
  double* x;
  double* b;        // right-hand side with Dirichlet entries zeroed
  const uint8_t* dmask;
  double* part1;    // nblk x (MMAX+1): dots with V, then |w|^2
  double* part2;    // nblk x MMAX
  double* partn;    // nblk
  double* partr;    // residual-norm partials of the cycle-end SpMV
  KState* st;
  void* r0;         // level-0 input of the preconditioner (T)
  void* z0;         // level-0 output of the preconditioner (T)
  int32_t n;
  int32_t blk0;
  int32_t nblk;
  int32_t nblkr;    // entries of partr
};

struct KappaDev {
  int32_t kind;
  int32_t nc;
  double value;
  double width;
  double c[MAXC * 3];
  double mu[MAXC];
};

struct AsmDesc {
  const double* xyz;
  const int32_t* tets;
  const int32_t* cptr;
  const int32_t* citem;
  const int32_t* rp;
  const int32_t* vptr;
  const int32_t* vitem;
  const uint8_t* dmask;
  double* elem;     // nt element matrices of 16 ncomp^2 entries, then nt volumes
  double* val64;
  float* val32;     // may be null
  double* b;        // may be null (load vector)
  const double* kappa_tet;  // kappa kind 2: value per tetrahedron
  const double* fval;       // load kinds 1 (per tetrahedron) and 2 (P1 nodal values)
  int64_t nt;
  int64_t nv;               // rows (unknowns): ncomp per vertex
  int32_t fkind;            // 0 constant, 1 per tetrahedron, 2 nodal
  int32_t ncomp;            // 1: -div(kappa grad u) = f; 3: linear elasticity, E = kappa
  double nu;                // Poisson's ratio (ncomp = 3)
  double fvec[3];           // constant body force (ncomp = 3, fkind 0)
};

}  // namespace nnms
