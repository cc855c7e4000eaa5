// Internal declarations of the nnms library (host structures and the
// device-side descriptors shared by the HIP kernels and the driver).
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "devtypes.h"
#include "nnms.h"

namespace nnms {

// Error carrying an nnms_status across internal C++ code; converted to a
// status at the C ABI.
struct Error : std::runtime_error {
  nnms_status code;
  Error(nnms_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);


// ---------------------------------------------------------------------------
// Host structure of one level (built once per hierarchy).
// ---------------------------------------------------------------------------
struct HostLevel {
  // nv: unknowns (rows of the level operator); nint: interior unknowns.  With
  // ncomp unknowns per vertex (field splitting) nvert is the vertex count and
  // nv = ncomp * nvert; per-vertex arrays: xyz, tets, vptr / vitem
  int64_t nv = 0, nt = 0, nint = 0;
  int64_t nvert = 0;
  int32_t ncomp = 1;
  std::vector<double> xyz;      // nv*3
  std::vector<int32_t> tets;    // nt*4
  std::vector<uint8_t> dir;     // nv

  // CSR pattern (Dirichlet rows: diagonal only; Dirichlet columns dropped)
  std::vector<int32_t> rp, col;
  // assembly gather: for every CSR slot, its element contributions
  // encoded t*16 + a*4 + b, ordered by element id
  std::vector<int32_t> cptr, citem;
  // vertex -> incident elements (t*4 + a), ordered by element id
  std::vector<int32_t> vptr, vitem;
  // the same pattern as sliced ELL: 64-row slices stored column-major (entry
  // k of row 64s + l at sell_off[s] + 64k + l), slice width = its longest
  // row; sell_src = CSR slot of every entry, -1 for padding (value 0, column
  // = the row's last column)
  std::vector<int32_t> sell_off;  // slices + 1
  std::vector<int32_t> sell_col, sell_src;

  // Schwarz partition (nparts subdomains; 1 on the coarsest level)
  int32_t nparts = 0;
  std::vector<int32_t> owner;       // nv, -1 on Dirichlet vertices
  std::vector<int64_t> s_ptr;       // nparts+1
  std::vector<int32_t> s_idx;       // S_p ascending
  // dense-block bookkeeping
  std::vector<int32_t> nblk;        // tiles per side of every subdomain
  std::vector<int64_t> fac_off;     // element offset of every factor
  int64_t fac_elems = 0;
  std::vector<int64_t> g_off;       // offset into gidx (multiples of 64)
  int64_t g_total = 0;
  std::vector<int32_t> gidx;        // encoded global ids, padded to nblk*64
  std::vector<int32_t> ext_rs;      // start in ext_lc of every local row (s_total+1, in local order)
  std::vector<int32_t> ext_lc;      // local column of every CSR entry of every local row, -1 outside S_p
  // Local order of a dense subdomain: with owned_last, the rows the
  // subdomain does not own come first and the owned ones last (each part in
  // ascending global order), so the backward sweep of the restricted solve
  // only has to run over the owned rows; otherwise S order (ILU levels,
  // whose factorisation depends on the order).  bwd0[p] = first 64-row block
  // holding an owned row.
  bool owned_last = false;
  std::vector<int32_t> bwd0;
  // Explicit inverse panels (NNMS_APPLY_INVERSE): X_p = J_p^{-1} E_o, N x No
  // tiles in column-major tile order (tile (i, j) at x_off[p] + (j N + i)
  // tiles), No = ceil(n_o / 64); nown[p] = n_o, the owned rows, which are
  // local rows n - n_o .. n-1.  That full form only exists during the
  // numeric setup; what stays is the packed symmetric form at xs_off[p]:
  // the overlap rows X_v (Nv = ceil(n_v / 64) tile rows of 64 local rows
  // 0 .. n_v-1, zero past n_v), Nv x No tiles column-major (tile (t, b) at
  // b Nv + t), then the lower triangle of the symmetric owned block X_oo
  // (tile rows of 64 owned rows, zero past n_o) by columns: tile (a, b),
  // a >= b, at Nv No + b No - b (b - 1) / 2 + (a - b).
  bool xinv = false;
  std::vector<int32_t> nown;
  std::vector<int64_t> x_off;
  int64_t x_elems = 0;
  std::vector<int64_t> xs_off;
  int64_t xs_elems = 0;
  // the smoother's partial sums per subdomain: 2 x 64 No column parts (overlap
  // and owned rows) and 64 per pair of owned tile columns
  std::vector<int64_t> xp_off;
  int64_t xp_elems = 0;

  // transfer P_l from level l+1 to l (empty on the coarsest level)
  std::vector<int32_t> p_idx;       // nv*4
  std::vector<double> p_w;          // nv*4
  std::vector<int32_t> pt_rp, pt_col;  // rows: coarse vertices
  std::vector<double> pt_w;
  // P_l^T in the sliced ELL layout (same rules as the operator's)
  std::vector<int32_t> pts_off, pts_col;
  std::vector<double> pts_w;
  int64_t ncoarse = 0;
  // transfer kind; P_l as CSR over the fine vertices (Dirichlet rows empty,
  // Dirichlet coarse columns dropped) for both kinds
  int32_t transfer = NNMS_TRANSFER_BARYCENTRIC;
  int32_t mls_restrict = 0;  // pt_* hold the fine-to-coarse MLS operator, not P^T
  std::vector<int32_t> p_rp, p_col;
  std::vector<double> p_val;
  // MLS only: -P_l in the sliced ELL layout (the prolongation's launch)
  std::vector<int32_t> pn_off, pn_col;
  std::vector<double> pn_w;

  // subdomain solver of the smoother; with ILU, the pattern of every
  // subdomain in local numbering, rows concatenated in S order
  int32_t subsolver = NNMS_SUBSOLVER_LU;
  int32_t ilu_fill = 0;
  int32_t ilu_lanes = 4;             // lanes per row of the ILU kernels
  std::vector<int32_t> ilu_rp;       // s_total+1, entry index of every row's first entry
  std::vector<int32_t> ilu_col;      // local column, ascending within a row
  std::vector<int32_t> ilu_asrc;     // CSR slot of A for every entry, -1 for fill
  std::vector<int32_t> ilu_dpos;     // entry index of every row's diagonal
  std::vector<int32_t> ilu_gid;      // global id, >= 0 owned, -g-2 overlap
  std::vector<int32_t> ilu_fperm, ilu_bperm;  // local rows by forward / backward level
  std::vector<int32_t> ilu_fmeta, ilu_bmeta;  // 4 per schedule position (see build_ilu)
  std::vector<int32_t> ilu_flev, ilu_blev;    // per subdomain: level boundaries (nlev+1) into its perm
  std::vector<int64_t> ilu_flev_off, ilu_blev_off;  // nparts+1: start of every subdomain's boundaries
};

struct HostHierarchy {
  int L = 0;
  nnms_setup_opts opts{};
  std::vector<HostLevel> lev;
};

// host setup steps
void build_pattern(HostLevel& lv);
// sliced ELL layout of a CSR matrix with nrows rows: 64-row slices stored
// column-major, slice width = its longest row; src = CSR slot of every
// entry, -1 for padding
void build_sell_layout(const std::vector<int32_t>& rp, const std::vector<int32_t>& col, int64_t nrows,
                       std::vector<int32_t>& off, std::vector<int32_t>& scol, std::vector<int32_t>& src);
void build_sell(HostLevel& lv);
// the column-sorted slices of a CSR matrix (layout with CSORT_SLOT_BITS):
// key, each slice's smallest column, the CSR position of every sorted entry
// and the most entries in one slice; false (and empty arrays) when a slice
// has more entries or spans more columns than a key holds
bool build_csort_layout(const std::vector<int32_t>& rp, const std::vector<int32_t>& col, int64_t nrows,
                        std::vector<int32_t>& key, std::vector<int32_t>& base, std::vector<int32_t>& src,
                        int32_t& cap);
void build_partition(HostLevel& lv, int nparts, int overlap, bool direct);
// dense-factor bookkeeping of the partition (called by build_partition)
void build_blocks(HostLevel& lv);
// field splitting: carries a vertex-level level (pattern, partition,
// transfer to the next level) to K unknowns per vertex
void expand_fields(HostLevel& lv, int K);
void build_transfer(HostLevel& fine, const HostLevel& coarse);
// moving-least-squares transfer (Section 3.2), initial scale alpha times the
// mean coarse edge length; with mls_restrict the restriction is the MLS
// interpolation from the fine to the coarse nodes, else P^T
// clip_parts > 0: every neighbourhood clipped to the overlapping subdomain of
// the target's processor, both levels split into clip_parts subdomains by
// coordinate bisection with `overlap` layers, a subdomain's nodes being those
// of the elements that touch it
void build_transfer_mls(HostLevel& fine, const HostLevel& coarse, double alpha, bool mls_restrict, int clip_parts = 0,
                        int overlap = 1);
// the owned sets and overlapping sets of a partition (build_partition without
// the factor bookkeeping), and a clipping partition: the owner of every
// vertex and the node set (vertices of the elements touching the overlapping
// set) of every part
void partition_sets(HostLevel& lv, int nparts, int overlap, bool direct);
void clip_partition(const HostLevel& lv, int nparts, int overlap, std::vector<int32_t>& owner,
                    std::vector<std::vector<uint8_t>>& nodes);
double mean_edge_length(const HostLevel& lv);
// ILU(fill) pattern and level schedules of every subdomain (after the partition)
void build_ilu(HostLevel& lv, int fill);
int default_nparts(int64_t nv);

}  // namespace nnms

struct nnms_mesh {
  int64_t nv = 0, nt = 0;
  std::vector<double> xyz;
  std::vector<int32_t> tets;
  std::vector<uint8_t> dir;
};
