// Host-side structure setup of a mesh hierarchy: mesh validation, the CSR
// pattern and its assembly maps, the Schwarz partition with overlap, and
// the barycentric point-location transfer between non-nested levels.
// Everything here depends on the meshes only and is reused across
// parameters (Section 2.1 of the paper: the mesh perspective is a reusable,
// parameter-independent object).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <set>

#include "nnms_internal.h"

namespace nnms {

int default_nparts(int64_t nv) {
  double q = double(nv) / 1500.0;
  if (q < 2.0) return 2;
  int e = int(std::floor(std::log2(q)));
  return std::max(2, 1 << e);
}

// ---------------------------------------------------------------------------
// CSR pattern of the vertex graph and the element->entry gather maps.
// Interior rows keep interior columns; Dirichlet rows keep the diagonal
// (the symmetric elimination of homogeneous Dirichlet data).
// ---------------------------------------------------------------------------
void build_pattern(HostLevel& lv) {
  const int64_t nv = lv.nv, nt = lv.nt;
  // vertex -> (element, local index), elements ascending
  lv.vptr.assign(nv + 1, 0);
  for (int64_t t = 0; t < nt; ++t)
    for (int a = 0; a < 4; ++a) lv.vptr[lv.tets[t * 4 + a] + 1]++;
  for (int64_t i = 0; i < nv; ++i) lv.vptr[i + 1] += lv.vptr[i];
  lv.vitem.resize(lv.vptr[nv]);
  {
    std::vector<int32_t> fill(lv.vptr.begin(), lv.vptr.end() - 1);
    for (int64_t t = 0; t < nt; ++t)
      for (int a = 0; a < 4; ++a) lv.vitem[fill[lv.tets[t * 4 + a]]++] = int32_t(t * 4 + a);
  }
  // rows
  lv.rp.assign(nv + 1, 0);
  std::vector<std::vector<int32_t>> rows(0);
  lv.col.clear();
  lv.col.reserve(nv * 15);
  std::vector<int32_t> nb;
  for (int64_t i = 0; i < nv; ++i) {
    nb.clear();
    if (lv.dir[i]) {
      nb.push_back(int32_t(i));
    } else {
      for (int32_t e = lv.vptr[i]; e < lv.vptr[i + 1]; ++e) {
        int32_t t = lv.vitem[e] >> 2;
        for (int b = 0; b < 4; ++b) {
          int32_t j = lv.tets[t * 4 + b];
          if (!lv.dir[j]) nb.push_back(j);
        }
      }
      std::sort(nb.begin(), nb.end());
      nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    }
    lv.col.insert(lv.col.end(), nb.begin(), nb.end());
    lv.rp[i + 1] = int32_t(lv.col.size());
  }
  if (lv.col.size() > size_t(INT32_MAX)) throw Error(NNMS_ERR_INVALID_ARG, "mesh too large for int32 CSR");
  // element contributions per CSR entry (interior rows only)
  const int64_t nnz = lv.col.size();
  lv.cptr.assign(nnz + 1, 0);
  auto find_slot = [&](int32_t i, int32_t j) -> int32_t {
    const int32_t* b = lv.col.data() + lv.rp[i];
    const int32_t* e = lv.col.data() + lv.rp[i + 1];
    const int32_t* p = std::lower_bound(b, e, j);
    return int32_t(p - lv.col.data());
  };
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int32_t> fill;
    if (pass == 1) {
      for (int64_t s = 0; s < nnz; ++s) lv.cptr[s + 1] += lv.cptr[s];
      lv.citem.resize(lv.cptr[nnz]);
      fill.assign(lv.cptr.begin(), lv.cptr.end() - 1);
    }
    for (int64_t i = 0; i < nv; ++i) {
      if (lv.dir[i]) continue;
      for (int32_t e = lv.vptr[i]; e < lv.vptr[i + 1]; ++e) {
        int32_t t = lv.vitem[e] >> 2, a = lv.vitem[e] & 3;
        for (int b = 0; b < 4; ++b) {
          int32_t j = lv.tets[t * 4 + b];
          if (lv.dir[j]) continue;
          int32_t s = find_slot(int32_t(i), j);
          if (pass == 0)
            lv.cptr[s + 1]++;
          else
            lv.citem[fill[s]++] = t * 16 + a * 4 + b;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Recursive coordinate bisection of the interior vertices (axis = depth mod
// 3, order by (coordinate, vertex id), the lower floor(n/2) to the lower
// part), then `overlap` layers of 1-ring growth restricted to interior
// vertices (Section 2.2: subdomains extended by delta layers of elements).
// ---------------------------------------------------------------------------
static void rcb(const HostLevel& lv, std::vector<int32_t>& ids, int nparts, int depth,
                std::vector<std::vector<int32_t>>& out) {
  if (nparts <= 1) {
    std::sort(ids.begin(), ids.end());
    out.push_back(ids);
    return;
  }
  const int ax = depth % 3;
  std::sort(ids.begin(), ids.end(), [&](int32_t a, int32_t b) {
    double xa = lv.xyz[size_t(a) * 3 + ax], xb = lv.xyz[size_t(b) * 3 + ax];
    if (xa != xb) return xa < xb;
    return a < b;
  });
  size_t half = ids.size() / 2;
  std::vector<int32_t> lo(ids.begin(), ids.begin() + half), hi(ids.begin() + half, ids.end());
  rcb(lv, lo, nparts / 2, depth + 1, out);
  rcb(lv, hi, nparts / 2, depth + 1, out);
}

void build_sell_layout(const std::vector<int32_t>& rp, const std::vector<int32_t>& col, int64_t nrows,
                       std::vector<int32_t>& off, std::vector<int32_t>& scol, std::vector<int32_t>& src) {
  const int64_t ns = (nrows + 63) / 64;
  off.assign(ns + 1, 0);
  for (int64_t sl = 0; sl < ns; ++sl) {
    int32_t w = 0;
    for (int64_t i = sl * 64; i < std::min(nrows, sl * 64 + 64); ++i) w = std::max(w, rp[i + 1] - rp[i]);
    if (int64_t(off[sl]) + int64_t(w) * 64 > INT32_MAX) throw Error(NNMS_ERR_INVALID_ARG, "level too large for 32-bit indices");
    off[sl + 1] = off[sl] + w * 64;
  }
  scol.assign(off[ns], 0);
  src.assign(off[ns], -1);
  for (int64_t sl = 0; sl < ns; ++sl) {
    const int32_t w = (off[sl + 1] - off[sl]) / 64;
    for (int l = 0; l < 64; ++l) {
      const int64_t i = sl * 64 + l;
      for (int32_t k = 0; k < w; ++k) {
        const int64_t e = off[sl] + int64_t(k) * 64 + l;
        if (i < nrows && rp[i] + k < rp[i + 1]) {
          scol[e] = col[rp[i] + k];
          src[e] = rp[i] + k;
        } else {
          // padding: value 0 times an entry of x the row already reads (the
          // same cache line), or x[0] for a row without entries
          scol[e] = (i < nrows && rp[i + 1] > rp[i]) ? col[rp[i + 1] - 1] : 0;
        }
      }
    }
  }
}

bool build_csort_layout(const std::vector<int32_t>& rp, const std::vector<int32_t>& col, int64_t nrows,
                        std::vector<int32_t>& key, std::vector<int32_t>& base, std::vector<int32_t>& src,
                        int32_t& cap) {
  const int64_t ns = (nrows + 63) / 64;
  key.assign(col.size(), 0);
  src.assign(col.size(), 0);
  base.assign(ns, 0);
  cap = 0;
  std::vector<int32_t> ord;
  for (int64_t sl = 0; sl < ns; ++sl) {
    const int32_t e0 = rp[sl * 64], e1 = rp[std::min(nrows, sl * 64 + 64)];
    const int32_t ne = e1 - e0;
    if (ne == 0) continue;
    int32_t lo = col[e0], hi = col[e0];
    for (int32_t e = e0; e < e1; ++e) lo = std::min(lo, col[e]), hi = std::max(hi, col[e]);
    if (ne > (1 << CSORT_SLOT_BITS) || int64_t(hi) - lo >= CSORT_MAX_SPAN) {
      key.clear(), src.clear(), base.clear(), cap = 0;
      return false;
    }
    base[sl] = lo;
    cap = std::max(cap, ne);
    ord.resize(ne);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return col[e0 + a] < col[e0 + b]; });
    for (int32_t k = 0; k < ne; ++k) {
      key[e0 + k] = ((col[e0 + ord[k]] - lo) << CSORT_SLOT_BITS) | ord[k];
      src[e0 + k] = e0 + ord[k];
    }
  }
  return true;
}

void build_sell(HostLevel& lv) { build_sell_layout(lv.rp, lv.col, lv.nv, lv.sell_off, lv.sell_col, lv.sell_src); }

void build_partition(HostLevel& lv, int nparts, int overlap, bool direct) {
  partition_sets(lv, nparts, overlap, direct);
  build_blocks(lv);
}

// owned sets by coordinate bisection and their overlapping extension (no
// factor bookkeeping)
void partition_sets(HostLevel& lv, int nparts, int overlap, bool direct) {
  const int64_t nv = lv.nv;
  std::vector<int32_t> interior;
  for (int64_t i = 0; i < nv; ++i)
    if (!lv.dir[i]) interior.push_back(int32_t(i));
  lv.nint = int64_t(interior.size());
  std::vector<std::vector<int32_t>> owned;
  if (direct) {
    nparts = 1;
    owned.push_back(interior);
    overlap = 0;
  } else {
    if (nparts < 1 || (nparts & (nparts - 1))) throw Error(NNMS_ERR_INVALID_ARG, "nparts must be a power of two");
    rcb(lv, interior, nparts, 0, owned);
  }
  lv.nparts = nparts;
  lv.owner.assign(nv, -1);
  for (int p = 0; p < nparts; ++p)
    for (int32_t v : owned[p]) lv.owner[v] = p;
  lv.s_ptr.assign(nparts + 1, 0);
  lv.s_idx.clear();
  std::vector<uint8_t> mark(nv), nxt(nv);
  for (int p = 0; p < nparts; ++p) {
    std::fill(mark.begin(), mark.end(), 0);
    for (int32_t v : owned[p]) mark[v] = 1;
    std::vector<int32_t> cur = owned[p];
    for (int d = 0; d < overlap; ++d) {
      std::vector<int32_t> grow;
      for (int32_t v : cur)
        for (int32_t e = lv.rp[v]; e < lv.rp[v + 1]; ++e) {
          int32_t c = lv.col[e];
          if (!mark[c]) {
            mark[c] = 1;
            grow.push_back(c);
          }
        }
      cur.insert(cur.end(), grow.begin(), grow.end());
    }
    std::sort(cur.begin(), cur.end());
    lv.s_idx.insert(lv.s_idx.end(), cur.begin(), cur.end());
    lv.s_ptr[p + 1] = int64_t(lv.s_idx.size());
  }
}

void clip_partition(const HostLevel& lv, int nparts, int overlap, std::vector<int32_t>& owner,
                    std::vector<std::vector<uint8_t>>& nodes) {
  HostLevel t;
  t.nv = lv.nv, t.nt = lv.nt;
  t.xyz = lv.xyz, t.tets = lv.tets, t.dir = lv.dir, t.rp = lv.rp, t.col = lv.col;
  partition_sets(t, nparts, overlap, false);
  owner = t.owner;
  nodes.assign(nparts, std::vector<uint8_t>(lv.nv, 0));
  std::vector<uint8_t> inset(lv.nv);
  for (int p = 0; p < nparts; ++p) {
    std::fill(inset.begin(), inset.end(), 0);
    for (int64_t k = t.s_ptr[p]; k < t.s_ptr[p + 1]; ++k) inset[t.s_idx[k]] = 1;
    for (int64_t e = 0; e < lv.nt; ++e) {
      const int32_t* v = &lv.tets[e * 4];
      if (inset[v[0]] | inset[v[1]] | inset[v[2]] | inset[v[3]])
        for (int a = 0; a < 4; ++a) nodes[p][v[a]] = 1;
    }
  }
}

// Dense-factor bookkeeping of the level's subdomains (tile counts, factor
// offsets, padded index maps with ownership, extraction map of every local
// row's CSR entries), from the partition and the level's CSR.  With
// lv.owned_last the local order puts the overlap rows first: the restricted
// solve R^0_p J_p^{-1} needs x_o = inv(U_oo) y_o of the owned rows only
// (U is upper triangular), so its backward sweep stops at block bwd0[p].
void build_blocks(HostLevel& lv) {
  const int nparts = lv.nparts;
  lv.nblk.assign(nparts, 0);
  lv.fac_off.assign(nparts + 1, 0);
  lv.g_off.assign(nparts + 1, 0);
  for (int p = 0; p < nparts; ++p) {
    int64_t n = lv.s_ptr[p + 1] - lv.s_ptr[p];
    int32_t N = int32_t((n + TILE - 1) / TILE);
    lv.nblk[p] = N;
    // N*N tiles (L, U, inv(U_ii)), N tiles inv(L_ii), 2 floor(N/2) pair coupling tiles
    lv.fac_off[p + 1] = lv.fac_off[p] + (int64_t(N) * N + N + 2 * (N / 2)) * TILE_ELEMS;
    lv.g_off[p + 1] = lv.g_off[p] + int64_t(N) * TILE;
  }
  lv.fac_elems = lv.fac_off[nparts];
  lv.g_total = lv.g_off[nparts];
  lv.gidx.assign(lv.g_total, -1);
  lv.ext_rs.assign(lv.s_idx.size() + 1, 0);
  lv.ext_lc.clear();
  lv.bwd0.assign(nparts, 0);
  lv.nown.assign(nparts, 0);
  lv.x_off.assign(nparts + 1, 0);
  lv.xs_off.assign(nparts + 1, 0);
  lv.xp_off.assign(nparts + 1, 0);
  std::vector<int32_t> ord, loc;  // local row -> position in S, and back
  for (int p = 0; p < nparts; ++p) {
    const int32_t* S = lv.s_idx.data() + lv.s_ptr[p];
    int64_t n = lv.s_ptr[p + 1] - lv.s_ptr[p];
    ord.clear();
    if (lv.owned_last) {
      for (int32_t k = 0; k < int32_t(n); ++k)
        if (lv.owner[S[k]] != p) ord.push_back(k);
      lv.bwd0[p] = int32_t(ord.size() / TILE);
      for (int32_t k = 0; k < int32_t(n); ++k)
        if (lv.owner[S[k]] == p) ord.push_back(k);
    } else {
      for (int32_t k = 0; k < int32_t(n); ++k) ord.push_back(k);
    }
    loc.assign(n, 0);
    for (int32_t k = 0; k < int32_t(n); ++k) loc[ord[k]] = k;
    for (int32_t k = 0; k < int32_t(n); ++k) lv.nown[p] += lv.owner[S[k]] == p;
    if (lv.xinv && !lv.owned_last && lv.nown[p] != int32_t(n))
      throw Error(NNMS_ERR_INVALID_ARG, "inverse panels need the owned rows last");
    const int64_t No = (lv.nown[p] + TILE - 1) / TILE;
    lv.x_off[p + 1] = lv.x_off[p] + (lv.xinv ? int64_t(lv.nblk[p]) * No * TILE_ELEMS : 0);
    const int64_t Nv = (n - lv.nown[p] + TILE - 1) / TILE;
    lv.xs_off[p + 1] = lv.xs_off[p] + (lv.xinv ? (Nv * No + No * (No + 1) / 2) * TILE_ELEMS : 0);
    lv.xp_off[p + 1] = lv.xp_off[p] + (lv.xinv ? 128 * No + 64 * (No * (No - 1) / 2) : 0);
    for (int64_t k = 0; k < n; ++k) {
      int32_t g = S[ord[k]];
      lv.gidx[lv.g_off[p] + k] = (lv.owner[g] == p) ? g : (-g - 2);
      lv.ext_rs[lv.s_ptr[p] + k] = int32_t(lv.ext_lc.size());
      for (int32_t e = lv.rp[g]; e < lv.rp[g + 1]; ++e) {
        int32_t c = lv.col[e];
        const int32_t* q = std::lower_bound(S, S + n, c);
        lv.ext_lc.push_back((q != S + n && *q == c) ? loc[q - S] : -1);
      }
    }
  }
  if (lv.ext_lc.size() > size_t(INT32_MAX)) throw Error(NNMS_ERR_INVALID_ARG, "subdomains too large");
  lv.ext_rs[lv.s_idx.size()] = int32_t(lv.ext_lc.size());
  lv.x_elems = lv.x_off[nparts];
  lv.xs_elems = lv.xs_off[nparts];
  lv.xp_elems = lv.xp_off[nparts];
}

// ---------------------------------------------------------------------------
// Field splitting (Section 3.2, equations field-split and interpolation
// split).  A level of a problem with K unknowns per vertex (the three
// displacement components of linear elasticity, numbered K v + c) is built
// from the vertex-level structure: every field has one unknown per vertex, so
// the pattern, the partition and the transfer of each field are those of
// the vertices.  The pattern couples every component of a vertex with every
// component of its neighbours (K x K blocks; a Dirichlet vertex keeps K
// identity rows), the element gather map addresses the 4K x 4K element
// matrices (row K a + c, column K b + d), a subdomain holds all components
// of its vertices, and the interpolation sum_f R_f^T P R~_f keeps every
// field apart: unknown K v + c takes P's row v applied to component c.
// Vertex-level arrays that assembly reads (coordinates, elements, the
// vertex -> element map) stay per vertex.
// ---------------------------------------------------------------------------
namespace {
// CSR of A (x) I_K: row K r + c holds the entries (K col + c, val) of row r
void kron_csr(const std::vector<int32_t>& rp, const std::vector<int32_t>& col, const std::vector<double>& val,
              int64_t nrows, int K, std::vector<int32_t>& orp, std::vector<int32_t>& ocol, std::vector<double>& oval) {
  orp.assign(nrows * K + 1, 0);
  ocol.clear(), oval.clear();
  ocol.reserve(col.size() * K), oval.reserve(col.size() * K);
  for (int64_t r = 0; r < nrows; ++r)
    for (int c = 0; c < K; ++c) {
      for (int32_t e = rp[r]; e < rp[r + 1]; ++e) {
        ocol.push_back(K * col[e] + c);
        oval.push_back(val[e]);
      }
      orp[r * K + c + 1] = int32_t(ocol.size());
    }
}
}  // namespace

void expand_fields(HostLevel& lv, int K) {
  lv.ncomp = K;
  lv.nvert = lv.nv;
  if (K == 1) return;
  const int64_t nv = lv.nv;
  if (nv * K > INT32_MAX / 2) throw Error(NNMS_ERR_INVALID_ARG, "level too large for 32-bit unknown ids");
  const std::vector<uint8_t> vdir = lv.dir;
  // pattern and element gather map
  std::vector<int32_t> rp(nv * K + 1, 0), col, cptr(1, 0), citem;
  col.reserve(lv.col.size() * K * K);
  citem.reserve(lv.citem.size() * K * K);
  for (int64_t i = 0; i < nv; ++i)
    for (int c = 0; c < K; ++c) {
      if (vdir[i]) {
        col.push_back(int32_t(K * i + c));
        cptr.push_back(int32_t(citem.size()));
      } else {
        for (int32_t s = lv.rp[i]; s < lv.rp[i + 1]; ++s)
          for (int d = 0; d < K; ++d) {
            col.push_back(K * lv.col[s] + d);
            for (int32_t q = lv.cptr[s]; q < lv.cptr[s + 1]; ++q) {
              const int32_t it = lv.citem[q], t = it >> 4, a = (it >> 2) & 3, b = it & 3;
              citem.push_back(t * (16 * K * K) + (K * a + c) * (4 * K) + K * b + d);
            }
            cptr.push_back(int32_t(citem.size()));
          }
      }
      rp[i * K + c + 1] = int32_t(col.size());
    }
  if (int64_t(lv.nt) * 16 * K * K > INT32_MAX) throw Error(NNMS_ERR_INVALID_ARG, "mesh too large for the element map");
  lv.rp.swap(rp), lv.col.swap(col), lv.cptr.swap(cptr), lv.citem.swap(citem);
  lv.dir.assign(nv * K, 0);
  for (int64_t i = 0; i < nv; ++i)
    for (int c = 0; c < K; ++c) lv.dir[i * K + c] = vdir[i];
  lv.nv = nv * K;
  lv.nint *= K;
  build_sell(lv);
  // partition: every component of a vertex with the vertex
  std::vector<int32_t> owner(nv * K);
  for (int64_t i = 0; i < nv; ++i)
    for (int c = 0; c < K; ++c) owner[i * K + c] = lv.owner[i];
  lv.owner.swap(owner);
  std::vector<int32_t> sidx;
  sidx.reserve(lv.s_idx.size() * K);
  for (int32_t v : lv.s_idx)
    for (int c = 0; c < K; ++c) sidx.push_back(K * v + c);
  lv.s_idx.swap(sidx);
  for (auto& p : lv.s_ptr) p *= K;
  build_blocks(lv);
  // transfers of every field (smoothed levels only)
  if (lv.p_rp.empty()) return;
  const int64_t nc = lv.ncoarse;
  if (!lv.p_idx.empty()) {
    std::vector<int32_t> idx(nv * K * 4);
    std::vector<double> w(nv * K * 4);
    for (int64_t v = 0; v < nv; ++v)
      for (int c = 0; c < K; ++c)
        for (int a = 0; a < 4; ++a) {
          idx[(v * K + c) * 4 + a] = K * lv.p_idx[v * 4 + a] + c;
          w[(v * K + c) * 4 + a] = lv.p_w[v * 4 + a];
        }
    lv.p_idx.swap(idx), lv.p_w.swap(w);
  }
  std::vector<int32_t> orp, ocol;
  std::vector<double> oval;
  kron_csr(lv.p_rp, lv.p_col, lv.p_val, nv, K, orp, ocol, oval);
  lv.p_rp.swap(orp), lv.p_col.swap(ocol), lv.p_val.swap(oval);
  kron_csr(lv.pt_rp, lv.pt_col, lv.pt_w, nc, K, orp, ocol, oval);
  lv.pt_rp.swap(orp), lv.pt_col.swap(ocol), lv.pt_w.swap(oval);
  lv.ncoarse = nc * K;
  std::vector<int32_t> src;
  build_sell_layout(lv.pt_rp, lv.pt_col, lv.ncoarse, lv.pts_off, lv.pts_col, src);
  lv.pts_w.assign(src.size(), 0.0);
  for (size_t e = 0; e < src.size(); ++e)
    if (src[e] >= 0) lv.pts_w[e] = lv.pt_w[src[e]];
  if (lv.transfer == NNMS_TRANSFER_MLS) {
    build_sell_layout(lv.p_rp, lv.p_col, lv.nv, lv.pn_off, lv.pn_col, src);
    lv.pn_w.assign(src.size(), 0.0);
    for (size_t e = 0; e < src.size(); ++e)
      if (src[e] >= 0) lv.pn_w[e] = -lv.p_val[src[e]];
  }
}

// ---------------------------------------------------------------------------
// Barycentric transfer: every interior fine vertex is located in a coarse
// tetrahedron (lowest id with min(lambda) >= -1e-12; otherwise the largest
// min(lambda), rejected below -1e-8) through a uniform bucket grid.
// ---------------------------------------------------------------------------
void build_transfer(HostLevel& fine, const HostLevel& coarse) {
  const double ACCEPT = -1e-12, REJECT = -1e-8;
  const int64_t nt = coarse.nt;
  std::vector<std::array<double, 12>> aff(nt);  // x0 (3) and J^{-1} (9, row-major)
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t v = 0; v < coarse.nv; ++v)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], coarse.xyz[v * 3 + a]);
      hi[a] = std::max(hi[a], coarse.xyz[v * 3 + a]);
    }
  for (int64_t t = 0; t < nt; ++t) {
    const double* x0 = &coarse.xyz[size_t(coarse.tets[t * 4]) * 3];
    double J[3][3];
    for (int c = 0; c < 3; ++c) {
      const double* xc = &coarse.xyz[size_t(coarse.tets[t * 4 + c + 1]) * 3];
      for (int r = 0; r < 3; ++r) J[r][c] = xc[r] - x0[r];
    }
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    double id = 1.0 / det;
    auto& A = aff[t];
    A[0] = x0[0], A[1] = x0[1], A[2] = x0[2];
    double* M = &A[3];
    M[0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
    M[1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    M[2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    M[3] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
    M[4] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    M[5] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    M[6] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
    M[7] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    M[8] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
  }
  int nb = std::max(1, int(std::lround(std::cbrt(double(nt)))));
  double cell[3], span = 0;
  for (int a = 0; a < 3; ++a) {
    cell[a] = std::max((hi[a] - lo[a]) / nb, 1e-300);
    span = std::max(span, hi[a] - lo[a]);
  }
  const double pad = 1e-9 * span;
  auto bucket = [&](double x, int a) {
    int b = int(std::floor((x - lo[a]) / cell[a]));
    return std::min(std::max(b, 0), nb - 1);
  };
  const int64_t nbk = int64_t(nb) * nb * nb;
  std::vector<int32_t> bptr(nbk + 1, 0), bitem;
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int32_t> fill;
    if (pass == 1) {
      for (int64_t b = 0; b < nbk; ++b) bptr[b + 1] += bptr[b];
      bitem.resize(bptr[nbk]);
      fill.assign(bptr.begin(), bptr.end() - 1);
    }
    for (int64_t t = 0; t < nt; ++t) {
      int bl[3], bh[3];
      for (int a = 0; a < 3; ++a) {
        double mn = 1e300, mx = -1e300;
        for (int k = 0; k < 4; ++k) {
          double x = coarse.xyz[size_t(coarse.tets[t * 4 + k]) * 3 + a];
          mn = std::min(mn, x), mx = std::max(mx, x);
        }
        bl[a] = bucket(mn - pad, a), bh[a] = bucket(mx + pad, a);
      }
      for (int k = bl[2]; k <= bh[2]; ++k)
        for (int j = bl[1]; j <= bh[1]; ++j)
          for (int i = bl[0]; i <= bh[0]; ++i) {
            int64_t b = i + int64_t(nb) * (j + int64_t(nb) * k);
            if (pass == 0)
              bptr[b + 1]++;
            else
              bitem[fill[b]++] = int32_t(t);  // t ascending within a bucket
          }
    }
  }
  const int64_t nf = fine.nv;
  fine.p_idx.assign(nf * 4, 0);
  fine.p_w.assign(nf * 4, 0.0);
  fine.ncoarse = coarse.nv;
  for (int64_t v = 0; v < nf; ++v) {
    if (fine.dir[v]) continue;
    const double* x = &fine.xyz[v * 3];
    int64_t b = bucket(x[0], 0) + int64_t(nb) * (bucket(x[1], 1) + int64_t(nb) * bucket(x[2], 2));
    int32_t best_t = -1;
    double best = -1e300, best_l[4] = {0, 0, 0, 0};
    for (int32_t e = bptr[b]; e < bptr[b + 1]; ++e) {
      int32_t t = bitem[e];
      const auto& A = aff[t];
      double d0 = x[0] - A[0], d1 = x[1] - A[1], d2 = x[2] - A[2];
      double l[4];
      l[1] = A[3] * d0 + A[4] * d1 + A[5] * d2;
      l[2] = A[6] * d0 + A[7] * d1 + A[8] * d2;
      l[3] = A[9] * d0 + A[10] * d1 + A[11] * d2;
      l[0] = 1.0 - l[1] - l[2] - l[3];
      double mn = std::min(std::min(l[0], l[1]), std::min(l[2], l[3]));
      if (mn >= ACCEPT) {
        best_t = t, best = 1e300;
        std::memcpy(best_l, l, sizeof l);
        break;
      }
      if (mn > best) {
        best_t = t, best = mn;
        std::memcpy(best_l, l, sizeof l);
      }
    }
    if (best_t < 0 || best < REJECT)
      throw Error(NNMS_ERR_POINT_LOCATION, "fine vertex " + std::to_string(v) + " lies outside the coarser mesh");
    for (int a = 0; a < 4; ++a) {
      int32_t c = coarse.tets[best_t * 4 + a];
      fine.p_idx[v * 4 + a] = c;
      fine.p_w[v * 4 + a] = coarse.dir[c] ? 0.0 : best_l[a];
    }
  }
  // explicit transpose: rows = interior coarse vertices, entries ordered by fine id
  const int64_t nc = coarse.nv;
  fine.pt_rp.assign(nc + 1, 0);
  for (int64_t v = 0; v < nf; ++v) {
    if (fine.dir[v]) continue;
    for (int a = 0; a < 4; ++a) {
      int32_t c = fine.p_idx[v * 4 + a];
      if (!coarse.dir[c]) fine.pt_rp[c + 1]++;
    }
  }
  for (int64_t c = 0; c < nc; ++c) fine.pt_rp[c + 1] += fine.pt_rp[c];
  fine.pt_col.resize(fine.pt_rp[nc]);
  fine.pt_w.resize(fine.pt_rp[nc]);
  std::vector<int32_t> fill(fine.pt_rp.begin(), fine.pt_rp.end() - 1);
  for (int64_t v = 0; v < nf; ++v) {
    if (fine.dir[v]) continue;
    for (int a = 0; a < 4; ++a) {
      int32_t c = fine.p_idx[v * 4 + a];
      if (coarse.dir[c]) continue;
      fine.pt_col[fill[c]] = int32_t(v);
      fine.pt_w[fill[c]++] = fine.p_w[v * 4 + a];
    }
  }
  std::vector<int32_t> src;
  build_sell_layout(fine.pt_rp, fine.pt_col, nc, fine.pts_off, fine.pts_col, src);
  fine.pts_w.assign(src.size(), 0.0);
  for (size_t e = 0; e < src.size(); ++e)
    if (src[e] >= 0) fine.pts_w[e] = fine.pt_w[src[e]];
  // the same operator as CSR over the fine vertices (inspection)
  fine.p_rp.assign(nf + 1, 0);
  fine.p_col.clear();
  fine.p_val.clear();
  for (int64_t v = 0; v < nf; ++v) {
    if (!fine.dir[v])
      for (int a = 0; a < 4; ++a) {
        int32_t c = fine.p_idx[v * 4 + a];
        if (coarse.dir[c]) continue;
        fine.p_col.push_back(c);
        fine.p_val.push_back(fine.p_w[v * 4 + a]);
      }
    fine.p_rp[v + 1] = int32_t(fine.p_col.size());
  }
  fine.transfer = NNMS_TRANSFER_BARYCENTRIC;
}

// ---------------------------------------------------------------------------
// ILU(k) structure of every subdomain matrix A[S_p, S_p], natural ordering
// (the subdomain's rows in ascending global id).  Level of fill: entries of
// A have level 0; eliminating entry (i, k) gives every (i, j), j > k, of
// row k's upper part the level lev(i, k) + lev(k, j) + 1, and entries of
// level <= fill are kept.  Schedules: the forward level of a row is one more
// than the largest among its lower columns (rows of one level depend only on
// earlier levels in the factorisation and in the forward solve); the
// backward level likewise over the upper columns.
// ---------------------------------------------------------------------------
void build_ilu(HostLevel& lv, int fill) {
  if (fill < 0) throw Error(NNMS_ERR_INVALID_ARG, "ILU fill level must be >= 0");
  const int np = lv.nparts;
  const int64_t ns = int64_t(lv.s_idx.size());
  lv.ilu_fill = fill;
  lv.ilu_rp.assign(ns + 1, 0);
  lv.ilu_col.clear();
  lv.ilu_asrc.clear();
  lv.ilu_dpos.assign(ns, 0);
  lv.ilu_fperm.assign(ns, 0);
  lv.ilu_bperm.assign(ns, 0);
  lv.ilu_gid.assign(ns, 0);
  lv.ilu_flev.clear();
  lv.ilu_blev.clear();
  lv.ilu_flev_off.assign(np + 1, 0);
  lv.ilu_blev_off.assign(np + 1, 0);
  std::vector<int32_t> lev_of, slot_of;
  for (int p = 0; p < np; ++p) {
    const int64_t base = lv.s_ptr[p];
    const int32_t n = int32_t(lv.s_ptr[p + 1] - base);
    const int32_t* S = lv.s_idx.data() + base;
    lev_of.assign(n, INT32_MAX);
    slot_of.assign(n, -1);
    std::vector<std::vector<int32_t>> rcol(n), rlev(n);
    std::set<int32_t> row;
    for (int32_t i = 0; i < n; ++i) {
      const int32_t g = S[i];
      lv.ilu_gid[base + i] = (lv.owner[g] == p) ? g : (-g - 2);
      row.clear();
      const int32_t e0 = lv.ext_rs[base + i], e1 = lv.ext_rs[base + i + 1];
      for (int32_t e = e0; e < e1; ++e) {
        const int32_t c = lv.ext_lc[e];
        if (c < 0) continue;
        lev_of[c] = 0;
        slot_of[c] = lv.rp[g] + (e - e0);
        row.insert(c);
      }
      if (lev_of[i] != 0) throw Error(NNMS_ERR_INVALID_ARG, "subdomain matrix without a diagonal entry");
      for (auto it = row.begin(); it != row.end() && *it < i; ++it) {
        const int32_t k = *it, lik = lev_of[k];
        for (size_t t = 0; t < rcol[k].size(); ++t) {
          const int32_t j = rcol[k][t];
          if (j <= k) continue;
          const int32_t nl = lik + rlev[k][t] + 1;
          if (nl <= fill && nl < lev_of[j]) {
            if (lev_of[j] == INT32_MAX) row.insert(j);
            lev_of[j] = nl;
          }
        }
      }
      lv.ilu_rp[base + i] = int32_t(lv.ilu_col.size());
      for (int32_t c : row) {
        rcol[i].push_back(c);
        rlev[i].push_back(lev_of[c]);
        if (c == i) lv.ilu_dpos[base + i] = int32_t(lv.ilu_col.size());
        lv.ilu_col.push_back(c);
        lv.ilu_asrc.push_back(slot_of[c]);
        lev_of[c] = INT32_MAX;
        slot_of[c] = -1;
      }
      if (lv.ilu_col.size() > size_t(INT32_MAX / 2)) throw Error(NNMS_ERR_INVALID_ARG, "ILU pattern too large");
    }
    // level schedules (counting sort by level, rows ascending within a level)
    std::vector<int32_t> fl(n, 0), bl(n, 0);
    int32_t nfl = 0, nbl = 0;
    for (int32_t i = 0; i < n; ++i) {
      for (int32_t c : rcol[i])
        if (c < i) fl[i] = std::max(fl[i], fl[c] + 1);
      nfl = std::max(nfl, fl[i] + 1);
    }
    for (int32_t i = n - 1; i >= 0; --i) {
      for (int32_t c : rcol[i])
        if (c > i) bl[i] = std::max(bl[i], bl[c] + 1);
      nbl = std::max(nbl, bl[i] + 1);
    }
    auto schedule = [&](const std::vector<int32_t>& lvl, int32_t nl, int32_t* perm, std::vector<int32_t>& offs) {
      std::vector<int32_t> cnt(nl + 1, 0);
      for (int32_t i = 0; i < n; ++i) cnt[lvl[i] + 1]++;
      for (int32_t k = 0; k < nl; ++k) cnt[k + 1] += cnt[k];
      offs.insert(offs.end(), cnt.begin(), cnt.end());
      for (int32_t i = 0; i < n; ++i) perm[cnt[lvl[i]]++] = i;
    };
    if (n > 0) {
      schedule(fl, nfl, lv.ilu_fperm.data() + base, lv.ilu_flev);
      schedule(bl, nbl, lv.ilu_bperm.data() + base, lv.ilu_blev);
    }
    lv.ilu_flev_off[p + 1] = int64_t(lv.ilu_flev.size());
    lv.ilu_blev_off[p + 1] = int64_t(lv.ilu_blev.size());
  }
  lv.ilu_rp[ns] = int32_t(lv.ilu_col.size());
  // per schedule position, the row and its entry ranges, so that a kernel
  // reaches a row's entries with one dependent load instead of three:
  // forward {row, first, diagonal, end}, backward {row, diagonal + 1, end,
  // diagonal} (entry indices global, rows local)
  lv.ilu_fmeta.assign(size_t(ns) * 4, 0);
  lv.ilu_bmeta.assign(size_t(ns) * 4, 0);
  for (int p = 0; p < np; ++p) {
    const int64_t base = lv.s_ptr[p], n = lv.s_ptr[p + 1] - base;
    for (int64_t q = 0; q < n; ++q) {
      const int32_t i = lv.ilu_fperm[base + q], r = int32_t(base) + i;
      int32_t* m = &lv.ilu_fmeta[size_t(base + q) * 4];
      m[0] = i, m[1] = lv.ilu_rp[r], m[2] = lv.ilu_dpos[r], m[3] = lv.ilu_rp[r + 1];
      const int32_t j = lv.ilu_bperm[base + q], t = int32_t(base) + j;
      int32_t* w = &lv.ilu_bmeta[size_t(base + q) * 4];
      w[0] = j, w[1] = lv.ilu_dpos[t] + 1, w[2] = lv.ilu_rp[t + 1], w[3] = lv.ilu_dpos[t];
    }
  }
  // lanes per row of the device kernels: a group stages at most 4 entries
  // per lane in the factorisation and takes at most 2 per lane of a row's
  // lower or upper part in the triangular solves
  int32_t maxlen = 0, maxhalf = 0;
  for (int64_t r = 0; r < ns; ++r) {
    const int32_t a = lv.ilu_rp[r], b = lv.ilu_rp[r + 1], d = lv.ilu_dpos[r];
    maxlen = std::max(maxlen, b - a);
    maxhalf = std::max(maxhalf, std::max(d - a, b - d - 1));
  }
  int32_t lanes = 4;
  while (lanes < 32 && (4 * lanes < maxlen || 2 * lanes < maxhalf)) lanes *= 2;
  if (4 * lanes < maxlen || 2 * lanes < maxhalf)
    throw Error(NNMS_ERR_INVALID_ARG, "ILU rows too long for the device kernels (" + std::to_string(maxlen) +
                                          " entries; lower the fill level)");
  lv.ilu_lanes = lanes;
  lv.subsolver = NNMS_SUBSOLVER_ILU;
}

// ---------------------------------------------------------------------------
// Moving-least-squares transfer (Section 3.2).  The row of P_l for a fine
// vertex x* holds phi_n = q(x*)^T M^{-1} w_n q_n over the coarse vertices
// x~_n with |x~_n - x*| < rho, where
//   q(x) = [1, (x - x*) / rho]  the linear basis centred at x* and scaled by
//                               rho (the space of [1, x, y, z], so the same
//                               operator, with a well-conditioned M),
//   w_n = 1 - 6 r^2 + 8 r^3 - 3 r^4,  r = |x~_n - x*| / rho,
//   M = sum_n w_n q_n q_n^T  (the paper's P1; w_n q_n are P2's columns).
// rho starts at alpha times the mean coarse edge length and grows by 1.25
// until rank(P) = 4, decided as lambda_min > 1e-12 lambda_max of the
// unweighted Gram matrix sum_n q_n q_n^T (singular values of P in the
// centred basis above 1e-6 of the largest).  Coarse Dirichlet columns are
// dropped after the solve; fine Dirichlet rows stay empty.
// ---------------------------------------------------------------------------
namespace {

// eigenvalues of a symmetric 4x4 matrix by cyclic Jacobi rotations
void sym4_eigenvalues(double A[4][4], double ev[4]) {
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0, diag = 0;
    for (int i = 0; i < 4; ++i) {
      diag += A[i][i] * A[i][i];
      for (int j = i + 1; j < 4; ++j) off += A[i][j] * A[i][j];
    }
    if (off <= 1e-34 * diag) break;
    for (int p = 0; p < 3; ++p)
      for (int q = p + 1; q < 4; ++q) {
        if (A[p][q] == 0.0) continue;
        const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < 4; ++k) {  // columns p, q
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq, A[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 4; ++k) {  // rows p, q
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk, A[q][k] = sn * apk + c * aqk;
        }
      }
  }
  for (int i = 0; i < 4; ++i) ev[i] = A[i][i];
}

// c = M^{-1} e_0 for a symmetric positive definite 4x4 M (Cholesky)
bool spd4_solve_e0(const double M[4][4], double c[4]) {
  double L[4][4] = {};
  for (int j = 0; j < 4; ++j) {
    double d = M[j][j];
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(d > 0)) return false;
    L[j][j] = std::sqrt(d);
    for (int i = j + 1; i < 4; ++i) {
      double v = M[i][j];
      for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
      L[i][j] = v / L[j][j];
    }
  }
  double y[4];
  for (int i = 0; i < 4; ++i) {
    double v = (i == 0) ? 1.0 : 0.0;
    for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
    y[i] = v / L[i][i];
  }
  for (int i = 3; i >= 0; --i) {
    double v = y[i];
    for (int k = i + 1; k < 4; ++k) v -= L[k][i] * c[k];
    c[i] = v / L[i][i];
  }
  return true;
}

}  // namespace

double mean_edge_length(const HostLevel& lv) {
  std::vector<uint64_t> e;
  e.reserve(size_t(lv.nt) * 6);
  for (int64_t t = 0; t < lv.nt; ++t)
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b) {
        uint64_t i = uint32_t(lv.tets[t * 4 + a]), j = uint32_t(lv.tets[t * 4 + b]);
        if (i > j) std::swap(i, j);
        e.push_back((i << 32) | j);
      }
  std::sort(e.begin(), e.end());
  e.erase(std::unique(e.begin(), e.end()), e.end());
  double sum = 0;
  for (uint64_t k : e) {
    const double* x = &lv.xyz[size_t(k >> 32) * 3];
    const double* y = &lv.xyz[size_t(k & 0xffffffffu) * 3];
    sum += std::sqrt((x[0] - y[0]) * (x[0] - y[0]) + (x[1] - y[1]) * (x[1] - y[1]) + (x[2] - y[2]) * (x[2] - y[2]));
  }
  return e.empty() ? 0.0 : sum / double(e.size());
}

// The MLS operator from the nodal values of `src` to the nodes of `dst`
// (rows: dst vertices, Dirichlet rows empty, Dirichlet src columns dropped),
// scale starting at alpha times the mean edge length of src.
// clip: null, or (owner of every target vertex, source-node masks of every
// processor): the neighbourhood of a target owned by p is clipped to mask p
struct MlsClip {
  std::vector<int32_t> owner;
  std::vector<std::vector<uint8_t>> nodes;
};

static void mls_operator(const HostLevel& dst, const HostLevel& src, double alpha, std::vector<int32_t>& p_rp,
                         std::vector<int32_t>& p_col, std::vector<double>& p_val, const MlsClip* clip = nullptr) {
  if (!(alpha > 0)) throw Error(NNMS_ERR_INVALID_ARG, "MLS scale factor must be positive");
  const double rho0 = alpha * mean_edge_length(src);
  if (!(rho0 > 0)) throw Error(NNMS_ERR_INVALID_ARG, "degenerate source mesh");
  const int64_t nc = src.nv, nf = dst.nv;  // source / target vertices
  // uniform bucket grid over the source vertices, cell edge rho0
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t v = 0; v < nc; ++v)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], src.xyz[v * 3 + a]);
      hi[a] = std::max(hi[a], src.xyz[v * 3 + a]);
    }
  int nb[3];
  for (int a = 0; a < 3; ++a) nb[a] = std::max(1, std::min(1024, int(std::floor((hi[a] - lo[a]) / rho0)) + 1));
  auto cell = [&](double x, int a) {
    int b = int(std::floor((x - lo[a]) / rho0));
    return std::min(std::max(b, 0), nb[a] - 1);
  };
  const int64_t ncell = int64_t(nb[0]) * nb[1] * nb[2];
  std::vector<int32_t> cptr(ncell + 1, 0), citem(nc);
  for (int64_t v = 0; v < nc; ++v) {
    const double* x = &src.xyz[v * 3];
    cptr[cell(x[0], 0) + int64_t(nb[0]) * (cell(x[1], 1) + int64_t(nb[1]) * cell(x[2], 2)) + 1]++;
  }
  for (int64_t c = 0; c < ncell; ++c) cptr[c + 1] += cptr[c];
  {
    std::vector<int32_t> fill(cptr.begin(), cptr.end() - 1);
    for (int64_t v = 0; v < nc; ++v) {
      const double* x = &src.xyz[v * 3];
      citem[fill[cell(x[0], 0) + int64_t(nb[0]) * (cell(x[1], 1) + int64_t(nb[1]) * cell(x[2], 2))]++] = int32_t(v);
    }
  }
  p_rp.assign(nf + 1, 0);
  p_col.clear();
  p_val.clear();
  std::vector<int32_t> ids;
  std::vector<double> q, w;
  for (int64_t v = 0; v < nf; ++v) {
    p_rp[v + 1] = p_rp[v];
    if (dst.dir[v]) continue;
    const double* xs = &dst.xyz[v * 3];
    const uint8_t* allowed = clip ? clip->nodes[clip->owner[v]].data() : nullptr;
    double rho = rho0;
    bool ok = false;
    for (int grow = 0; grow < 200 && !ok; ++grow, rho *= 1.25) {
      ids.clear();
      int bl[3], bh[3];
      for (int a = 0; a < 3; ++a) bl[a] = cell(xs[a] - rho, a), bh[a] = cell(xs[a] + rho, a);
      for (int k = bl[2]; k <= bh[2]; ++k)
        for (int j = bl[1]; j <= bh[1]; ++j)
          for (int i = bl[0]; i <= bh[0]; ++i) {
            const int64_t c = i + int64_t(nb[0]) * (j + int64_t(nb[1]) * k);
            for (int32_t e = cptr[c]; e < cptr[c + 1]; ++e) {
              const double* y = &src.xyz[size_t(citem[e]) * 3];
              const double d2 = (y[0] - xs[0]) * (y[0] - xs[0]) + (y[1] - xs[1]) * (y[1] - xs[1]) +
                                (y[2] - xs[2]) * (y[2] - xs[2]);
              if (std::sqrt(d2) < rho && (!allowed || allowed[citem[e]])) ids.push_back(citem[e]);
            }
          }
      if (ids.size() < 4) continue;
      std::sort(ids.begin(), ids.end());
      const size_t m = ids.size();
      q.resize(m * 4), w.resize(m);
      double G[4][4] = {}, M[4][4] = {};
      for (size_t n = 0; n < m; ++n) {
        const double* y = &src.xyz[size_t(ids[n]) * 3];
        double* qn = &q[n * 4];
        qn[0] = 1.0;
        for (int a = 0; a < 3; ++a) qn[a + 1] = (y[a] - xs[a]) / rho;
        const double r = std::sqrt(qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
        w[n] = 1.0 + r * r * (-6.0 + r * (8.0 - 3.0 * r));
        for (int i = 0; i < 4; ++i)
          for (int j = 0; j < 4; ++j) G[i][j] += qn[i] * qn[j], M[i][j] += w[n] * qn[i] * qn[j];
      }
      double ev[4];
      sym4_eigenvalues(G, ev);
      const double emax = std::max(std::max(ev[0], ev[1]), std::max(ev[2], ev[3]));
      const double emin = std::min(std::min(ev[0], ev[1]), std::min(ev[2], ev[3]));
      if (!(emin > 1e-12 * emax)) continue;
      double c[4];
      if (!spd4_solve_e0(M, c)) continue;
      for (size_t n = 0; n < m; ++n) {
        if (src.dir[ids[n]]) continue;
        const double* qn = &q[n * 4];
        p_col.push_back(ids[n]);
        p_val.push_back(w[n] * (c[0] * qn[0] + c[1] * qn[1] + c[2] * qn[2] + c[3] * qn[3]));
      }
      p_rp[v + 1] = int32_t(p_col.size());
      ok = true;
    }
    if (!ok) throw Error(NNMS_ERR_POINT_LOCATION, "no full-rank MLS neighbourhood for vertex " + std::to_string(v));
    if (p_col.size() > size_t(INT32_MAX / 2)) throw Error(NNMS_ERR_INVALID_ARG, "MLS transfer too large");
  }
}

void build_transfer_mls(HostLevel& fine, const HostLevel& coarse, double alpha, bool mls_restrict, int clip_parts,
                        int overlap) {
  const int64_t nc = coarse.nv, nf = fine.nv;
  // clipping: every level split across the same clip_parts processors
  std::unique_ptr<MlsClip> cp, cr;
  if (clip_parts > 0) {
    MlsClip fc, cc;
    clip_partition(fine, clip_parts, overlap, fc.owner, fc.nodes);
    clip_partition(coarse, clip_parts, overlap, cc.owner, cc.nodes);
    cp.reset(new MlsClip{fc.owner, cc.nodes});  // fine targets, coarse sources
    cr.reset(new MlsClip{cc.owner, fc.nodes});  // coarse targets, fine sources
  }
  mls_operator(fine, coarse, alpha, fine.p_rp, fine.p_col, fine.p_val, cp.get());
  fine.p_idx.assign(nf * 4, 0);  // the four-entry form is not used by this transfer
  fine.p_w.assign(nf * 4, 0.0);
  fine.ncoarse = nc;
  if (mls_restrict) {
    // the paper's second interpolation: fine nodal values to the coarse
    // nodes by MLS, in place of the transpose
    mls_operator(coarse, fine, alpha, fine.pt_rp, fine.pt_col, fine.pt_w, cr.get());
  } else {
    // explicit transpose: rows = coarse vertices, entries ordered by fine id
    fine.pt_rp.assign(nc + 1, 0);
    for (int32_t c : fine.p_col) fine.pt_rp[c + 1]++;
    for (int64_t c = 0; c < nc; ++c) fine.pt_rp[c + 1] += fine.pt_rp[c];
    fine.pt_col.resize(fine.pt_rp[nc]);
    fine.pt_w.resize(fine.pt_rp[nc]);
    std::vector<int32_t> fill(fine.pt_rp.begin(), fine.pt_rp.end() - 1);
    for (int64_t v = 0; v < nf; ++v)
      for (int32_t e = fine.p_rp[v]; e < fine.p_rp[v + 1]; ++e) {
        const int32_t c = fine.p_col[e];
        fine.pt_col[fill[c]] = int32_t(v);
        fine.pt_w[fill[c]++] = fine.p_val[e];
      }
  }
  fine.mls_restrict = mls_restrict ? 1 : 0;
  std::vector<int32_t> src;
  build_sell_layout(fine.pt_rp, fine.pt_col, nc, fine.pts_off, fine.pts_col, src);
  fine.pts_w.assign(src.size(), 0.0);
  for (size_t e = 0; e < src.size(); ++e)
    if (src[e] >= 0) fine.pts_w[e] = fine.pt_w[src[e]];
  // the prolongation as sliced ELL holding -P: the residual form of the
  // sliced-ELL product, y = r - A x with r = y = z_f, adds P z_c to z_f
  build_sell_layout(fine.p_rp, fine.p_col, nf, fine.pn_off, fine.pn_col, src);
  fine.pn_w.assign(src.size(), 0.0);
  for (size_t e = 0; e < src.size(); ++e)
    if (src[e] >= 0) fine.pn_w[e] = -fine.p_val[src[e]];
  fine.transfer = NNMS_TRANSFER_MLS;
}

}  // namespace nnms

using namespace nnms;

// ---------------------------------------------------------------------------
// C ABI: meshes and host-only hierarchy inspection
// ---------------------------------------------------------------------------
extern "C" nnms_status nnms_mesh_create(int64_t nv, const double* xyz, int64_t nt, const int32_t* tets,
                                        const uint8_t* dirichlet, nnms_mesh** out) {
  try {
    if (!out || !xyz || !tets || nv < 4 || nt < 1 || nv > INT32_MAX || nt > (INT32_MAX >> 4))
      throw Error(NNMS_ERR_INVALID_ARG, "nnms_mesh_create: bad arguments");
    *out = nullptr;
    auto* m = new nnms_mesh;
    m->nv = nv, m->nt = nt;
    m->xyz.assign(xyz, xyz + nv * 3);
    m->tets.assign(tets, tets + nt * 4);
    for (int64_t k = 0; k < nt * 4; ++k)
      if (m->tets[k] < 0 || m->tets[k] >= nv) {
        delete m;
        throw Error(NNMS_ERR_BAD_MESH, "tetrahedron " + std::to_string(k / 4) + " has a vertex id out of range");
      }
    for (int64_t t = 0; t < nt; ++t) {
      const double* p[4];
      for (int a = 0; a < 4; ++a) p[a] = &m->xyz[size_t(m->tets[t * 4 + a]) * 3];
      double e[3][3];
      for (int a = 0; a < 3; ++a)
        for (int r = 0; r < 3; ++r) e[a][r] = p[a + 1][r] - p[0][r];
      double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) - e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                   e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
      if (!(det > 0)) {
        delete m;
        throw Error(NNMS_ERR_BAD_MESH, "tetrahedron " + std::to_string(t) + " has non-positive volume");
      }
    }
    m->dir.assign(nv, 0);
    if (dirichlet) {
      for (int64_t v = 0; v < nv; ++v) m->dir[v] = dirichlet[v] ? 1 : 0;
    } else {
      double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
      for (int64_t v = 0; v < nv; ++v)
        for (int a = 0; a < 3; ++a) lo[a] = std::min(lo[a], m->xyz[v * 3 + a]), hi[a] = std::max(hi[a], m->xyz[v * 3 + a]);
      for (int64_t v = 0; v < nv; ++v)
        for (int a = 0; a < 3; ++a)
          if (m->xyz[v * 3 + a] == lo[a] || m->xyz[v * 3 + a] == hi[a]) m->dir[v] = 1;
    }
    *out = m;
    return NNMS_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host out of memory");
    return NNMS_ERR_OUT_OF_MEMORY;
  }
}

extern "C" void nnms_mesh_destroy(nnms_mesh* m) { delete m; }

extern "C" nnms_status nnms_setup_opts_default(nnms_setup_opts* o) {
  if (!o) return NNMS_ERR_INVALID_ARG;
  std::memset(o, 0, sizeof *o);
  o->overlap = 1;
  o->its = 3;
  o->precision = NNMS_FP64;
  o->transfer = NNMS_TRANSFER_BARYCENTRIC;
  o->mls_alpha = 1.0;
  o->subsolver = NNMS_SUBSOLVER_LU;
  o->ilu_fill[0] = 2;  // ILU(2) on the finest level, ILU(0) on the others
  o->mls_restrict = 0;
  o->ncomp = 1;
  return NNMS_OK;
}
