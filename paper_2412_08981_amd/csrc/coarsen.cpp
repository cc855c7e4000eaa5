// Geometry-preserving mesh coarsening (Algorithm 1 of the paper, Section
// 3.1), host side.  Every round takes a maximal independent set S of the
// interior vertices of the current mesh (Luby's parallel rounds: a vertex
// joins when its priority is below that of every undecided neighbour) and
// removes each vertex of S by contracting it onto one of its neighbours,
// which re-meshes the cavity left by the vertex's star as the cone from
// that neighbour over the cavity's surface (the edge-contraction method the
// paper builds on; its CPAFT mesher is only cited).  Boundary (Dirichlet)
// vertices are never removed, so the boundary surface stays as it was.
//
// Choices the paper leaves open, fixed here: priority(v) =
// splitmix64(seed + 2^40 round + v), ties by id; of the neighbours u
// (ascending id) the one whose new elements have the largest smallest
// quality q = sqrt(2) 6V / l_rms^3 is taken, and a vertex without a
// neighbour reaching q > 0.02 stays; vertices keep their positions; the
// output numbers the surviving vertices in ascending old id and keeps the
// elements in their old order.  Stars of independent vertices are
// disjoint, so the contractions of one round do not interact.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "nnms_internal.h"

namespace nnms {
namespace {

constexpr double QMIN = 0.02;

uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double det6(const double* p0, const double* p1, const double* p2, const double* p3) {
  const double a[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
  const double b[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
  const double c[3] = {p3[0] - p0[0], p3[1] - p0[1], p3[2] - p0[2]};
  return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) + a[2] * (b[0] * c[1] - b[1] * c[0]);
}

double quality(const double* p0, const double* p1, const double* p2, const double* p3) {
  const double* p[4] = {p0, p1, p2, p3};
  double s = 0.0;
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j) {
      const double dx = p[i][0] - p[j][0], dy = p[i][1] - p[j][1], dz = p[i][2] - p[j][2];
      s += dx * dx + dy * dy + dz * dz;
    }
  const double lr = std::sqrt(s / 6.0);
  return std::sqrt(2.0) * det6(p0, p1, p2, p3) / (lr * lr * lr);
}

}  // namespace

// the coarsening rounds on (xyz, tets, dir); returns the number of removed
// vertices and the coarse mesh in out_*
int64_t coarsen_mesh(const std::vector<double>& xyz, const std::vector<int32_t>& tets_in,
                     const std::vector<uint8_t>& dir, int rounds, uint64_t seed, std::vector<double>& out_xyz,
                     std::vector<int32_t>& out_tets, std::vector<uint8_t>& out_dir) {
  const int64_t nv = int64_t(dir.size()), nt = int64_t(tets_in.size() / 4);
  std::vector<int32_t> T(tets_in);
  std::vector<uint8_t> tdead(nt, 0), alive(nv, 1);
  int64_t removed = 0;
  std::vector<std::vector<int32_t>> nb(nv);
  for (int rnd = 0; rnd < rounds; ++rnd) {
    // vertex graph of the current mesh
    for (auto& v : nb) v.clear();
    for (int64_t e = 0; e < nt; ++e) {
      if (tdead[e]) continue;
      const int32_t* t = &T[e * 4];
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
          if (i != j) nb[t[i]].push_back(t[j]);
    }
    for (auto& v : nb) {
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
    }
    // Luby's rounds with fixed priorities (the greedy MIS in priority order)
    std::vector<uint64_t> key(nv, 0);
    std::vector<int8_t> state(nv, -1);  // -1 not a candidate, 0 undecided, 1 in S, 2 out
    int64_t undecided = 0;
    for (int64_t v = 0; v < nv; ++v)
      if (alive[v] && !dir[v]) {
        state[v] = 0, ++undecided;
        key[v] = splitmix64(seed + (uint64_t(rnd) << 40) + uint64_t(v));
      }
    auto less = [&](int64_t a, int64_t b) { return key[a] < key[b] || (key[a] == key[b] && a < b); };
    std::vector<int32_t> joins;
    while (undecided > 0) {
      joins.clear();
      for (int64_t v = 0; v < nv; ++v) {
        if (state[v] != 0) continue;
        bool minimal = true;
        for (int32_t w : nb[v])
          if (state[w] == 0 && less(w, v)) {
            minimal = false;
            break;
          }
        if (minimal) joins.push_back(int32_t(v));
      }
      for (int32_t v : joins) state[v] = 1, --undecided;
      for (int32_t v : joins)
        for (int32_t w : nb[v])
          if (state[w] == 0) state[w] = 2, --undecided;
    }
    std::vector<int32_t> S;
    for (int64_t v = 0; v < nv; ++v)
      if (state[v] == 1) S.push_back(int32_t(v));
    if (S.empty()) break;
    // stars (elements around each vertex of S, ascending)
    std::vector<int32_t> sidx(nv, -1);
    for (size_t k = 0; k < S.size(); ++k) sidx[S[k]] = int32_t(k);
    std::vector<std::vector<int32_t>> star(S.size());
    for (int64_t e = 0; e < nt; ++e) {
      if (tdead[e]) continue;
      for (int i = 0; i < 4; ++i)
        if (sidx[T[e * 4 + i]] >= 0) star[sidx[T[e * 4 + i]]].push_back(int32_t(e));
    }
    for (size_t k = 0; k < S.size(); ++k) {
      const int32_t v = S[k];
      int32_t best_u = -1;
      double best_q = QMIN;
      for (int32_t u : nb[v]) {
        double qmin = INFINITY;
        for (int32_t e : star[k]) {
          const int32_t* t = &T[size_t(e) * 4];
          if (t[0] == u || t[1] == u || t[2] == u || t[3] == u) continue;
          int32_t n[4];
          for (int i = 0; i < 4; ++i) n[i] = t[i] == v ? u : t[i];
          qmin = std::min(qmin, quality(&xyz[size_t(n[0]) * 3], &xyz[size_t(n[1]) * 3], &xyz[size_t(n[2]) * 3],
                                        &xyz[size_t(n[3]) * 3]));
        }
        if (qmin > best_q) best_u = u, best_q = qmin;
      }
      if (best_u < 0) continue;
      for (int32_t e : star[k]) {
        int32_t* t = &T[size_t(e) * 4];
        if (t[0] == best_u || t[1] == best_u || t[2] == best_u || t[3] == best_u) {
          tdead[e] = 1;
        } else {
          for (int i = 0; i < 4; ++i)
            if (t[i] == v) t[i] = best_u;
        }
      }
      alive[v] = 0;
      ++removed;
    }
  }
  std::vector<int32_t> nid(nv, -1);
  int32_t m = 0;
  out_xyz.clear(), out_dir.clear(), out_tets.clear();
  for (int64_t v = 0; v < nv; ++v)
    if (alive[v]) {
      nid[v] = m++;
      out_xyz.insert(out_xyz.end(), &xyz[size_t(v) * 3], &xyz[size_t(v) * 3] + 3);
      out_dir.push_back(dir[v]);
    }
  for (int64_t e = 0; e < nt; ++e)
    if (!tdead[e])
      for (int i = 0; i < 4; ++i) out_tets.push_back(nid[T[e * 4 + i]]);
  return removed;
}

}  // namespace nnms

extern "C" nnms_status nnms_mesh_coarsen(const nnms_mesh* fine, int32_t rounds, uint64_t seed, nnms_mesh** out,
                                         int64_t* removed) {
  using namespace nnms;
  try {
    if (!fine || !out || rounds < 0) throw Error(NNMS_ERR_INVALID_ARG, "bad coarsening arguments");
    *out = nullptr;
    std::unique_ptr<nnms_mesh> m(new nnms_mesh());
    const int64_t r = coarsen_mesh(fine->xyz, fine->tets, fine->dir, rounds, seed, m->xyz, m->tets, m->dir);
    m->nv = int64_t(m->dir.size());
    m->nt = int64_t(m->tets.size() / 4);
    if (removed) *removed = r;
    *out = m.release();
    return NNMS_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host out of memory");
    return NNMS_ERR_OUT_OF_MEMORY;
  }
}

extern "C" nnms_status nnms_mesh_read(const nnms_mesh* m, int64_t* nv, int64_t* nt, double* xyz, int32_t* tets,
                                      uint8_t* dirichlet) {
  if (!m) {
    nnms::set_last_error("null mesh");
    return NNMS_ERR_INVALID_ARG;
  }
  if (nv) *nv = m->nv;
  if (nt) *nt = m->nt;
  if (xyz) std::memcpy(xyz, m->xyz.data(), m->xyz.size() * sizeof(double));
  if (tets) std::memcpy(tets, m->tets.data(), m->tets.size() * sizeof(int32_t));
  if (dirichlet) std::memcpy(dirichlet, m->dir.data(), m->dir.size());
  return NNMS_OK;
}
