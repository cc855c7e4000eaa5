// Numeric assembly of the P1 system on the device (Section 2.1: the
// Jacobian and right-hand side of the discrete residual; for
// -div(kappa grad u) = f these are the stiffness matrix and load vector).
//
//   k_elem:   per tetrahedron, kappa at the centroid, |T| and the 4x4
//             element matrix kappa_T |T| grad(lambda_a).grad(lambda_b)
//   k_elem_elastic: linear elasticity (Section 4.2: sigma = lambda tr(eps) I
//             + 2 mu eps, Lame coefficients from Young's modulus E = kappa_T
//             and Poisson's ratio nu), three unknowns per vertex: the 12x12
//             element matrix of the bilinear form 2 mu eps(u):eps(v) +
//             lambda div u div v for u = phi_b e_d, v = phi_a e_c,
//             |T| (mu delta_cd g_a.g_b + mu g_a[d] g_b[c] + lambda g_a[c] g_b[d])
//             with g = grad lambda, at row 3a + c and column 3b + d
//   k_gather: per CSR row, every entry sums its element contributions in
//             element order (deterministic, no atomics); Dirichlet rows
//             get a unit diagonal; the load vector sums over the incident
//             elements of interior vertices: f |T| / 4 for a constant f,
//             f_T |T| / 4 for an f constant per element, and the element
//             mass matrix |T| (1 + delta_ab) / 20 applied to P1 nodal values
//             (the exact integral of the interpolant against phi_i).
#include "devcommon.h"
#include "kernels.h"

namespace nnms {

// vertices, barycentric gradients, volume and kappa of tetrahedron t
struct TetGeom {
  double g[4][3];
  double vol, kT;
};

__device__ __forceinline__ TetGeom tet_geom(const AsmDesc& a, const KappaDev& kap, int64_t t) {
  TetGeom G;
  const int4 v = ((const int4*)a.tets)[t];
  double x[4][3];
  const int vid[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) x[k][c] = a.xyz[int64_t(vid[k]) * 3 + c];
  double J[3][3];  // columns are the edges x_{c+1} - x_0
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int r = 0; r < 3; ++r) J[r][c] = x[c + 1][r] - x[0][r];
  const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  const double id = 1.0 / det;
  double(&g)[4][3] = G.g;  // g[a] = grad lambda_a; rows of J^{-1} for a = 1..3
  g[1][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
  g[1][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
  g[1][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
  g[2][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
  g[2][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
  g[2][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
  g[3][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
  g[3][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
  g[3][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
#pragma unroll
  for (int c = 0; c < 3; ++c) g[0][c] = -(g[1][c] + g[2][c] + g[3][c]);
  const double vol = fabs(det) / 6.0;
  double kT = kap.value;
  if (kap.kind == 2) {
    kT = a.kappa_tet[t];
  } else if (kap.kind == 1) {
    double cx = 0.25 * (x[0][0] + x[1][0] + x[2][0] + x[3][0]);
    double cy = 0.25 * (x[0][1] + x[1][1] + x[2][1] + x[3][1]);
    double cz = 0.25 * (x[0][2] + x[1][2] + x[2][2] + x[3][2]);
    double s = 0.0;
    for (int k = 0; k < kap.nc; ++k) {
      double dx = cx - kap.c[3 * k], dy = cy - kap.c[3 * k + 1], dz = cz - kap.c[3 * k + 2];
      s += kap.mu[k] * exp(-(dx * dx + dy * dy + dz * dz) / kap.width);
    }
    kT = exp(s);
  }
  G.vol = vol, G.kT = kT;
  return G;
}

__global__ __launch_bounds__(256) void k_elem(AsmDesc a, KappaDev kap) {
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (t >= a.nt) return;
  const TetGeom G = tet_geom(a, kap, t);
  const double sc = G.kT * G.vol;
  double* e = a.elem + t * 16;
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      e[p * 4 + q] = sc * (G.g[p][0] * G.g[q][0] + G.g[p][1] * G.g[q][1] + G.g[p][2] * G.g[q][2]);
  a.elem[a.nt * 16 + t] = G.vol;
}

__global__ __launch_bounds__(256) void k_elem_elastic(AsmDesc a, KappaDev kap) {
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (t >= a.nt) return;
  const TetGeom G = tet_geom(a, kap, t);
  const double mu = G.kT / (2.0 * (1.0 + a.nu));
  const double lam = G.kT * a.nu / ((1.0 + a.nu) * (1.0 - 2.0 * a.nu));
  double* e = a.elem + t * 144;
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double gg = G.g[p][0] * G.g[q][0] + G.g[p][1] * G.g[q][1] + G.g[p][2] * G.g[q][2];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d)
          e[(3 * p + c) * 12 + 3 * q + d] =
              G.vol * ((c == d ? mu * gg : 0.0) + mu * G.g[p][d] * G.g[q][c] + lam * G.g[p][c] * G.g[q][d]);
    }
  a.elem[a.nt * 144 + t] = G.vol;
}

__global__ __launch_bounds__(256) void k_gather(AsmDesc a, double f) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= a.nv) return;
  const int s = a.rp[i], e = a.rp[i + 1];
  if (a.dmask[i]) {
    a.val64[s] = 1.0;  // the only entry of a Dirichlet row is its diagonal
    if (a.val32) a.val32[s] = 1.0f;
    if (a.b) a.b[i] = 0.0;
    return;
  }
  for (int q = s; q < e; ++q) {
    double acc = 0.0;
    for (int c = a.cptr[q]; c < a.cptr[q + 1]; ++c) acc += a.elem[a.citem[c]];
    a.val64[q] = acc;
    if (a.val32) a.val32[q] = float(acc);
  }
  if (a.b) {
    // row i is component k of vertex v (K unknowns per vertex)
    const int K = a.ncomp;
    const int64_t v = i / K;
    const int k = int(i - v * K);
    const double* vol = a.elem + a.nt * 16 * K * K;
    double acc = 0.0;
    if (a.fkind == 0) {
      for (int c = a.vptr[v]; c < a.vptr[v + 1]; ++c) acc += vol[a.vitem[c] >> 2];
      a.b[i] = (K == 1 ? f : a.fvec[k]) * acc * 0.25;
    } else if (a.fkind == 1) {
      for (int c = a.vptr[v]; c < a.vptr[v + 1]; ++c) {
        const int t = a.vitem[c] >> 2;
        acc += a.fval[int64_t(t) * K + k] * vol[t];
      }
      a.b[i] = acc * 0.25;
    } else {
      const double fi = a.fval[i];
      for (int c = a.vptr[v]; c < a.vptr[v + 1]; ++c) {
        const int t = a.vitem[c] >> 2;
        const int4 w = ((const int4*)a.tets)[t];
        const double s4 = (a.fval[int64_t(w.x) * K + k] + a.fval[int64_t(w.y) * K + k]) +
                          (a.fval[int64_t(w.z) * K + k] + a.fval[int64_t(w.w) * K + k]);
        acc += vol[t] * (s4 + fi);
      }
      a.b[i] = acc / 20.0;
    }
  }
}

hipError_t launch_assemble(const AsmDesc& a, const KappaDev& k, double f, hipStream_t s) {
  if (a.ncomp != 1 && a.ncomp != 3) return hipErrorInvalidValue;
  if (a.nt > 0) {
    if (a.ncomp == 3)
      hipLaunchKernelGGL(k_elem_elastic, dim3(int((a.nt + 255) / 256)), dim3(256), 0, s, a, k);
    else
      hipLaunchKernelGGL(k_elem, dim3(int((a.nt + 255) / 256)), dim3(256), 0, s, a, k);
  }
  if (a.nv > 0) hipLaunchKernelGGL(k_gather, dim3(int((a.nv + 255) / 256)), dim3(256), 0, s, a, f);
  return hipGetLastError();
}

}  // namespace nnms
