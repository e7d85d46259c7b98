// H(div) space on 2D meshes, host side (see hdiv.hpp).
#include "hdiv.hpp"

#include <cmath>

#include "refelem.hpp"

namespace dghdiv {

using dgref::real;

static real legendre01(int l, real s) {  // sqrt(2l+1) P_l(2s-1)
  const real x = 2 * s - 1;
  real p0 = 1, p1 = x;
  if (l == 0) return 1;
  for (int n = 1; n < l; ++n) {
    const real p2 = ((2 * n + 1) * x * p1 - n * p0) / (n + 1);
    p0 = p1;
    p1 = p2;
  }
  return std::sqrt((real)(2 * l + 1)) * p1;
}

// first-kind Nedelec N_{k-1} basis at (x, y): fills out[r][2]
static void nedelec(int k, real x, real y, std::vector<real>& out) {
  out.clear();
  auto mono = [](real x, real y, int a, int b) {
    real v = 1;
    for (int i = 0; i < a; ++i) v *= x;
    for (int i = 0; i < b; ++i) v *= y;
    return v;
  };
  for (int deg = 0; deg <= k - 2; ++deg)
    for (int a = deg; a >= 0; --a) {
      const real m = mono(x, y, a, deg - a);
      out.push_back(m); out.push_back(0);
      out.push_back(0); out.push_back(m);
    }
  for (int a = k - 2; a >= 0; --a) {
    const real m = mono(x, y, a, k - 2 - a);
    out.push_back(-y * m); out.push_back(x * m);
  }
}

void reference_dual(int k, std::vector<double>& table) {
  const int np = dgref::n_basis(2, k), nd = 2 * np;
  std::vector<real> G((size_t)nd * nd, 0);  // G[j][n], n = a np + m
  std::vector<real> sp, sw, vp, vw, phi(np);
  dgref::facet_rule<real>(2, k + 2, sp, sw);
  dgref::collapsed_rule<real>(2, k + 2, vp, vw);
  const real V[3][2] = {{0, 0}, {1, 0}, {0, 1}};
  int row = 0;
  for (int f = 0; f < 3; ++f) {
    int a0 = -1, b0 = -1;
    for (int v = 0; v < 3; ++v)
      if (v != f) (a0 < 0 ? a0 : b0) = v;
    const real tx = V[b0][0] - V[a0][0], ty = V[b0][1] - V[a0][1];
    const real len = std::sqrt(tx * tx + ty * ty);
    real nx = ty / len, ny = -tx / len;
    if (nx * (V[f][0] - V[a0][0]) + ny * (V[f][1] - V[a0][1]) > 0) { nx = -nx; ny = -ny; }
    for (int l = 0; l <= k; ++l, ++row)
      for (size_t q = 0; q < sw.size(); ++q) {
        const real s = sp[q];
        const real xi[2] = {V[a0][0] + s * tx, V[a0][1] + s * ty};
        dgref::eval_basis_t<real>(2, k, xi, phi.data(), nullptr);
        const real c = len * sw[q] * legendre01(l, s);
        for (int m = 0; m < np; ++m) {
          G[(size_t)row * nd + m] += c * nx * phi[m];
          G[(size_t)row * nd + np + m] += c * ny * phi[m];
        }
      }
  }
  std::vector<real> psi;
  const int nint = k * k - 1;
  for (size_t q = 0; q < vw.size(); ++q) {
    const real* xi = &vp[2 * q];
    dgref::eval_basis_t<real>(2, k, xi, phi.data(), nullptr);
    nedelec(k, xi[0], xi[1], psi);
    for (int r = 0; r < nint; ++r)
      for (int m = 0; m < np; ++m) {
        G[(size_t)(row + r) * nd + m] += vw[q] * psi[2 * r] * phi[m];
        G[(size_t)(row + r) * nd + np + m] += vw[q] * psi[2 * r + 1] * phi[m];
      }
  }
  // C = G^-1 by Gauss-Jordan elimination with partial pivoting (long double)
  std::vector<real> A = G, Cm((size_t)nd * nd, 0);
  for (int i = 0; i < nd; ++i) Cm[(size_t)i * nd + i] = 1;
  for (int c = 0; c < nd; ++c) {
    int p = c;
    for (int r = c + 1; r < nd; ++r)
      if (std::fabs(A[(size_t)r * nd + c]) > std::fabs(A[(size_t)p * nd + c])) p = r;
    if (p != c)
      for (int j = 0; j < nd; ++j) {
        std::swap(A[(size_t)p * nd + j], A[(size_t)c * nd + j]);
        std::swap(Cm[(size_t)p * nd + j], Cm[(size_t)c * nd + j]);
      }
    const real d = A[(size_t)c * nd + c];
    for (int j = 0; j < nd; ++j) { A[(size_t)c * nd + j] /= d; Cm[(size_t)c * nd + j] /= d; }
    for (int r = 0; r < nd; ++r) {
      if (r == c) continue;
      const real f = A[(size_t)r * nd + c];
      if (f == 0) continue;
      for (int j = 0; j < nd; ++j) {
        A[(size_t)r * nd + j] -= f * A[(size_t)c * nd + j];
        Cm[(size_t)r * nd + j] -= f * Cm[(size_t)c * nd + j];
      }
    }
  }
  // Cm = G^-1: row n (DG basis index), column j (dof); table [j][a][m]
  table.assign((size_t)nd * nd, 0.0);
  for (int j = 0; j < nd; ++j)
    for (int n = 0; n < nd; ++n) table[(size_t)j * nd + n] = (double)Cm[(size_t)n * nd + j];
}

int build(const dgmesh::Host& H, Host& o, std::string& err) {
  if (H.dim != 2) { err = "the H(div) transfer is built for 2D meshes"; return -4; }
  if (H.k < 1) { err = "the H(div) transfer needs k >= 1"; return -1; }
  o = Host();
  o.k = H.k;
  o.np = H.np;
  o.ndof = 2 * H.np;
  o.nint = H.k * H.k - 1;
  const int64_t E = H.E;
  o.elem_facet.assign((size_t)E * 3, 0);
  std::vector<int64_t> fid((size_t)E * 3, -1);
  for (int64_t t = 0; t < E; ++t)
    for (int f = 0; f < 3; ++f) {
      const int32_t nb = H.nbr[t * 3 + f];
      if (nb < 0 || t < nb) {
        fid[t * 3 + f] = o.nfacet++;
        o.facet_elem.push_back(t * 3 + f);
        o.facet_elem.push_back(-1);
      }
    }
  for (int64_t t = 0; t < E; ++t)
    for (int f = 0; f < 3; ++f) {
      const int32_t nb = H.nbr[t * 3 + f];
      if (nb >= 0 && t > nb) {
        const int64_t id = fid[(size_t)nb * 3 + H.nbr_facet[t * 3 + f]];
        fid[t * 3 + f] = id;
        o.facet_elem[2 * id + 1] = t * 3 + f;
      }
    }
  for (int64_t t = 0; t < E; ++t) {
    const double* ji = &H.jinv[(size_t)t * 4];
    const bool neg = ji[0] * ji[3] - ji[1] * ji[2] < 0;  // sign(det J) = sign(det J^-1)
    for (int f = 0; f < 3; ++f) {
      const int32_t nb = H.nbr[t * 3 + f];
      const bool owner = nb < 0 || t < nb;
      int cv[3];
      dgmesh::canonical_vertices(2, f, H.perm_own[t * 3 + f], cv);
      const int asc0 = f == 0 ? 1 : 0;  // first of the facet's ascending local vertices
      const bool rev = cv[0] != asc0;
      const bool sneg = neg != !owner;   // s_f = sign(det J) * (owner ? 1 : -1)
      const int64_t id = fid[t * 3 + f];
      if (id < 0 || id >= (int64_t(1) << 29)) { err = "facet numbering"; return -6; }
      o.elem_facet[t * 3 + f] = (int32_t)(id << 2) | (sneg ? 2 : 0) | (rev ? 1 : 0);
    }
  }
  o.N = o.nfacet * (H.k + 1) + E * o.nint;
  reference_dual(H.k, o.table);
  return 0;
}

}  // namespace dghdiv
