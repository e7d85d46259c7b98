// H(div) space on 2D and 3D meshes, host side (see hdiv.hpp).
#include "hdiv.hpp"

#include <array>
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

static real mono(const real* x, int dim, const int* e) {
  real v = 1;
  for (int c = 0; c < dim; ++c)
    for (int i = 0; i < e[c]; ++i) v *= x[c];
  return v;
}

// exponents of the monomials of degree deg: a descending, then b descending
static std::vector<std::array<int, 3>> monomials(int dim, int deg) {
  std::vector<std::array<int, 3>> out;
  for (int a = deg; a >= 0; --a) {
    if (dim == 2) {
      out.push_back({a, deg - a, 0});
      continue;
    }
    for (int b = deg - a; b >= 0; --b) out.push_back({a, b, deg - a - b});
  }
  return out;
}

// first-kind Nedelec N_{k-1} basis at x: fills out[r][dim]
static void nedelec(int dim, int k, const real* x, std::vector<real>& out) {
  out.clear();
  for (int deg = 0; deg <= k - 2; ++deg)
    for (const auto& e : monomials(dim, deg)) {
      const real m = mono(x, dim, e.data());
      for (int i = 0; i < dim; ++i)
        for (int c = 0; c < dim; ++c) out.push_back(c == i ? m : 0);
    }
  if (k < 2) return;
  for (const auto& e : monomials(dim, k - 2)) {
    const real m = mono(x, dim, e.data());
    if (dim == 2) {
      out.push_back(-x[1] * m);
      out.push_back(x[0] * m);
      continue;
    }
    for (int i = 0; i < 3; ++i) {
      if (i == 0 && e[0] >= 1) continue;  // x ^ (e_0 x q) is a combination of the other two
      // x ^ e_i, times m
      const real r[3][3] = {{0, x[2], -x[1]}, {-x[2], 0, x[0]}, {x[1], -x[0], 0}};
      for (int c = 0; c < 3; ++c) out.push_back(r[i][c] * m);
    }
  }
}

// the orthonormal facet basis at facet parameter s (d - 1 values): q[0..nfd)
static void facet_tests(int dim, int k, const real* s, real* q) {
  if (dim == 2) {
    for (int l = 0; l <= k; ++l) q[l] = legendre01(l, s[0]);
    return;
  }
  dgref::eval_basis_t<real>(2, k, s, q, nullptr);
  const real r = 1 / std::sqrt((real)2);
  for (int l = 0; l < facet_dofs(3, k); ++l) q[l] *= r;
}

// Gauss-Jordan inverse with partial pivoting (long double), in place of a copy
static std::vector<real> inverse(const std::vector<real>& G, int nd) {
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
  return Cm;
}

void reference_dual(int dim, int k, std::vector<double>& table) {
  const int np = dgref::n_basis(dim, k), nd = dim * np, nfd = facet_dofs(dim, k);
  std::vector<real> G((size_t)nd * nd, 0);  // G[j][n], n = a np + m
  std::vector<real> sp, sw, vp, vw, phi(np), q(nfd);
  dgref::facet_rule<real>(dim, k + 2, sp, sw);
  dgref::collapsed_rule<real>(dim, k + 2, vp, vw);
  real V[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  int row = 0;
  const int nsp = dim - 1;  // facet parameters per point
  for (int f = 0; f <= dim; ++f) {
    int vs[3], c = 0;
    for (int v = 0; v <= dim; ++v)
      if (v != f) vs[c++] = v;
    real e[2][3];
    for (int a = 0; a < dim - 1; ++a)
      for (int x = 0; x < dim; ++x) e[a][x] = V[vs[a + 1]][x] - V[vs[0]][x];
    real n[3], meas;
    if (dim == 2) {
      meas = std::sqrt(e[0][0] * e[0][0] + e[0][1] * e[0][1]);
      n[0] = e[0][1] / meas; n[1] = -e[0][0] / meas;
    } else {
      const real cx = e[0][1] * e[1][2] - e[0][2] * e[1][1];
      const real cy = e[0][2] * e[1][0] - e[0][0] * e[1][2];
      const real cz = e[0][0] * e[1][1] - e[0][1] * e[1][0];
      const real len = std::sqrt(cx * cx + cy * cy + cz * cz);
      meas = len / 2;
      n[0] = cx / len; n[1] = cy / len; n[2] = cz / len;
    }
    real dot = 0;
    for (int x = 0; x < dim; ++x) dot += n[x] * (V[f][x] - V[vs[0]][x]);
    if (dot > 0)
      for (int x = 0; x < dim; ++x) n[x] = -n[x];
    for (size_t qp = 0; qp < sw.size(); ++qp) {
      const real* s = &sp[qp * nsp];
      real xi[3];
      for (int x = 0; x < dim; ++x) {
        xi[x] = V[vs[0]][x];
        for (int a = 0; a < dim - 1; ++a) xi[x] += s[a] * e[a][x];
      }
      dgref::eval_basis_t<real>(dim, k, xi, phi.data(), nullptr);
      facet_tests(dim, k, s, q.data());
      for (int l = 0; l < nfd; ++l) {
        const real cq = meas * sw[qp] * q[l];
        for (int a = 0; a < dim; ++a)
          for (int m = 0; m < np; ++m) G[(size_t)(row + l) * nd + a * np + m] += cq * n[a] * phi[m];
      }
    }
    row += nfd;
  }
  std::vector<real> psi;
  const int nint = nd - (dim + 1) * nfd;
  for (size_t qp = 0; qp < vw.size(); ++qp) {
    const real* xi = &vp[dim * qp];
    dgref::eval_basis_t<real>(dim, k, xi, phi.data(), nullptr);
    nedelec(dim, k, xi, psi);
    for (int r = 0; r < nint; ++r)
      for (int a = 0; a < dim; ++a)
        for (int m = 0; m < np; ++m)
          G[(size_t)(row + r) * nd + a * np + m] += vw[qp] * psi[(size_t)r * dim + a] * phi[m];
  }
  const std::vector<real> Cm = inverse(G, nd);  // G^-1: row n (DG basis index), column j (dof)
  table.assign((size_t)nd * nd, 0.0);
  for (int j = 0; j < nd; ++j)
    for (int n = 0; n < nd; ++n) table[(size_t)j * nd + n] = (double)Cm[(size_t)n * nd + j];
}

void orientation_tables(int k, std::vector<double>& table) {
  const int nfd = facet_dofs(3, k);
  std::vector<real> sp, sw, ql(nfd), qc(nfd);
  dgref::facet_rule<real>(3, k + 2, sp, sw);
  table.assign((size_t)6 * nfd * nfd, 0.0);
  for (int p = 0; p < 6; ++p) {
    int pos[3];  // canonical vertex j is the local-ascending vertex pos[j] (facet 3: 0, 1, 2)
    dgmesh::canonical_vertices(3, 3, p, pos);
    std::vector<real> Q((size_t)nfd * nfd, 0);
    for (size_t qp = 0; qp < sw.size(); ++qp) {
      const real lc[3] = {1 - sp[2 * qp] - sp[2 * qp + 1], sp[2 * qp], sp[2 * qp + 1]};
      real ll[3];
      for (int j = 0; j < 3; ++j) ll[pos[j]] = lc[j];
      facet_tests(3, k, &ll[1], ql.data());
      facet_tests(3, k, &sp[2 * qp], qc.data());
      for (int l = 0; l < nfd; ++l)
        for (int i = 0; i < nfd; ++i) Q[(size_t)l * nfd + i] += sw[qp] * ql[l] * qc[i];
    }
    for (size_t i = 0; i < Q.size(); ++i) table[(size_t)p * nfd * nfd + i] = (double)Q[i];
  }
}

int build(const dgmesh::Host& H, Host& o, std::string& err) {
  if (H.dim != 2 && H.dim != 3) { err = "the H(div) transfer needs dim 2 or 3"; return -4; }
  if (H.k < 1) { err = "the H(div) transfer needs k >= 1"; return -1; }
  const int d = H.dim, nf = d + 1;
  o = Host();
  o.dim = d;
  o.k = H.k;
  o.np = H.np;
  o.ndof = d * H.np;
  o.nfd = facet_dofs(d, H.k);
  o.nint = o.ndof - nf * o.nfd;
  const int64_t E = H.E;
  o.elem_facet.assign((size_t)E * nf, 0);
  std::vector<int64_t> fid((size_t)E * nf, -1);
  for (int64_t t = 0; t < E; ++t)
    for (int f = 0; f < nf; ++f) {
      const int32_t nb = H.nbr[t * nf + f];
      if (nb < 0 || t < nb) {
        fid[t * nf + f] = o.nfacet++;
        o.facet_elem.push_back(t * nf + f);
        o.facet_elem.push_back(-1);
      }
    }
  for (int64_t t = 0; t < E; ++t)
    for (int f = 0; f < nf; ++f) {
      const int32_t nb = H.nbr[t * nf + f];
      if (nb >= 0 && t > nb) {
        const int64_t id = fid[(size_t)nb * nf + H.nbr_facet[t * nf + f]];
        fid[t * nf + f] = id;
        o.facet_elem[2 * id + 1] = t * nf + f;
      }
    }
  const int shift = d == 2 ? 2 : 4;
  for (int64_t t = 0; t < E; ++t) {
    const double* ji = &H.jinv[(size_t)t * d * d];
    // sign(det J) = sign(det J^-1)
    const double det = d == 2 ? ji[0] * ji[3] - ji[1] * ji[2]
                              : ji[0] * (ji[4] * ji[8] - ji[5] * ji[7]) -
                                    ji[1] * (ji[3] * ji[8] - ji[5] * ji[6]) +
                                    ji[2] * (ji[3] * ji[7] - ji[4] * ji[6]);
    const bool neg = det < 0;
    for (int f = 0; f < nf; ++f) {
      const int32_t nb = H.nbr[t * nf + f];
      const bool owner = nb < 0 || t < nb;
      const bool sneg = neg != !owner;  // s_f = sign(det J) * (owner ? 1 : -1)
      const int64_t id = fid[t * nf + f];
      if (id < 0 || id >= (int64_t(1) << (31 - shift))) { err = "facet numbering"; return -6; }
      int code;
      if (d == 2) {
        int cv[2];
        dgmesh::canonical_vertices(2, f, H.perm_own[t * nf + f], cv);
        const int asc0 = f == 0 ? 1 : 0;  // first of the facet's ascending local vertices
        code = (sneg ? 2 : 0) | (cv[0] != asc0 ? 1 : 0);
      } else {
        code = (sneg ? 8 : 0) | H.perm_own[t * nf + f];
      }
      o.elem_facet[t * nf + f] = (int32_t)(id << shift) | code;
    }
  }
  o.N = o.nfacet * o.nfd + E * o.nint;
  reference_dual(d, H.k, o.table);
  if (d == 3) {
    std::vector<double> q;
    orientation_tables(H.k, q);
    o.table.insert(o.table.end(), q.begin(), q.end());
  }
  return 0;
}

}  // namespace dghdiv
