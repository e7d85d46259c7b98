// Reference-simplex math for the device tables (host, FP64).
//
// Orthonormal Dubiner basis on the unit simplex (the L2-orthogonal element basis that makes
// the DG mass matrix diagonal, Sec. 2.3 of the paper; Dubiner's construction is the one the
// paper uses for its facet spaces, Sec. 2.2).  Evaluated through division-free "scaled"
// Jacobi recurrences carried in forward-mode dual numbers, so values and reference gradients
// come from one pass and stay finite everywhere on the closed simplex:
//
//   2D  phi_pq  = c_pq  * L_p(2xi+eta-1, 1-eta) * P_q^(2p+1,0)(2eta-1)
//   3D  phi_pqr = c_pqr * L_p(2xi+eta+zeta-1, 1-eta-zeta) * S_q^(2p+1)(2eta+zeta-1, 1-zeta)
//                       * P_r^(2p+2q+2,0)(2zeta-1)
//
// with L_n(x, s) = s^n P_n(x/s) (scaled Legendre) and S_n^(a)(y, s) = s^n P_n^(a,0)(y/s), and
// c the normalisation to unit L2 norm on the reference simplex.  Order of the basis: total
// degree ascending, then r descending, then q descending.
//
// Quadrature: Gauss-Jacobi nodes by Newton iteration with polynomial deflation; collapsed
// (Duffy) tensor rules on the simplex; the fully symmetric volume and 3D facet rules of
// sym_rules.hpp (fewer points at the same degree) where there is one.  Everything is evaluated in long double and rounded to
// FP64 once, so the device tables are correctly rounded up to a few ulp.
#pragma once
#include <array>
#include <cmath>
#include <vector>
#include "sym_rules.hpp"

namespace dgref {

// value and up to three partial derivatives
// Host tables are computed in long double (x87 extended precision) and rounded to FP64 once.
typedef long double real;

struct Dual {
  real v = 0, d[3] = {0, 0, 0};
  Dual() = default;
  explicit Dual(real x) : v(x) {}
};
inline Dual operator+(const Dual& a, const Dual& b) {
  Dual r; r.v = a.v + b.v;
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
inline Dual operator-(const Dual& a, const Dual& b) {
  Dual r; r.v = a.v - b.v;
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
inline Dual operator*(const Dual& a, const Dual& b) {
  Dual r; r.v = a.v * b.v;
  for (int i = 0; i < 3; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
inline Dual operator*(real s, const Dual& a) {
  Dual r; r.v = s * a.v;
  for (int i = 0; i < 3; ++i) r.d[i] = s * a.d[i];
  return r;
}

// s^n P_n^(alpha,0)(y/s), n = 0..nmax, by the three-term recurrence multiplied through by s^n
inline std::vector<Dual> scaled_jacobi(int nmax, real alpha, const Dual& y, const Dual& s) {
  std::vector<Dual> J(nmax + 1);
  J[0] = Dual(1.0L);
  if (nmax >= 1) J[1] = 0.5L * ((alpha + 2.0L) * y + alpha * s);
  const Dual s2 = s * s;
  for (int n = 2; n <= nmax; ++n) {
    const real a = alpha;
    const real c0 = 2.0L * n * (n + a) * (2.0L * n + a - 2.0L);
    const real c1 = (2.0L * n + a - 1.0L) * (2.0L * n + a) * (2.0L * n + a - 2.0L);
    const real c2 = (2.0L * n + a - 1.0L) * a * a;
    const real c3 = 2.0L * (n + a - 1.0L) * (n - 1.0L) * (2.0L * n + a);
    J[n] = (1.0L / c0) * ((c1 * y + c2 * s) * J[n - 1] - c3 * (s2 * J[n - 2]));
  }
  return J;
}

inline int n_basis(int dim, int k) {
  return dim == 2 ? (k + 1) * (k + 2) / 2 : (k + 1) * (k + 2) * (k + 3) / 6;
}

// (p,q,r) in canonical order (r = 0 in 2D)
inline std::vector<std::array<int, 3>> basis_indices(int dim, int k) {
  std::vector<std::array<int, 3>> out;
  for (int n = 0; n <= k; ++n) {
    if (dim == 2) {
      for (int q = n; q >= 0; --q) out.push_back({n - q, q, 0});
    } else {
      for (int r = n; r >= 0; --r)
        for (int q = n - r; q >= 0; --q) out.push_back({n - r - q, q, r});
    }
  }
  return out;
}

// phi_m and d phi_m / d xi_j at one reference point; val[m], grad[m*dim + j]
template <typename Out>
inline void eval_basis_t(int dim, int k, const real* xi, Out* val, Out* grad) {
  Dual X[3];
  for (int j = 0; j < dim; ++j) { X[j].v = xi[j]; X[j].d[j] = 1.0L; }
  const auto idx = basis_indices(dim, k);
  const Dual one(1.0L);
  if (dim == 2) {
    const Dual x = 2.0L * X[0] + X[1] - one, s = one - X[1];
    const auto L = scaled_jacobi(k, 0.0L, x, s);
    const Dual b = 2.0L * X[1] - one;
    for (size_t m = 0; m < idx.size(); ++m) {
      const int p = idx[m][0], q = idx[m][1];
      const auto Q = scaled_jacobi(q, 2.0L * p + 1.0L, b, one);
      const real c = std::sqrt((real)(2.0L * (2 * p + 1) * (p + q + 1)));
      const Dual f = c * (L[p] * Q[q]);
      val[m] = (Out)f.v;
      if (grad) for (int j = 0; j < 2; ++j) grad[m * 2 + j] = (Out)f.d[j];
    }
  } else {
    const Dual x = 2.0L * X[0] + X[1] + X[2] - one, s1 = one - X[1] - X[2];
    const Dual y = 2.0L * X[1] + X[2] - one, s2 = one - X[2];
    const Dual z = 2.0L * X[2] - one;
    const auto L = scaled_jacobi(k, 0.0L, x, s1);
    for (size_t m = 0; m < idx.size(); ++m) {
      const int p = idx[m][0], q = idx[m][1], r = idx[m][2];
      const auto S = scaled_jacobi(q, 2.0L * p + 1.0L, y, s2);
      const auto Rr = scaled_jacobi(r, 2.0L * p + 2.0L * q + 2.0L, z, one);
      const real c = std::sqrt((real)(2.0L * (2 * p + 1) * (p + q + 1) * (2 * p + 2 * q + 2 * r + 3)));
      const Dual f = c * (L[p] * (S[q] * Rr[r]));
      val[m] = (Out)f.v;
      if (grad) for (int j = 0; j < 3; ++j) grad[m * 3 + j] = (Out)f.d[j];
    }
  }
}

// double interface (points given in FP64)
inline void eval_basis(int dim, int k, const double* xi, double* val, double* grad) {
  real x[3] = {0, 0, 0};
  for (int j = 0; j < dim; ++j) x[j] = xi[j];
  eval_basis_t<double>(dim, k, x, val, grad);
}

// P_n^(alpha,0)(x) and its derivative (plain recurrence, used for Newton)
inline void jacobi_pd(int n, real alpha, real x, real* p, real* dp) {
  real p0 = 1.0L, p1 = 0.5L * ((alpha + 2.0L) * x + alpha);
  real d0 = 0.0L, d1 = 0.5L * (alpha + 2.0L);
  if (n == 0) { *p = 1.0L; *dp = 0.0L; return; }
  for (int m = 2; m <= n; ++m) {
    const real a = alpha;
    const real c0 = 2.0L * m * (m + a) * (2.0L * m + a - 2.0L);
    const real c1 = (2.0L * m + a - 1.0L) * (2.0L * m + a) * (2.0L * m + a - 2.0L);
    const real c2 = (2.0L * m + a - 1.0L) * a * a;
    const real c3 = 2.0L * (m + a - 1.0L) * (m - 1.0L) * (2.0L * m + a);
    const real p2 = ((c1 * x + c2) * p1 - c3 * p0) / c0;
    const real d2 = ((c1 * x + c2) * d1 + c1 * p1 - c3 * d0) / c0;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  *p = p1; *dp = d1;
}

// n-point Gauss-Jacobi rule on [-1,1] for the weight (1-x)^alpha (beta = 0): Newton on the
// zeros of P_n^(alpha,0) with deflation by the zeros already found; for beta = 0 the
// Christoffel weights reduce to w = 2^(alpha+1) / ((1 - x^2) P_n'(x)^2).
inline void gauss_jacobi_r(int n, real alpha, std::vector<real>& x, std::vector<real>& w) {
  x.assign(n, 0.0L); w.assign(n, 0.0L);
  const real pi = 3.141592653589793238462643383279502884L;
  for (int k = 0; k < n; ++k) {
    real r = -std::cos((2.0L * k + 1.0L) * pi / (2.0L * n));
    if (k > 0) r = 0.5L * (r + x[k - 1]);
    for (int it = 0; it < 200; ++it) {
      real p, dp;
      jacobi_pd(n, alpha, r, &p, &dp);
      real s = 0.0L;
      for (int i = 0; i < k; ++i) s += 1.0L / (r - x[i]);
      const real delta = -p / (dp - s * p);
      r += delta;
      if (std::fabs(delta) < 1e-19L) break;
    }
    x[k] = r;
  }
  for (int k = 0; k < n; ++k) {
    real p, dp;
    jacobi_pd(n, alpha, x[k], &p, &dp);
    w[k] = std::pow(2.0L, alpha + 1.0L) / ((1.0L - x[k] * x[k]) * dp * dp);
  }
}

inline void gauss_jacobi(int n, double alpha, std::vector<double>& x, std::vector<double>& w) {
  std::vector<real> xr, wr;
  gauss_jacobi_r(n, alpha, xr, wr);
  x.assign(xr.begin(), xr.end());
  w.assign(wr.begin(), wr.end());
}

// collapsed rule on the reference simplex, n points per direction; weights sum to |T^|.
// Point order: a fastest, then b, then c.
template <typename T>
inline void collapsed_rule(int dim, int n, std::vector<T>& pts, std::vector<T>& wts) {
  std::vector<real> xa, wa, xb, wb, xc, wc;
  gauss_jacobi_r(n, 0.0L, xa, wa);
  gauss_jacobi_r(n, 1.0L, xb, wb);
  pts.clear(); wts.clear();
  if (dim == 2) {
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        pts.push_back((T)((1 + xa[i]) * (1 - xb[j]) / 4.0L));
        pts.push_back((T)((1 + xb[j]) / 2.0L));
        wts.push_back((T)(wa[i] * wb[j] / 8.0L));
      }
    return;
  }
  gauss_jacobi_r(n, 2.0L, xc, wc);
  for (int l = 0; l < n; ++l)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        pts.push_back((T)((1 + xa[i]) * (1 - xb[j]) * (1 - xc[l]) / 8.0L));
        pts.push_back((T)((1 + xb[j]) * (1 - xc[l]) / 4.0L));
        pts.push_back((T)((1 + xc[l]) / 2.0L));
        wts.push_back((T)(wa[i] * wb[j] * wc[l] / 64.0L));
      }
}

// rule on the reference facet, weights summing to 1: 2D s in [0,1]; 3D (s,t) on the
// reference triangle collapsed toward the third canonical vertex.
template <typename T>
inline void facet_rule(int dim, int n, std::vector<T>& pts, std::vector<T>& wts) {
  if (dim == 2) {
    std::vector<real> x, w;
    gauss_jacobi_r(n, 0.0L, x, w);
    pts.resize(n); wts.resize(n);
    for (int i = 0; i < n; ++i) { pts[i] = (T)((1 + x[i]) / 2.0L); wts[i] = (T)(w[i] / 2.0L); }
    return;
  }
  collapsed_rule<T>(2, n, pts, wts);
  for (auto& v : wts) v *= 2;
}

inline int vol_points_1d(int k) { int n = (3 * k + 1) / 2; return n < 1 ? 1 : n; }   // exact to 3k-1
inline int facet_points_1d(int k) { int n = (3 * k + 2) / 2; return n < 1 ? 1 : n; } // exact to 3k

// The volume rule of the operator, exact to degree 3k-1 (the degree of the volume integrand):
// the fully symmetric rule of sym_rules.hpp where there is one, else the collapsed rule
// with vol_points_1d(k) points per direction.  Weights sum to |T^|.
template <typename T>
inline void volume_rule(int dim, int k, std::vector<T>& pts, std::vector<T>& wts) {
  const long double *p = nullptr, *w = nullptr;
  if (sym_vol_rule(dim, k, &p, &w)) {
    const int n = sym_vol_points(dim, k);
    pts.assign(p, p + (size_t)n * dim);
    wts.assign(w, w + n);
    return;
  }
  collapsed_rule<T>(dim, vol_points_1d(k), pts, wts);
}

// The facet rule of the operator, exact to degree 3k, weights summing to 1 (part of the
// operator's definition, the upwind value being taken pointwise): 2D facet_rule with
// facet_points_1d(k) points; 3D the symmetric rule of sym_rules.hpp where there is one (k = 2,
// 3), else the collapsed facet_rule with facet_points_1d(k)^2 points.
template <typename T>
inline void operator_facet_rule(int dim, int k, std::vector<T>& pts, std::vector<T>& wts) {
  const long double *p = nullptr, *w = nullptr;
  if (dim == 3 && sym_facet_rule(k, &p, &w)) {
    const int n = sym_facet_points(k);
    pts.assign(p, p + (size_t)n * 2);
    wts.assign(w, w + n);
    return;
  }
  facet_rule<T>(dim, facet_points_1d(k), pts, wts);
}

}  // namespace dgref
