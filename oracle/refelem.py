"""Reference simplex for the oracle: orthonormal Dubiner basis and collapsed Gauss rules.

Test infrastructure (see ``oracle/__init__``).

Reference simplex: T^ = {xi_i >= 0, sum xi_i <= 1} (area 1/2 in 2D, volume 1/6 in 3D).

Basis.  The paper asks for an L2-orthogonal basis on every element so that the DG mass matrix
is diagonal (Sec. 2.3) and uses Dubiner's orthogonal polynomials for its facet spaces
(Sec. 2.2).  We take Dubiner's basis on T^, normalised to be orthonormal on T^:

  2D  phi_pq  = sqrt(2(2p+1)(p+q+1))              P_p(a) (1-eta)^p       P_q^(2p+1,0)(b)
  3D  phi_pqr = sqrt(2(2p+1)(p+q+1)(2p+2q+2r+3))  P_p(a) (1-eta-zeta)^p  P_q^(2p+1,0)(b) (1-zeta)^q
                                                  P_r^(2p+2q+2,0)(c)

with collapsed coordinates a = 2xi/(1-eta)-1, b = 2eta-1 (2D) and a = 2xi/(1-eta-zeta)-1,
b = 2eta/(1-zeta)-1, c = 2zeta-1 (3D).  Order: total degree ascending, then r descending, then
q descending.  Pins (tests/test_oracle_refelem.py): Gram matrix = I under a quadrature pinned
against exact monomial integrals, and equality with exact rational Gram-Schmidt of the
monomials xi^p eta^q zeta^r taken in the same order.

Gradients are taken by complex-step differentiation of the same closed form (no derivative
formula to get wrong); pinned against central differences.

Quadrature.  Collapsed (Duffy) tensor rules: n Gauss-Legendre points in a, n Gauss-Jacobi
(alpha=1) in b, n Gauss-Jacobi (alpha=2) in c; exact for total degree <= 2n-1.
"""
import functools
from math import comb

import numpy as np
from scipy.special import eval_jacobi, roots_jacobi


def n_basis(dim, k):
    """Number of polynomials of total degree <= k in `dim` variables."""
    return comb(k + dim, dim)


def basis_indices(dim, k):
    """Index tuples (p, q) or (p, q, r) in the canonical order of the basis."""
    out = []
    for n in range(k + 1):
        if dim == 2:
            for q in range(n, -1, -1):
                out.append((n - q, q))
        else:
            for r in range(n, -1, -1):
                for q in range(n - r, -1, -1):
                    out.append((n - r - q, q, r))
    return out


def ref_volume(dim):
    return 0.5 if dim == 2 else 1.0 / 6.0


def ref_vertices(dim):
    """Vertices of T^: origin then unit vectors (the local frame of every element)."""
    return np.vstack([np.zeros(dim), np.eye(dim)])


def _eval_closed_form(dim, k, pts):
    """phi_m(pts) for complex or real points of shape [..., dim] -> [..., Np]."""
    pts = np.asarray(pts)
    xi = pts[..., 0]
    eta = pts[..., 1]
    vals = []
    if dim == 2:
        one_m_eta = 1.0 - eta
        safe = np.where(np.abs(one_m_eta) < 1e-300, 1.0, one_m_eta)
        a = 2.0 * xi / safe - 1.0
        b = 2.0 * eta - 1.0
        for p, q in basis_indices(2, k):
            nrm = np.sqrt(2.0 * (2 * p + 1) * (p + q + 1))
            vals.append(nrm * eval_jacobi(p, 0.0, 0.0, a) * one_m_eta ** p
                        * eval_jacobi(q, 2.0 * p + 1.0, 0.0, b))
    else:
        zeta = pts[..., 2]
        s1 = 1.0 - eta - zeta
        s2 = 1.0 - zeta
        safe1 = np.where(np.abs(s1) < 1e-300, 1.0, s1)
        safe2 = np.where(np.abs(s2) < 1e-300, 1.0, s2)
        a = 2.0 * xi / safe1 - 1.0
        b = 2.0 * eta / safe2 - 1.0
        c = 2.0 * zeta - 1.0
        for p, q, r in basis_indices(3, k):
            nrm = np.sqrt(2.0 * (2 * p + 1) * (p + q + 1) * (2 * p + 2 * q + 2 * r + 3))
            vals.append(nrm * eval_jacobi(p, 0.0, 0.0, a) * s1 ** p
                        * eval_jacobi(q, 2.0 * p + 1.0, 0.0, b) * s2 ** q
                        * eval_jacobi(r, 2.0 * p + 2.0 * q + 2.0, 0.0, c))
    return np.stack(vals, axis=-1)


def eval_basis(dim, k, pts):
    """Orthonormal Dubiner basis at real points [..., dim] -> [..., Np] (FP64)."""
    return np.real(_eval_closed_form(dim, k, np.asarray(pts, dtype=np.float64)))


def eval_grad(dim, k, pts):
    """Reference gradients d phi_m / d xi_j at points [..., dim] -> [..., Np, dim].

    Complex-step derivative: Im phi(x + i h e_j) / h is the exact derivative up to rounding
    for any analytic function, independent of any hand-derived chain rule.
    """
    pts = np.asarray(pts, dtype=np.float64)
    h = 1e-30
    out = []
    for j in range(dim):
        z = pts.astype(np.complex128)
        z[..., j] += 1j * h
        out.append(np.imag(_eval_closed_form(dim, k, z)) / h)
    return np.stack(out, axis=-1)


def gauss_jacobi(n, alpha):
    """n-point Gauss-Jacobi rule on [-1,1] for the weight (1-x)^alpha."""
    x, w = roots_jacobi(n, alpha, 0.0)
    return np.asarray(x, dtype=np.float64), np.asarray(w, dtype=np.float64)


def collapsed_rule(dim, n):
    """Collapsed tensor Gauss rule on T^ with n points per direction.

    Returns points [n^dim, dim] and weights summing to |T^|.  Exact for total degree <= 2n-1.
    Point order: a fastest, then b, then c.
    """
    xa, wa = gauss_jacobi(n, 0.0)
    xb, wb = gauss_jacobi(n, 1.0)
    if dim == 2:
        B, A = np.meshgrid(xb, xa, indexing="ij")
        WB, WA = np.meshgrid(wb, wa, indexing="ij")
        xi = (1 + A) * (1 - B) / 4.0
        eta = (1 + B) / 2.0
        w = WA * WB / 8.0
        return np.stack([xi.ravel(), eta.ravel()], axis=1), w.ravel()
    xc, wc = gauss_jacobi(n, 2.0)
    C, B, A = np.meshgrid(xc, xb, xa, indexing="ij")
    WC, WB, WA = np.meshgrid(wc, wb, wa, indexing="ij")
    xi = (1 + A) * (1 - B) * (1 - C) / 8.0
    eta = (1 + B) * (1 - C) / 4.0
    zeta = (1 + C) / 2.0
    w = WA * WB * WC / 64.0
    return np.stack([xi.ravel(), eta.ravel(), zeta.ravel()], axis=1), w.ravel()


def facet_rule(dim, n):
    """Rule on the reference facet, weights summing to 1.

    2D: points s in [0,1] (Gauss-Legendre), shape [n, 1].
    3D: points (s, t) on the reference triangle, collapsed toward the third vertex
        (t = (1+b)/2, s = (1+a)(1-b)/4), shape [n*n, 2].
    A facet with canonical vertices (A, B[, C]) carries the point A + s(B-A) [+ t(C-A)].
    """
    if dim == 2:
        x, w = gauss_jacobi(n, 0.0)
        return ((1 + x) / 2.0)[:, None], w / 2.0
    p, w = collapsed_rule(2, n)
    return p, w * 2.0


# Fully symmetric triangle rules with positive weights and interior points: the degree-6
# rule with 12 points and the degree-9 rule with 19 points of D. A. Dunavant, "High degree
# efficient symmetrical Gaussian quadrature rules for the triangle", Int. J. Numer. Methods
# Eng. 21 (1985) 1129-1148.  Each is given by its orbits under the vertex permutations, with
# barycentric generators ("3": the centroid; "21": (a, a, 1-2a); "111": (a, b, 1-a-b)), and
# starting values of the free parameters to three digits; Gauss-Newton on the moment
# equations fixes them and the weights.  The equations integrate the orthonormal basis of
# degree <= the rule's degree (int phi_m = |T^|^(1/2) delta_m0), which keeps them well
# conditioned; the pins check the result against the exact monomial integrals.
_SYM_TRI = {
    6: [("21", (0.063,)), ("21", (0.249,)), ("111", (0.053, 0.310))],
    9: [("3", ()), ("21", (0.045,)), ("21", (0.188,)), ("21", (0.437,)), ("21", (0.490,)),
        ("111", (0.037, 0.222))],
}


def _tri_orbit(kind, p):
    """Distinct permutations of a barycentric generator, as (s, t) = (l1, l2) rows."""
    import itertools
    if kind == "3":
        g = (1.0 / 3, 1.0 / 3, 1.0 / 3)
    elif kind == "21":
        g = (p[0], p[0], 1.0 - 2.0 * p[0])
    else:
        g = (p[0], p[1], 1.0 - p[0] - p[1])
    out = []
    for perm in itertools.permutations(range(3)):
        b = tuple(g[i] for i in perm)
        if not any(np.allclose(b, c, rtol=0, atol=1e-12) for c in out):
            out.append(b)
    return np.array(out)[:, 1:]


@functools.lru_cache(maxsize=None)
def symmetric_triangle_rule(degree):
    """The symmetric rule of _SYM_TRI for `degree` on the unit triangle: points (s, t) [Q, 2],
    weights summing to 1/2 (the area)."""
    spec = _SYM_TRI[degree]
    target = np.zeros(n_basis(2, degree))
    target[0] = np.sqrt(0.5)
    npar = [len(p) for _, p in spec]
    npos = sum(npar)

    def moments_matrix(x):
        cols, k = [], 0
        for (kind, _), n in zip(spec, npar):
            P = _tri_orbit(kind, x[k:k + n])
            k += n
            cols.append(eval_basis(2, degree, P).sum(axis=0))
        return np.stack(cols, axis=1)

    def resid(z):
        return moments_matrix(z[:npos]) @ z[npos:] - target

    pos = np.array([v for _, p in spec for v in p], dtype=np.float64)
    w = np.linalg.lstsq(moments_matrix(pos), target, rcond=None)[0]
    z = np.concatenate([pos, w])
    for it in range(12):
        r = resid(z)
        J = np.empty((len(r), len(z)))
        for c in range(len(z)):
            hz = 1e-7
            zp, zm = z.copy(), z.copy()
            zp[c] += hz
            zm[c] -= hz
            J[:, c] = (resid(zp) - resid(zm)) / (2 * hz)
        dz = np.linalg.lstsq(J, r, rcond=None)[0]
        z = z - dz
        if np.abs(dz).max() < 1e-15:  # quadratic convergence: the next step is at rounding
            break
    pos, w = z[:npos], z[npos:]
    assert np.abs(resid(z)).max() < 1e-15 and np.all(w > 0)
    pts, wts, k = [], [], 0
    for (kind, _), n, wo in zip(spec, npar, w):
        P = _tri_orbit(kind, pos[k:k + n])
        k += n
        pts.append(P)
        wts.append(np.full(len(P), wo))
    return np.concatenate(pts), np.concatenate(wts)


def operator_facet_rule(dim, k):
    """The facet rule of the convection operator: exact to degree 3k, weights summing to 1.
    2D: facet_rule(2, facet_points(k)).  3D: the symmetric rule of degree 3k where there is
    one (k = 2: 12 points, k = 3: 19 points), else facet_rule(3, facet_points(k))."""
    if dim == 3 and 3 * k in _SYM_TRI:
        p, w = symmetric_triangle_rule(3 * k)
        return p, 2.0 * w
    return facet_rule(dim, facet_points(k))


def volume_points_for_oracle(k):
    """Points per direction of the oracle's volume rule.

    The volume integrand w_i u_j d_j phi_m has degree 3k-1 on an affine element, so any rule
    exact to 3k-1 gives the same operator up to rounding.  The oracle deliberately takes one
    point more than the minimum ceil(3k/2) (exact to 3k+1).
    """
    return (3 * k + 1) // 2 + 1


def facet_points(k):
    """Points per direction of the facet rule: exact to degree 3k.

    The upwind value is taken pointwise, so the facet rule is part of the definition of the
    discrete operator when the normal velocity changes sign inside a facet.
    """
    return max(1, (3 * k + 2) // 2)
