"""Exact rational assembly of the frozen-velocity operator on tiny meshes (a pin).

Test infrastructure (see ``oracle/__init__``).

For a constant convecting velocity u (exactly divergence-free, normal-continuous) the upwind
trilinear form of Sec. 2.3 is bilinear in (w, z), the normal speed u.n is constant on every
facet, and the upwind side is fixed per facet, so every integrand is a polynomial.  This
module assembles the matrix L of  r = -(M^V)^-1 C_h(u; w, .)  entry by entry with exact
rational arithmetic (SymPy):

  * its own L2-orthogonal basis: Gram-Schmidt of the monomials xi^p eta^q zeta^r in the same
    order as the oracle's basis, exact over Q (normalisation applied in FP64 at the end);
  * exact monomial integrals on the reference simplex, int xi^a eta^b = a! b! / (a+b+2)! and
    int xi^a eta^b zeta^c = a! b! c! / (a+b+c+3)!;
  * facet integrals by exact parametrisation of each facet, int_F g ds = |F| * mean over the
    reference facet, with |F| n = the rotated edge (2D) or half the cross product (3D), which
    keeps (u.n)|F| rational.

It shares nothing with the oracle's quadrature, basis evaluation or facet-point machinery.
"""
from fractions import Fraction
from math import factorial, sqrt

import numpy as np
import sympy as sp


def monomial_exponents(dim, k):
    """Exponents (p,q[,r]) in the canonical basis order (degree up, then r down, then q down)."""
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


def ref_monomial_integral(e):
    """Exact integral of xi^a eta^b (zeta^c) over the reference simplex."""
    num = 1
    for a in e:
        num *= factorial(a)
    return Fraction(num, factorial(sum(e) + len(e)))


def _poly_integral_ref(poly, gens):
    """Exact integral of a SymPy polynomial over the reference simplex in `gens`."""
    P = sp.Poly(sp.expand(poly), *gens)
    tot = Fraction(0)
    for mon, c in P.terms():
        c = Fraction(int(sp.numer(c)), int(sp.denom(c)))
        tot += c * ref_monomial_integral(mon)
    return tot


class ExactBasis:
    """Orthogonal (unnormalised) polynomials psi_m with rational coefficients, norms^2 D_m."""

    def __init__(self, dim, k):
        self.dim, self.k = dim, k
        self.gens = sp.symbols("x0:%d" % dim)
        exps = monomial_exponents(dim, k)
        mons = [sp.Mul(*[g ** a for g, a in zip(self.gens, e)]) for e in exps]
        psis, norms = [], []
        for mono in mons:
            p = mono
            for q, nq in zip(psis, norms):
                coef = _poly_integral_ref(mono * q, self.gens) / nq
                p = p - sp.Rational(coef.numerator, coef.denominator) * q
            p = sp.expand(p)
            psis.append(p)
            norms.append(_poly_integral_ref(p * p, self.gens))
        self.psi = psis
        self.norm2 = norms  # Fractions


def _rat(x):
    return sp.Rational(Fraction(float(x)).limit_denominator(1 << 40)) if not isinstance(
        x, sp.Rational) else x


def assemble_frozen_constant(X, period, k, u, nbr, nbr_facet, shift):
    """Dense L with r = L c for frozen constant u, by exact integration.

    X: [E, d+1, d] element vertices (rational-valued floats); u: constant velocity (floats
    with small rational values); nbr, nbr_facet, shift: facet connectivity (any correct
    matching, e.g. the oracle mesh's).  Returns L over the flattened index (T, m) for one
    velocity component (the frozen operator acts componentwise) as an FP64 array.
    """
    E, nv, d = X.shape
    B = ExactBasis(d, k)
    gens = B.gens
    Np = len(B.psi)
    u = [sp.Rational(Fraction(float(v)).limit_denominator(1 << 20)) for v in u]
    Xr = [[[_rat(X[t, a, j]) for j in range(d)] for a in range(nv)] for t in range(E)]
    Jm, Jinv, adet = [], [], []
    for t in range(E):
        J = sp.Matrix(d, d, lambda i, j: Xr[t][j + 1][i] - Xr[t][0][i])
        Jm.append(J)
        Jinv.append(J.inv())
        adet.append(abs(J.det()))
    C = [[Fraction(0)] * (E * Np) for _ in range(E * Np)]  # C[(T,m)][(T',m')]

    def add(i, j, val):
        C[i][j] += val

    # volume: - int_T psi_m' u . grad psi_m dx = -|J| int_ref psi_m' (J^-1 u) . grad^ psi_m
    grads = [[sp.diff(p, g) for g in gens] for p in B.psi]
    for t in range(E):
        uh = Jinv[t] * sp.Matrix(u)
        for m in range(Np):
            conv = sum(uh[j] * grads[m][j] for j in range(d))
            for mp in range(Np):
                val = _poly_integral_ref(B.psi[mp] * conv, gens)
                add(t * Np + m, t * Np + mp, -Fraction(int(sp.numer(adet[t])),
                                                       int(sp.denom(adet[t]))) * val)
    # facets: int_F (u.n) w^ psi_m ds
    s = sp.symbols("s0:%d" % (d - 1))
    for t in range(E):
        for f in range(d + 1):
            fv = [a for a in range(d + 1) if a != f]
            A = sp.Matrix(Xr[t][fv[0]])
            Vs = [sp.Matrix(Xr[t][a]) - A for a in fv[1:]]
            if d == 2:
                nF = sp.Matrix([Vs[0][1], -Vs[0][0]])  # |F| n up to sign
                meas_factor = 1  # int_F g = |F| int_0^1 g(A + s V) ds ; |F| absorbed in nF
            else:
                nF = Vs[0].cross(Vs[1]) / 2
                meas_factor = 2  # int_F g = 2|F| int_ref-tri g(A + s V0 + t V1)
            opp = sp.Matrix(Xr[t][f]) - A
            if (nF.T * opp)[0] > 0:
                nF = -nF
            un = sum(u[j] * nF[j] for j in range(d))  # (u.n)|F|, rational
            if un == 0:
                continue
            x = A + sum((s[c] * Vs[c] for c in range(d - 1)), sp.zeros(d, 1))
            xi_own = Jinv[t] * (x - sp.Matrix(Xr[t][0]))
            if un > 0:
                up_t, xi_up = t, xi_own
            else:
                up_t = int(nbr[t, f])
                sh = sp.Matrix([_rat(v) for v in shift[t, f]])
                xi_up = Jinv[up_t] * (x - sh - sp.Matrix(Xr[up_t][0]))
            sub_own = {gens[j]: xi_own[j] for j in range(d)}
            sub_up = {gens[j]: xi_up[j] for j in range(d)}
            own_vals = [sp.expand(p.subs(sub_own, simultaneous=True)) for p in B.psi]
            up_vals = [sp.expand(p.subs(sub_up, simultaneous=True)) for p in B.psi]
            for m in range(Np):
                for mp in range(Np):
                    val = _poly_integral_ref(up_vals[mp] * own_vals[m], s) * meas_factor
                    add(t * Np + m, up_t * Np + mp,
                        Fraction(int(sp.numer(un)), int(sp.denom(un))) * val)
    # r = -(M^V)^-1 C in the orthonormal basis phi = psi / sqrt(D)
    L = np.zeros((E * Np, E * Np))
    for t in range(E):
        for m in range(Np):
            i = t * Np + m
            mass = float(adet[t])  # int_T phi_m^2 = |J|
            for j in range(E * Np):
                if C[i][j] != 0:
                    mp = j % Np
                    L[i, j] = -float(C[i][j]) / (mass * sqrt(float(B.norm2[m]) *
                                                           float(B.norm2[mp])))
    return L
