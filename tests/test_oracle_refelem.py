"""Pins of the oracle's reference element against closed forms (no GPU)."""
from fractions import Fraction
from math import factorial

import numpy as np
import pytest

from oracle import refelem as R
from oracle.bruteforce import ExactBasis, monomial_exponents


def exact_monomial(e):
    num = 1
    for a in e:
        num *= factorial(a)
    return num / factorial(sum(e) + len(e))


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_collapsed_rule_exact_on_monomials(dim, n):
    p, w = R.collapsed_rule(dim, n)
    assert np.isclose(w.sum(), R.ref_volume(dim), rtol=0, atol=1e-15)
    for e in monomial_exponents(dim, 2 * n - 1):
        val = np.sum(w * np.prod(p ** np.array(e), axis=1))
        assert abs(val - exact_monomial(e)) < 1e-15 * max(1.0, 1.0), (e, val)


@pytest.mark.parametrize("dim", [2, 3])
def test_collapsed_rule_not_exact_beyond(dim):
    # degree 2n must fail for some monomial (checks we do not over-claim exactness)
    n = 3
    p, w = R.collapsed_rule(dim, n)
    errs = [abs(np.sum(w * np.prod(p ** np.array(e), axis=1)) - exact_monomial(e))
            for e in monomial_exponents(dim, 2 * n) if sum(e) == 2 * n]
    assert max(errs) > 1e-10


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("n", [1, 2, 4, 7])
def test_facet_rule_exact(dim, n):
    p, w = R.facet_rule(dim, n)
    assert np.isclose(w.sum(), 1.0, atol=1e-15)
    exps = [(a,) for a in range(2 * n)] if dim == 2 else monomial_exponents(2, 2 * n - 1)
    for e in exps:
        val = np.sum(w * np.prod(p ** np.array(e), axis=1))
        # mean over the reference facet: integral / |facet|
        ref = exact_monomial(e) * (1.0 if dim == 2 else 2.0)
        assert abs(val - ref) < 1e-15, (e, val, ref)


@pytest.mark.parametrize("dim,k", [(2, 0), (2, 1), (2, 4), (2, 6), (3, 0), (3, 2), (3, 4)])
def test_basis_orthonormal(dim, k):
    p, w = R.collapsed_rule(dim, k + 1)  # exact to 2k+1
    phi = R.eval_basis(dim, k, p)
    G = np.einsum("q,qm,qn->mn", w, phi, phi)
    assert np.abs(G - np.eye(R.n_basis(dim, k))).max() < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_constant_basis_function(dim):
    v = R.eval_basis(dim, 2, np.array([[0.1] * dim]))[0, 0]
    assert np.isclose(v, np.sqrt(2.0) if dim == 2 else np.sqrt(6.0), rtol=0, atol=1e-15)


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2)])
def test_basis_equals_exact_gram_schmidt(dim, k):
    """The oracle's Dubiner basis is Gram-Schmidt of the ordered monomials (exact over Q)."""
    import sympy as sp
    B = ExactBasis(dim, k)
    rng = np.random.default_rng(1)
    pts = rng.dirichlet(np.ones(dim + 1), size=20)[:, :dim]
    phi = R.eval_basis(dim, k, pts)
    f = sp.lambdify(B.gens, B.psi, "numpy")
    for j in range(pts.shape[0]):
        vals = np.array(f(*pts[j]), dtype=float) / np.sqrt([float(x) for x in B.norm2])
        assert np.abs(vals - phi[j]).max() < 1e-12


@pytest.mark.parametrize("dim,k", [(2, 3), (2, 5), (3, 3)])
def test_gradient_vs_central_differences(dim, k):
    rng = np.random.default_rng(2)
    pts = rng.dirichlet(np.ones(dim + 1), size=8)[:, :dim] * 0.9 + 0.02
    g = R.eval_grad(dim, k, pts)
    h = 1e-4
    for j in range(dim):
        e = np.zeros(dim)
        e[j] = h
        # 4th-order central difference
        fd = (-R.eval_basis(dim, k, pts + 2 * e) + 8 * R.eval_basis(dim, k, pts + e)
              - 8 * R.eval_basis(dim, k, pts - e) + R.eval_basis(dim, k, pts - 2 * e)) / (12 * h)
        assert np.abs(fd - g[..., j]).max() < 1e-6 * max(1.0, np.abs(g).max())


def test_basis_counts_and_order():
    assert R.n_basis(2, 4) == 15 and R.n_basis(3, 3) == 20 and R.n_basis(3, 2) == 10
    assert R.basis_indices(2, 1) == [(0, 0), (0, 1), (1, 0)]
    assert R.basis_indices(3, 1) == [(0, 0, 0), (0, 0, 1), (0, 1, 0), (1, 0, 0)]


@pytest.mark.parametrize("k,npts", [(2, 12), (3, 19)])
def test_symmetric_facet_rule(k, npts):
    """The 3D operator's facet rule for k = 2, 3: exact to degree 3k and not beyond, weights
    summing to 1, positive weights, points inside the triangle, invariant under the six
    permutations of the triangle's vertices, fewer points than the collapsed rule."""
    import itertools
    p, w = R.operator_facet_rule(3, k)
    assert len(w) == npts < R.facet_points(k) ** 2
    assert abs(w.sum() - 1.0) < 1e-15 and np.all(w > 0)
    bary = np.concatenate([1 - p.sum(1, keepdims=True), p], 1)
    assert bary.min() > 0
    for e in monomial_exponents(2, 3 * k):
        val = np.sum(w * np.prod(p ** np.array(e), axis=1))
        assert abs(val - 2.0 * exact_monomial(e)) < 1e-15, (e, val)
    errs = [abs(np.sum(w * np.prod(p ** np.array(e), axis=1)) - 2.0 * exact_monomial(e))
            for e in monomial_exponents(2, 3 * k + 1) if sum(e) == 3 * k + 1]
    assert max(errs) > 1e-10
    key = {tuple(np.round(b, 12)): x for b, x in zip(bary, w)}
    for perm in itertools.permutations(range(3)):
        for b, x in zip(bary, w):
            pb = tuple(np.round(b[list(perm)], 12))
            assert pb in key and abs(key[pb] - x) < 1e-15
