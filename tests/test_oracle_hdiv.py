"""Pins of the oracle's H(div) space W_h (BDM degrees of freedom, 2D and 3D) and the transfer
operators I = (M^V)^-1 M^{U,V} and I^T (Sec. 2.2, Sec. 2.4).

The transfer is pinned against the degrees of freedom evaluated directly in physical
coordinates (duality), against normal continuity (the defining property of W_h), against
exact reproduction of polynomial fields, and by rank and transpose identities.
"""
import numpy as np
import pytest

from oracle import refelem as R
from oracle.dg import Space
from oracle.hdiv import HdivSpace
from oracle.mesh import Mesh, box_mesh


def shuffled(N, per, seed, dim=2):
    base = box_mesh(dim, N, jitter=0.15, seed=seed, periodic=per)
    rng = np.random.default_rng(seed)
    X = base.X.copy()
    for t in range(base.E):
        X[t] = X[t][rng.permutation(dim + 1)]
    return Mesh(X, base.period)


MESHES = {
    "jittered": lambda: box_mesh(2, 3, jitter=0.15, seed=1),
    "shuffled": lambda: shuffled(3, (True, True), 2),
    "bounded": lambda: shuffled(3, (False, False), 3),
    "jittered3": lambda: box_mesh(3, 2, jitter=0.15, seed=1),
    "shuffled3": lambda: shuffled(2, (True, True, True), 2, dim=3),
    "bounded3": lambda: shuffled(2, (False, True, False), 3, dim=3),
}
MESHES_2D = ["bounded", "jittered", "shuffled"]
MESHES_3D = ["bounded3", "jittered3", "shuffled3"]


@pytest.mark.parametrize("name,k", [(n, k) for n in MESHES_2D for k in (1, 2, 3, 4, 5, 6)] +
                         [(n, k) for n in MESHES_3D for k in (1, 2, 3)] + [("shuffled3", 4)])
def test_dof_duality(name, k):
    """The dof functionals, evaluated directly on the DG field I u, give back u.

    The reference dual basis is the inverse of the reference moment matrix G, whose condition
    number grows with k (2D: 5e3 at k = 4, 6e4 at k = 5, 7e5 at k = 6: the Nedelec and facet
    moments of a monomial-based spanning set).  Inverting it in FP64 costs about eps cond(G)
    relative accuracy, so the bar is 1e-11 or 32 eps cond(G) max|u|, whichever is larger."""
    m = MESHES[name]()
    H = HdivSpace(m, k)
    u = np.random.default_rng(k).normal(size=H.N)
    bar = max(1e-11, 32 * np.finfo(float).eps * np.linalg.cond(H.C) * np.abs(u).max())
    assert np.abs(H.dofs(H.to_dg(u)) - u).max() < bar


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("k", [1, 3])
def test_normal_component_is_continuous(name, k):
    m = MESHES[name]()
    H = HdivSpace(m, k)
    sp = Space(m, k)
    v = H.to_dg(np.random.default_rng(5).normal(size=H.N))
    T = np.arange(m.E)
    pown, pnbr = sp.facet_basis(T)
    worst = 0.0
    for f in range(m.dim + 1):
        inner = m.nbr[:, f] >= 0
        N = np.where(inner, m.nbr[:, f], T)
        a = np.einsum("tqm,tim->tqi", pown[:, f], v)
        b = np.einsum("tqm,tim->tqi", pnbr[:, f], v[N])
        jump = np.einsum("tqi,ti->tq", a - b, m.normal[:, f])[inner]
        worst = max(worst, np.abs(jump).max())
    assert worst < 1e-12 * np.abs(v).max()


@pytest.mark.parametrize("k", [1, 2, 4])
def test_polynomial_fields_are_reproduced(k):
    """A global polynomial field p of degree <= k lies in W_h on a bounded mesh: its dof
    vector u_p = l(p) gives I u_p = the DG coefficients of p exactly."""
    m = shuffled(3, (False, False), 4)
    H = HdivSpace(m, k)
    sp = Space(m, k)
    rng = np.random.default_rng(6)
    coef = rng.normal(size=(2, k + 1, k + 1))
    def p(x):
        out = np.zeros(x.shape)
        for i in range(2):
            for a in range(k + 1):
                for b in range(k + 1 - a):
                    out[..., i] += coef[i, a, b] * x[..., 0] ** a * x[..., 1] ** b
        return out
    q = k + 3
    pdg = sp.project(p(sp.quad_points(q)), q)
    up = H.dofs(pdg)
    assert np.abs(H.to_dg(up) - pdg).max() < 1e-11 * np.abs(pdg).max()


def test_dimension_and_injectivity():
    m = shuffled(2, (True, True), 7)
    k = 2
    H = HdivSpace(m, k)
    assert H.n_facets == m.E * 3 // 2
    assert H.N == H.n_facets * (k + 1) + m.E * (k * k - 1)
    Imat = np.stack([H.to_dg(e).ravel() for e in np.eye(H.N)], axis=1)
    assert np.linalg.matrix_rank(Imat) == H.N


def test_transpose_identity():
    m = MESHES["shuffled"]()
    H = HdivSpace(m, 3)
    rng = np.random.default_rng(8)
    u = rng.normal(size=H.N)
    F = rng.normal(size=(m.E, 2, R.n_basis(2, 3)))
    assert abs(np.sum(H.to_dg(u) * F) - np.dot(u, H.transpose(F))) < 1e-11 * np.abs(F).sum()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_polynomial_fields_are_reproduced_3d(k):
    m = shuffled(2, (False, False, False), 4, dim=3)
    H = HdivSpace(m, k)
    sp = Space(m, k)
    rng = np.random.default_rng(16)
    terms = [(a, b, c) for a in range(k + 1) for b in range(k + 1 - a) for c in range(k + 1 - a - b)]
    coef = rng.normal(size=(3, len(terms)))
    def p(x):
        out = np.zeros(x.shape)
        for i in range(3):
            for n, (a, b, c) in enumerate(terms):
                out[..., i] += coef[i, n] * x[..., 0] ** a * x[..., 1] ** b * x[..., 2] ** c
        return out
    q = k + 3
    pdg = sp.project(p(sp.quad_points(q)), q)
    up = H.dofs(pdg)
    assert np.abs(H.to_dg(up) - pdg).max() < 1e-11 * np.abs(pdg).max()


def test_dimension_and_transpose_3d():
    m = MESHES["shuffled3"]()
    k = 2
    H = HdivSpace(m, k)
    assert H.n_facets == m.E * 4 // 2
    assert H.N == H.n_facets * 6 + m.E * 6
    Imat = np.stack([H.to_dg(e).ravel() for e in np.eye(H.N)], axis=1)
    assert np.linalg.matrix_rank(Imat) == H.N
    rng = np.random.default_rng(18)
    u = rng.normal(size=H.N)
    F = rng.normal(size=(m.E, 3, R.n_basis(3, k)))
    assert abs(np.sum(H.to_dg(u) * F) - np.dot(u, H.transpose(F))) < 1e-11 * np.abs(F).sum()


@pytest.mark.parametrize("dim,k", [(2, 3), (3, 1), (3, 3)])
def test_facet_orientation_matrices(dim, k):
    """The facet basis is orthonormal (identity for the identity permutation), every change
    of parameter is an orthogonal matrix, and reversing a 2D facet flips the odd Legendre
    moments."""
    import itertools
    from oracle.hdiv import orientation_matrix, n_facet_dofs
    nfd = n_facet_dofs(dim, k)
    for pos in itertools.permutations(range(dim)):
        Q = orientation_matrix(dim, k, pos)
        assert np.abs(Q @ Q.T - np.eye(nfd)).max() < 1e-13
        if pos == tuple(range(dim)):
            assert np.abs(Q - np.eye(nfd)).max() < 1e-13
        if dim == 2 and pos == (1, 0):
            assert np.abs(Q - np.diag([(-1.0) ** l for l in range(nfd)])).max() < 1e-13
