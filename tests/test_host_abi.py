"""Host-side checks of the C ABI (no GPU): symbols, mesh processing, basis, projection, errors.

These compare the library's host code (its own basis recurrences, Gauss rules, facet matching)
with the oracle, which shares no code with it.
"""
import ctypes
import itertools
import os
import re

import numpy as np
import pytest

import paper_1508_04245_amd as dg
from oracle import refelem as R
from oracle.dg import Space
from oracle.mesh import Mesh as OMesh, box_mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "dgconv.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    L = dg.lib()
    names = header_functions()
    assert "dg_convection_apply" in names and "dg_rk_substeps" in names
    for n in names:
        assert hasattr(L, n), n
    assert b"gfx950" in L.dg_version()


def lattice_mesh(dim, N, jitter=0.0, seed=0):
    """(N+1)^dim vertex array + connectivity in the oracle box ordering (+ periodic jitter)."""
    h = 1.0 / N
    rng = np.random.default_rng(seed)
    off = rng.uniform(-1, 1, size=(N,) * dim + (dim,)) * jitter * h if jitter else None
    grid = np.stack(np.meshgrid(*([np.arange(N + 1)] * dim), indexing="ij"), -1)
    grid = np.moveaxis(grid, list(range(dim)), list(range(dim))[::-1]).reshape(-1, dim)
    # vertex id = i + (N+1) j (+ (N+1)^2 l), coordinates lattice * h (+ jitter of the wrap)
    xyz = grid * h
    if off is not None:
        xyz = xyz + off[tuple(np.mod(grid[:, a], N) for a in range(dim))]
    vid = lambda idx: sum(int(idx[a]) * (N + 1) ** a for a in range(dim))
    elem = []
    if dim == 2:
        for j in range(N):
            for i in range(N):
                b = np.array([i, j])
                elem.append([vid(b), vid(b + [1, 0]), vid(b + [1, 1])])
                elem.append([vid(b + [1, 1]), vid(b + [0, 1]), vid(b)])
    else:
        eye = np.eye(3, dtype=int)
        for l in range(N):
            for j in range(N):
                for i in range(N):
                    b = np.array([i, j, l])
                    for s in itertools.permutations(range(3)):
                        elem.append([vid(b), vid(b + eye[s[0]]), vid(b + eye[s[0]] + eye[s[1]]),
                                     vid(b + 1)])
    return xyz, np.array(elem, dtype=np.int64)


@pytest.mark.parametrize("dim,N", [(2, 4), (2, 1), (3, 3), (3, 1)])
def test_box_mesh_matches_oracle(dim, N):
    m = dg.Mesh.box(dim, N, 2)
    om = box_mesh(dim, N)
    assert m.E == om.E
    assert np.array_equal(m.vertices(), om.X)
    nb, nf = m.neighbors()
    assert np.array_equal(nb, om.nbr) and np.array_equal(nf, om.nbr_facet)
    assert 1 <= m.info["n_types"] <= (2 if dim == 2 else 6)
    assert np.isclose(m.info["volume"], 1.0)


@pytest.mark.parametrize("dim,N,jit", [(2, 5, 0.25), (3, 3, 0.2)])
def test_general_mesh_matches_oracle(dim, N, jit):
    xyz, elem = lattice_mesh(dim, N, jit, seed=3)
    m = dg.Mesh.from_arrays(dim, 2, xyz, elem, np.ones(dim))
    om = OMesh(xyz[elem], np.ones(dim))
    nb, nf = m.neighbors()
    assert np.array_equal(nb, om.nbr) and np.array_equal(nf, om.nbr_facet)
    assert m.info["n_types"] >= (2 if dim == 2 else 6)


@pytest.mark.parametrize("dim,k", [(2, 0), (2, 3), (2, 6), (3, 1), (3, 4)])
def test_basis_matches_oracle(dim, k):
    rng = np.random.default_rng(0)
    pts = rng.dirichlet(np.ones(dim + 1), size=50)[:, :dim]
    pts = np.vstack([pts, R.ref_vertices(dim)])  # vertices too (collapsed-coordinate poles)
    v, g = dg.eval_basis(dim, k, pts)
    assert np.abs(v - R.eval_basis(dim, k, pts)).max() < 1e-12
    inner = pts[:50]
    ge = R.eval_grad(dim, k, inner)
    assert np.abs(g[:50] - ge).max() <= 1e-13 * max(1.0, np.abs(ge).max())


@pytest.mark.parametrize("dim,k,n", [(2, 4, 9), (3, 2, 6)])
def test_projection_matches_oracle(dim, k, n):
    from paper_1508_04245_amd import synth
    m = dg.Mesh.box(dim, 3, k)
    sp = Space(box_mesh(dim, 3), k)
    x = m.project_points(n)
    assert np.abs(x - sp.quad_points(n)).max() < 1e-15
    f = synth.taylor_green_2d(x) if dim == 2 else synth.taylor_green_3d(x)
    c = m.project(f, n)
    assert np.abs(c - sp.project(f, n)).max() < 1e-13


def test_error_paths():
    with pytest.raises(dg.DGError) as e:
        dg.Mesh.box(4, 2, 1)
    assert e.value.status == -1
    with pytest.raises(dg.DGError) as e:
        dg.Mesh.box(3, 2, 5)
    assert e.value.status == -4
    # non-periodic use of a box: facets on the boundary are unmatched
    xyz, elem = lattice_mesh(2, 3)
    with pytest.raises(dg.DGError) as e:
        dg.Mesh.from_arrays(2, 1, xyz, elem, np.array([2.0, 2.0]))
    assert e.value.status == -6
    # degenerate element
    xyz2 = xyz.copy()
    bad = elem.copy()
    bad[0] = [bad[0][0], bad[0][0], bad[0][2]]
    with pytest.raises(dg.DGError) as e:
        dg.Mesh.from_arrays(2, 1, xyz2, bad, np.ones(2))
    assert e.value.status == -6
    # vertex id out of range
    bad = elem.copy()
    bad[3, 1] = 10 ** 6
    with pytest.raises(dg.DGError) as e:
        dg.Mesh.from_arrays(2, 1, xyz, bad, np.ones(2))
    assert e.value.status == -1
    # rule queries: dimension, degree, missing count pointer
    L = dg.lib()
    for fn in (L.dg_volume_rule, L.dg_facet_rule):
        n = ctypes.c_int(-7)
        assert fn(4, 1, ctypes.byref(n), None, None) == -1
        assert fn(3, 5, ctypes.byref(n), None, None) == -4
        assert fn(2, 7, ctypes.byref(n), None, None) == -4
        assert fn(2, 2, None, None, None) == -1
        assert n.value == -7  # nothing written on an error
        assert fn(2, 2, ctypes.byref(n), None, None) == 0 and n.value > 0


@pytest.mark.parametrize("name", ["dubiner_2d_k3.txt", "dubiner_3d_k2.txt"])
def test_basis_matches_golden_exact_values(name):
    """Stored exact-rational Gram-Schmidt basis values (tests/golden/make_golden.py)."""
    from fractions import Fraction
    lines = open(os.path.join(ROOT, "tests", "golden", name)).read().split("\n")
    dim, k = map(int, lines[0].split())
    for ln in lines[1:]:
        if not ln.strip():
            continue
        tok = ln.split()
        pt = np.array([[float(Fraction(t)) for t in tok[:dim]]])
        ref = np.array([float(t) for t in tok[dim:]])
        v, _ = dg.eval_basis(dim, k, pt)
        assert np.abs(v[0] - ref).max() < 1e-14 * max(1.0, np.abs(ref).max())
        assert np.abs(R.eval_basis(dim, k, pt)[0] - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())


def test_extrap_argument_errors_before_device_work():
    """Invalid velocity arguments are rejected before any device access."""
    L = dg.lib()
    m = dg.Mesh.box(2, 4, 2)
    w, ua, ub = 4096, 8192, 12288  # never dereferenced: the checks fail first
    assert L.dg_rk_substeps_extrap(m._h, 0, w, 0.01, 1, 0.0, None, 0.0, ub, 1.0, None, None) == -1
    assert L.dg_rk_substeps_extrap(m._h, 0, w, 0.01, 1, 0.0, ua, 0.0, None, 1.0, None, None) == -1
    assert L.dg_rk_substeps_extrap(m._h, 0, w, 0.01, 1, 0.0, ua, 1.0, ub, 1.0, None, None) == -1
    assert L.dg_rk_substeps_extrap(m._h, 0, w, 0.01, 1, 0.0, w, 0.0, ub, 1.0, None, None) == -1
    assert L.dg_rk_substeps_extrap(m._h, 0, w, 0.01, 1, float("nan"), ua, 0.0, ub, 1.0, None,
                                   None) == -1


def test_richardson_argument_errors_before_device_work():
    L = dg.lib()
    m = dg.Mesh.box(2, 4, 2)
    v, g, u = 4096, 8192, 12288  # never dereferenced: the checks fail first
    f = L.dg_richardson
    assert f(m._h, 0, v, g, None, 0.1, 0.5, 1e-6, 10, None, None, None, None) == -1
    assert f(m._h, 0, v, v, u, 0.1, 0.5, 1e-6, 10, None, None, None, None) == -1
    assert f(m._h, 0, v, g, u, 0.1, 0.0, 1e-6, 10, None, None, None, None) == -1
    assert f(m._h, 0, v, g, u, 0.1, 0.5, -1.0, 10, None, None, None, None) == -1
    assert f(m._h, 0, v, g, u, 0.1, 0.5, 1e-6, -1, None, None, None, None) == -1
    assert f(m._h, 1, v, g, u, 0.1, 0.5, 1e-6, 10, None, None, None, None) == -4  # FP32


@pytest.mark.parametrize("dim,N,per,jit", [(2, 4, (False, True), 0.2),
                                           (3, 2, (False, True, False), 0.1)])
def test_boundary_facets_and_points_match_the_oracle(dim, N, per, jit):
    """Bounded directions (period <= 0): the library finds the same boundary facets as the
    oracle, in the same order, and places their quadrature points at the same physical
    points (the order the outer values are given in)."""
    from oracle.dg import Space
    from oracle.mesh import box_mesh
    om = box_mesh(dim, N, jitter=jit, seed=3, periodic=per)
    sp = Space(om, 2)
    E = om.E
    m = dg.Mesh.from_arrays(dim, 2, om.X.reshape(-1, dim),
                            np.arange(E * (dim + 1)).reshape(E, dim + 1),
                            np.where(per, 1.0, 0.0))
    assert m.info["n_bfacet"] == len(om.bfacets)
    assert m.info["n_facet"] == (E * (dim + 1) + len(om.bfacets)) // 2
    nbr, nbf = m.neighbors()
    bnd = nbr < 0
    assert np.array_equal(bnd, om.nbr < 0)
    assert np.array_equal(-1 - nbr[bnd], om.bf_id[bnd])
    assert np.array_equal(nbr[~bnd], om.nbr[~bnd])
    assert np.abs(m.boundary_points() - sp.boundary_points()).max() < 1e-14


def test_boundary_mesh_needs_the_bc_entry_points():
    """Errors raised before any device work."""
    from oracle.mesh import box_mesh
    om = box_mesh(2, 3, periodic=(False, True))
    E = om.E
    m = dg.Mesh.from_arrays(2, 1, om.X.reshape(-1, 2), np.arange(E * 3).reshape(E, 3),
                            np.array([0.0, 1.0]))
    L = dg.lib()
    w, r, u = 4096, 8192, 12288
    assert L.dg_convection_apply(m._h, 0, w, None, r, None) == -1
    assert L.dg_rk_substeps(m._h, 0, w, 0.01, 1, None, None, None) == -1
    assert L.dg_convection_apply_bc(m._h, 0, w, None, None, None, r, None) == -1  # no wb
    assert L.dg_convection_apply_bc(m._h, 0, w, u, 16384, None, r, None) == -1  # frozen, no ub
    assert L.dg_rk_substeps_extrap(m._h, 0, w, 0.01, 1, 0.0, u, 0.0, 16384, 1.0, None,
                                   None) == -4
    assert L.dg_richardson(m._h, 0, w, 16384, u, 0.1, 0.5, 1e-6, 3, None, None, None,
                           None) == -4


def test_surrogate_rejects_meshes_with_boundary_facets():
    """The network's inputs gather the neighbour across every facet, so a mesh with boundary
    facets is refused at creation, before any device work (and other element types too)."""
    from oracle.mesh import box_mesh
    om = box_mesh(2, 4, periodic=(False, True))
    E = om.E
    m = dg.Mesh.from_arrays(2, 3, om.X.reshape(-1, 2), np.arange(E * 3).reshape(E, 3),
                            np.array([0.0, 1.0]))
    assert m.info["n_bfacet"] > 0
    h = ctypes.c_void_p()
    assert dg.lib().dg_surrogate_create(m._h, 8, ctypes.byref(h)) == -4
    assert b"boundary" in dg.lib().dg_last_error()
    assert not h.value
    m2 = dg.Mesh.box(2, 4, 2)
    assert dg.lib().dg_surrogate_create(m2._h, 8, ctypes.byref(h)) == -4
    assert not h.value


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (2, 4), (2, 6), (3, 1), (3, 2), (3, 3), (3, 4)])
def test_hdiv_reference_basis_matches_the_oracle(dim, k):
    """The library's reference dual basis (long double Gauss-Jordan of its own moment matrix)
    equals the oracle's (NumPy inverse), dof by dof."""
    from oracle import refelem as R
    from oracle.hdiv import reference_dual
    nb = R.n_basis(dim, k)
    tab = np.zeros((dim * nb, dim, nb))
    assert dg.lib().dg_hdiv_reference(dim, k, dg._ptr(tab)) == 0
    C = reference_dual(dim, k)  # [(a, m), j]
    ref = C.T.reshape(-1, dim, nb)
    assert np.abs(tab - ref).max() < 1e-9 * np.abs(ref).max()
    assert dg.lib().dg_hdiv_reference(dim, 7 if dim == 2 else 5, dg._ptr(tab)) == -1


def test_hdiv_size_matches_the_oracle():
    from oracle.hdiv import HdivSpace
    from oracle.mesh import box_mesh
    for dim, per, k in [(2, (True, True), 3), (2, (False, True), 3), (3, (True, True, True), 2),
                        (3, (False, True, False), 3)]:
        om = box_mesh(dim, 4 if dim == 2 else 2, jitter=0.1, seed=2, periodic=per)
        E = om.E
        m = dg.Mesh.from_arrays(dim, k, om.X.reshape(-1, dim),
                                np.arange(E * (dim + 1)).reshape(E, dim + 1),
                                np.where(per, 1.0, 0.0))
        H = HdivSpace(om, k)
        assert m.hdiv_size() == (H.N, H.n_facets)
    m0 = dg.Mesh.box(2, 2, 0)  # k = 0 has no H(div) space
    with pytest.raises(dg.DGError) as e:
        m0.hdiv_size()
    assert e.value.status == -1


def test_reduce_noalloc_errors_before_device_work():
    """dg_reduce_noalloc allocates nothing: a mesh above the static array's size and a mesh
    whose tables are not resident yet are refused before any device call."""
    L = dg.lib()
    a, out = 4096, 8192  # never dereferenced: the checks fail first
    big = dg.Mesh.box(2, 2049, 0)  # 8 396 802 triangles, above 8 388 608
    assert L.dg_reduce_noalloc(big._h, 1, a, None, out, None) == -1
    assert b"too large" in L.dg_last_error()
    del big
    m = dg.Mesh.box(2, 4, 2)
    assert L.dg_reduce_noalloc(m._h, 1, a, None, out, None) == -1
    assert b"resident" in L.dg_last_error()
    assert L.dg_reduce_noalloc(m._h, 3, a, None, out, None) == -1  # L2DIFF without b
    assert L.dg_reduce_noalloc(m._h, 9, a, None, out, None) == -1  # unknown reduction
    assert L.dg_reduce_noalloc(m._h, 1, None, None, out, None) == -1


def _simplex_moment(e):
    """int over the reference simplex of prod x_a^e_a = prod e_a! / (sum e + dim)!"""
    from math import factorial
    num = 1
    for a in e:
        num *= factorial(a)
    return num / factorial(sum(e) + len(e))


@pytest.mark.parametrize("dim,k", [(2, k) for k in range(7)] + [(3, k) for k in range(5)])
def test_volume_rule_exact_to_the_volume_integrand_degree(dim, k):
    """The library's volume rule integrates every monomial of degree <= 3k-1 (the degree of the
    volume integrand (u (x) w) : grad phi) exactly, against the closed form; positive weights,
    points inside the simplex; the symmetric rules are invariant under every permutation of
    the vertices and need fewer points than the collapsed rule of ceil(3k/2) per direction."""
    pts, wts = dg.volume_rule(dim, k)
    deg = max(0, 3 * k - 1)
    n_coll = max(1, (3 * k + 1) // 2) ** dim
    assert pts.shape == (len(wts), dim) and len(wts) <= n_coll
    for e in itertools.product(range(deg + 1), repeat=dim):
        if sum(e) > deg:
            continue
        got = float(np.sum(wts * np.prod(pts ** np.array(e), axis=1)))
        ex = _simplex_moment(e)
        assert abs(got - ex) <= 2e-15 * ex * max(1, len(wts)) ** 0.5, (e, got, ex)
    bary = np.concatenate([1 - pts.sum(1, keepdims=True), pts], 1)
    assert np.all(wts > 0) and bary.min() > 0
    symmetric = (dim, k) in [(2, 1), (2, 2), (2, 3), (2, 4), (2, 5), (3, 1), (3, 2), (3, 3)]
    if symmetric:
        assert len(wts) < n_coll
        key = {tuple(np.round(b, 12)): w for b, w in zip(bary, wts)}
        for perm in itertools.permutations(range(dim + 1)):
            for b, w in zip(bary, wts):
                pb = tuple(np.round(b[list(perm)], 12))
                assert pb in key and abs(key[pb] - w) <= 1e-15, (perm, b)
    m = dg.Mesh.box(dim, 2 if dim == 3 else 3, k)
    assert m.info["nq_vol"] == len(wts)


@pytest.mark.parametrize("dim,k", [(2, 2), (2, 4), (3, 1), (3, 2), (3, 3), (3, 4)])
def test_facet_rule_matches_the_oracle(dim, k):
    """The library's facet rule (part of the operator's definition) is the oracle's point set
    with the oracle's weights (the order of the points may differ)."""
    pts, wts = dg.facet_rule(dim, k)
    op, ow = R.operator_facet_rule(dim, k)
    assert pts.shape == op.shape and abs(wts.sum() - 1.0) < 1e-15
    key = {tuple(np.round(p, 12)): w for p, w in zip(op, ow)}
    for p, w in zip(pts, wts):
        kp = tuple(np.round(p, 12))
        assert kp in key and abs(key[kp] - w) < 1e-15, (p, w)
    m = dg.Mesh.box(dim, 2 if dim == 3 else 3, k)
    assert m.info["nq_facet"] == len(wts)
