"""Affine simplicial meshes of a box, periodic or bounded in each direction, for the oracle.

Test infrastructure (see ``oracle/__init__``).

A mesh is given by the unwrapped vertex coordinates of every element, X[T, a, :] for local
vertex a = 0..d, and the period vector L of the box.  The local vertex order defines the
element map F_T(xi) = X[T,0] + J_T xi with J_T = [X1-X0, ..., Xd-X0]; coefficients refer to
the Dubiner basis pulled back through F_T, so the vertex order is part of the data and is
never changed.

Local facet f is the facet opposite local vertex f.  Facets of two elements are matched by
their centroids modulo the period (a KD-tree with periodic box), so the oracle needs no vertex
numbering at all.  A period entry <= 0 marks a bounded direction: facets left unmatched there
are boundary facets (nbr = -1), numbered in (element, local facet) order.

Canonical facet orientation: the facet's vertices sorted lexicographically by coordinate.  The
order is invariant under the periodic translation that relates the two sides, so both sides
place the facet quadrature points at the same physical points.
"""
import itertools

import numpy as np
from scipy.spatial import cKDTree


class Mesh:
    """Element geometry + facet connectivity, all plain arrays."""

    def __init__(self, X, period):
        X = np.asarray(X, dtype=np.float64)
        self.X = X
        self.E, nv, self.dim = X.shape
        d = self.dim
        assert nv == d + 1
        self.period = np.asarray(period, dtype=np.float64)
        # Jacobian of the affine map, its inverse and |det|
        self.J = np.stack([X[:, a + 1, :] - X[:, 0, :] for a in range(d)], axis=2)  # [E,d,d]
        self.detJ = np.linalg.det(self.J)
        self.absdetJ = np.abs(self.detJ)
        self.Jinv = np.linalg.inv(self.J)
        self.h = None
        self._facets()

    def facet_vertices(self, f):
        """Local vertex ids of local facet f (opposite vertex f), ascending."""
        return [a for a in range(self.dim + 1) if a != f]

    def _facets(self):
        d, E = self.dim, self.E
        nf = d + 1
        # physical facet data per (T, f)
        cen = np.zeros((E, nf, d))
        normal = np.zeros((E, nf, d))
        area = np.zeros((E, nf))
        canon = np.zeros((E, nf, d, d))  # canonical vertex coordinates (unwrapped, own frame)
        canon_idx = np.zeros((E, nf, d), dtype=np.int64)  # their local vertex ids
        for f in range(nf):
            V = self.X[:, self.facet_vertices(f), :]  # [E, d, d]
            cen[:, f] = V.mean(axis=1)
            if d == 2:
                t = V[:, 1] - V[:, 0]
                nvec = np.stack([t[:, 1], -t[:, 0]], axis=1)
                meas = np.linalg.norm(t, axis=1)
            else:
                nvec = np.cross(V[:, 1] - V[:, 0], V[:, 2] - V[:, 0])
                meas = 0.5 * np.linalg.norm(nvec, axis=1)
            nvec = nvec / np.linalg.norm(nvec, axis=1)[:, None]
            # outward: pointing away from the opposite vertex
            opp = self.X[:, f, :] - V[:, 0]
            sgn = np.sign(np.einsum("ej,ej->e", nvec, opp))
            normal[:, f] = -sgn[:, None] * nvec
            area[:, f] = meas
            canon[:, f], order = _lex_sort_vertices(V)
            canon_idx[:, f] = np.array(self.facet_vertices(f))[order]
        self.centroid = cen
        self.normal = normal
        self.area = area
        self.canon = canon
        self.canon_idx = canon_idx
        # match facets by centroid modulo the period (bounded directions: no wrap, a box far
        # larger than the mesh so the tree never wraps them either)
        per = self.period > 0
        flat = cen.reshape(-1, d).copy()
        lo = flat.min(axis=0)
        ext = flat.max(axis=0) - lo
        box = np.where(per, self.period, 4.0 * ext + 4.0)
        flat = np.where(per, flat % np.where(per, self.period, 1.0), flat - lo + ext + 1.0)
        flat = np.where(per & (np.abs(flat - box) < 1e-12 * box), 0.0, flat)
        tree = cKDTree(flat, boxsize=box)
        dist, idx = tree.query(flat, k=2)
        hmin = np.min(area) if d == 2 else np.sqrt(np.min(area))
        self_idx = np.arange(flat.shape[0])
        other = np.where(idx[:, 0] == self_idx, idx[:, 1], idx[:, 0])
        dd = np.where(idx[:, 0] == self_idx, dist[:, 1], dist[:, 0])
        matched = dd < 1e-8 * hmin
        if per.all() and not matched.all():
            raise ValueError("unmatched facet: mesh is not periodic-conforming")
        # a facet's nearest other facet must match it back, else it lies on the boundary
        matched &= other[np.where(matched, other, self_idx)] == self_idx
        other = np.where(matched, other, -1)
        self.nbr = np.where(matched, other // nf, -1).reshape(E, nf)
        self.nbr_facet = np.where(matched, other % nf, -1).reshape(E, nf)
        # boundary facets in (element, local facet) order
        self.bfacets = np.argwhere(~matched.reshape(E, nf))  # [nb, 2]: (T, f)
        self.bf_id = np.full((E, nf), -1, dtype=np.int64)
        self.bf_id[self.bfacets[:, 0], self.bfacets[:, 1]] = np.arange(len(self.bfacets))
        # periodic shift taking the neighbour's unwrapped frame onto ours: x_own = x_nbr + shift
        Nn = np.where(self.nbr >= 0, self.nbr, np.arange(E)[:, None])
        Ff = np.where(self.nbr >= 0, self.nbr_facet, np.arange(nf)[None, :])
        self.shift = cen - cen[Nn, Ff]
        self.h = hmin


def _lex_sort_vertices(V, rtol=1e-10):
    """Sort the d vertices of each facet lexicographically by coordinate. V: [E, d, d].

    Returns the sorted coordinates and, per facet, the positions (0..d-1) of the sorted
    vertices in the input order."""
    E, nvert, d = V.shape
    scale = np.max(np.abs(V[:, 1:] - V[:, :1])) + 1e-300
    tol = rtol * scale
    out = V.copy()
    order = np.tile(np.arange(nvert), (E, 1))
    # simple insertion sort over the (at most 3) vertices, vectorised over facets
    for i in range(1, nvert):
        for j in range(i, 0, -1):
            a = out[:, j - 1].copy()
            b = out[:, j].copy()
            swap = np.zeros(E, dtype=bool)
            decided = np.zeros(E, dtype=bool)
            for c in range(d):
                gt = (a[:, c] > b[:, c] + tol) & ~decided
                lt = (a[:, c] < b[:, c] - tol) & ~decided
                swap |= gt
                decided |= gt | lt
            out[swap, j - 1] = b[swap]
            out[swap, j] = a[swap]
            oa = order[:, j - 1].copy()
            order[swap, j - 1] = order[swap, j]
            order[swap, j] = oa[swap]
    return out, order


def box_mesh(dim, N, jitter=0.0, seed=0, periodic=None):
    """Unit box, N^d squares split in 2 triangles / cubes split in 6 tetrahedra; periodic in
    every direction unless `periodic` (one flag per direction) says otherwise.

    2D: square (i,j) -> lower (v00, v10, v11), id 2(jN+i); upper (v11, v01, v00), id 2(jN+i)+1.
    3D: cube (i,j,l), index (lN+j)N+i, Kuhn split along v000 -> v111: tet s = (v000,
        v000+e_s0, v000+e_s0+e_s1, v111) for the permutations s of (x,y,z) in lexicographic
        order; id 6*cube + index(s).
    `jitter` > 0 displaces every lattice vertex by a seeded periodic random offset of that
    size times h (identified vertices move together), giving a general affine mesh; vertices
    on a bounded side stay on it.
    """
    periodic = np.ones(dim, dtype=bool) if periodic is None else np.asarray(periodic, bool)
    h = 1.0 / N
    rng = np.random.default_rng(seed)
    shape = tuple(N if periodic[a] else N + 1 for a in range(dim))
    off = rng.uniform(-1, 1, size=shape + (dim,)) * jitter * h if jitter else None
    if off is not None:
        for a in range(dim):
            if not periodic[a]:  # keep the bounded sides straight
                sl = [slice(None)] * dim
                sl[a] = 0
                off[tuple(sl) + (a,)] = 0.0
                sl[a] = N
                off[tuple(sl) + (a,)] = 0.0

    def vert(idx):  # idx: [..., dim] integer lattice coordinates (unwrapped)
        x = idx * h
        if off is not None:
            w = np.where(periodic, np.mod(idx, N), idx)
            x = x + off[tuple(w[..., a] for a in range(dim))]
        return x

    if dim == 2:
        j, i = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
        base = np.stack([i.ravel(), j.ravel()], axis=1)  # square index jN+i
        v00, v10 = base, base + [1, 0]
        v11, v01 = base + [1, 1], base + [0, 1]
        lower = np.stack([v00, v10, v11], axis=1)
        upper = np.stack([v11, v01, v00], axis=1)
        lat = np.stack([lower, upper], axis=1).reshape(-1, 3, 2)
    else:
        l, j, i = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
        base = np.stack([i.ravel(), j.ravel(), l.ravel()], axis=1)  # cube index (lN+j)N+i
        eye = np.eye(3, dtype=np.int64)
        tets = []
        for s in itertools.permutations(range(3)):
            e0, e1 = eye[s[0]], eye[s[1]]
            tets.append(np.stack([base, base + e0, base + e0 + e1, base + 1], axis=1))
        lat = np.stack(tets, axis=1).reshape(-1, 4, 3)
    return Mesh(vert(lat), np.where(periodic, 1.0, 0.0))
