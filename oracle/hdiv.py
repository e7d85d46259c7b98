"""The H(div)-conforming velocity space W_h and the transfer operators between it and the
DG space V_h (2D and 3D), written out plainly.

Test infrastructure (see ``oracle/__init__``).

W_h (Sec. 2.2, the space of element-wise [P^k]^d fields whose normal components are
continuous across facets, e.g. Brezzi-Douglas-Marini) is given the BDM degrees of freedom
(Brezzi-Fortin), k >= 1:
  facet    l_{F,l}(v) = int_F (v . n_F) q_l(s) ds,   l over an L2-orthonormal basis of P^k(F),
           n_F the unit outward normal of the lower-numbered element sharing F (a boundary
           facet: of its element), s the facet parameter from its canonical vertices (the
           mesh's lexicographic order: A + s (B - A) [+ t (C - A)]);
           2D: q_l(s) = sqrt(2l+1) P_l(2s-1), l = 0..k;
           3D: q_l(s, t) = phi^_l(s, t) / sqrt(2), the orthonormal DG basis of the reference
           triangle scaled to unit mean square, (k+1)(k+2)/2 functions;
  interior l_{T,r}(v) = sign(det J_T) int_T v . (J_T^-T psi_r(F_T^-1 x)) dx,
           psi_r over a basis of the first-kind Nedelec space N_{k-1} of the reference
           simplex, [P^{k-2}]^d + {x -> x ^ q : q homogeneous of degree k-2}:
           2D: (x^a y^b, 0), (0, x^a y^b) for a+b <= k-2, then (-y, x) x^a y^b for a+b = k-2
               (k^2 - 1 functions);
           3D: e_i m for the monomials m of degree <= k-2, then x ^ (e_i m) for the monomials
               m of degree k-2, leaving out i = 0 when x divides m (x ^ (e_0 x q) is a
               combination of the other two); (k-1)(k+1)(k+2)/2 functions;
           monomials x^a y^b z^c by degree, then a descending, then b descending; for each
           monomial i = 0..d-1.
The basis of W_h is dual to these functionals.  Global numbering: the dofs of each facet
(facets in the order of their lower-numbered element, then local facet), then the interior
dofs of each element in element order.

Transfer (Sec. 2.4, eq. l2I): I = (M^V)^-1 M^{U,V} gives the DG coefficients of a W_h field
(exact: W_h is a subspace of V_h on affine meshes); I^T is its transpose, which maps a
functional on V_h (values on the DG basis) to one on W_h.

Construction, per element T with the contravariant Piola map v = J v^(F_T^-1 x) / det J:
a W_h basis function restricted to T is Piola(sum_j P_jJ psi^_j), psi^_j the reference dual
basis (inverse of the reference moment matrix over the DG basis e_a phi^_m, facet moments in
each local facet's ascending-vertex parameter and reference outward normal) and P the local
map of element T: on the dofs of local facet f, sign(det J) (the signed Piola map carries
normal fluxes over with that sign) times +-1 (owner normal or not) times Q, the change from
the canonical to the local facet parameter of the orthonormal facet basis, q_l(local) =
sum_i Q_li q_i(canonical); the identity on the interior dofs.  So
  c_T[i][m] = (1/det J) sum_a J_ia sum_j C[(a, m), j] (P u)_j,   C = G^-1.
"""
import numpy as np
from scipy.special import eval_legendre

from . import refelem as R


def n_facet_dofs(dim, k):
    return k + 1 if dim == 2 else (k + 1) * (k + 2) // 2


def n_local(dim, k):
    return dim * R.n_basis(dim, k)


def n_interior(dim, k):
    return n_local(dim, k) - (dim + 1) * n_facet_dofs(dim, k)


def _monomials(dim, deg):
    """Exponent tuples of the monomials of degree deg: a descending, then b descending."""
    out = []
    for a in range(deg, -1, -1):
        if dim == 2:
            out.append((a, deg - a))
        else:
            for b in range(deg - a, -1, -1):
                out.append((a, b, deg - a - b))
    return out


def _mono(pts, e):
    v = np.ones(pts.shape[0])
    for c, p in enumerate(e):
        v = v * pts[:, c] ** p
    return v


def _nedelec_basis(dim, k, pts):
    """psi_r at reference points [Q, d] -> [R, Q, d] (first-kind Nedelec N_{k-1})."""
    Q = pts.shape[0]
    out = []
    for deg in range(k - 1):
        for e in _monomials(dim, deg):
            m = _mono(pts, e)
            for i in range(dim):
                v = np.zeros((Q, dim))
                v[:, i] = m
                out.append(v)
    if k >= 2:
        for e in _monomials(dim, k - 2):
            m = _mono(pts, e)
            if dim == 2:
                out.append(np.stack([-pts[:, 1] * m, pts[:, 0] * m], -1))
                continue
            for i in range(dim):
                if i == 0 and e[0] >= 1:
                    continue  # x ^ (e_0 x q) is a combination of the other two
                ei = np.zeros(3)
                ei[i] = 1.0
                out.append(np.cross(pts, ei[None, :]) * m[:, None])
    out = np.array(out).reshape(-1, Q, dim)
    assert out.shape[0] == n_interior(dim, k)
    return out


def facet_tests(dim, k, s):
    """The orthonormal facet basis q_l at facet parameters s [Q, d-1] -> [Q, nfd]."""
    if dim == 2:
        return np.stack([np.sqrt(2 * l + 1) * eval_legendre(l, 2 * s[:, 0] - 1)
                         for l in range(k + 1)], axis=1)
    return R.eval_basis(2, k, s) / np.sqrt(2.0)


def _barycentric(s):
    """Facet barycentric coordinates (1 - sum s, s_1, ...) of parameters s [Q, d-1]."""
    return np.concatenate([1.0 - s.sum(axis=1, keepdims=True), s], axis=1)


def orientation_matrix(dim, k, pos):
    """Q with q_l(local parameter) = sum_i Q_li q_i(canonical parameter) on a facet whose
    canonical vertex j is the local-ascending vertex pos[j]."""
    s, w = R.facet_rule(dim, k + 2)
    lam_c = _barycentric(s)
    lam_l = np.zeros_like(lam_c)
    for j in range(dim):
        lam_l[:, pos[j]] = lam_c[:, j]
    ql = facet_tests(dim, k, lam_l[:, 1:])
    qc = facet_tests(dim, k, s)
    return np.einsum("q,ql,qi->li", w, ql, qc)


def reference_dual(dim, k):
    """C = G^-1 with G[j, (a, m)] = the reference dof j of e_a phi^_m: the coefficients
    C[(a, m), j] of the reference dual basis psi^_j on the DG basis.  Reference facet dofs use
    each local facet's ascending local vertices and the reference outward normal."""
    assert k >= 1
    npb = R.n_basis(dim, k)
    ndof = n_local(dim, k)
    nfd = n_facet_dofs(dim, k)
    G = np.zeros((ndof, dim * npb))
    s, ws = R.facet_rule(dim, k + 2)
    V = R.ref_vertices(dim)
    row = 0
    for f in range(dim + 1):
        vs = [v for v in range(dim + 1) if v != f]
        A = V[vs[0]]
        edges = [V[v] - A for v in vs[1:]]
        if dim == 2:
            t = edges[0]
            meas = np.linalg.norm(t)
            n = np.array([t[1], -t[0]]) / meas
        else:
            c = np.cross(edges[0], edges[1])
            meas = 0.5 * np.linalg.norm(c)
            n = c / np.linalg.norm(c)
        if np.dot(n, V[f] - A) > 0:
            n = -n
        x = A[None, :] + sum(s[:, a:a + 1] * edges[a][None, :] for a in range(dim - 1))
        phi = R.eval_basis(dim, k, x)  # [Q, Np]
        q = facet_tests(dim, k, s)
        for l in range(nfd):
            for ai in range(dim):
                G[row, ai * npb:(ai + 1) * npb] = meas * np.einsum("q,q,qm->m", ws, n[ai] * q[:, l], phi)
            row += 1
    p, w = R.collapsed_rule(dim, k + 2)
    phi = R.eval_basis(dim, k, p)
    psi = _nedelec_basis(dim, k, p)
    for r in range(psi.shape[0]):
        for ai in range(dim):
            G[row, ai * npb:(ai + 1) * npb] = np.einsum("q,q,qm->m", w, psi[r, :, ai], phi)
        row += 1
    assert row == ndof
    return np.linalg.inv(G)


class HdivSpace:
    """W_h on a 2D or 3D mesh (degree k >= 1), global dof numbering and the transfer
    operators."""

    def __init__(self, mesh, k):
        assert mesh.dim in (2, 3) and k >= 1
        self.mesh, self.k = mesh, k
        d = mesh.dim
        E, nf = mesh.E, d + 1
        self.npb = R.n_basis(d, k)
        self.nfd = n_facet_dofs(d, k)
        # global facets: owned by the lower-numbered element (or the only one)
        fid = -np.ones((E, nf), dtype=np.int64)
        n_f = 0
        for t in range(E):
            for f in range(nf):
                nb = mesh.nbr[t, f]
                if nb < 0 or t < nb:
                    fid[t, f] = n_f
                    n_f += 1
        for t in range(E):
            for f in range(nf):
                nb = mesh.nbr[t, f]
                if nb >= 0 and t > nb:
                    fid[t, f] = fid[nb, mesh.nbr_facet[t, f]]
        self.facet_id = fid
        self.n_facets = n_f
        self.n_int = n_interior(d, k)
        self.N = n_f * self.nfd + E * self.n_int
        owner = (mesh.nbr < 0) | (np.arange(E)[:, None] < mesh.nbr)
        self.sig_n = np.where(owner, 1.0, -1.0)
        self.C = reference_dual(d, k)
        self._qcache = {}

    def _orientation(self, t, f):
        asc = self.mesh.facet_vertices(f)
        pos = tuple(asc.index(int(v)) for v in self.mesh.canon_idx[t, f])
        if pos not in self._qcache:
            self._qcache[pos] = orientation_matrix(self.mesh.dim, self.k, pos)
        return self._qcache[pos]

    def local_map(self, t):
        """Global ids of the local dofs of element t (reference dof order) and the local map
        P: the local dof values of a W_h field are P u[ids]."""
        d, nfd = self.mesh.dim, self.nfd
        ids = []
        nl = n_local(d, self.k)
        P = np.zeros((nl, nl))
        sd = np.sign(self.mesh.detJ[t])
        for f in range(d + 1):
            ids += [self.facet_id[t, f] * nfd + l for l in range(nfd)]
            P[f * nfd:(f + 1) * nfd, f * nfd:(f + 1) * nfd] = (
                sd * self.sig_n[t, f] * self._orientation(t, f))
        base = self.n_facets * nfd + t * self.n_int
        ids += list(range(base, base + self.n_int))
        o = (d + 1) * nfd
        P[o:, o:] = np.eye(self.n_int)
        return np.array(ids), P

    def to_dg(self, u):
        """I u: DG coefficients [E, d, Np] of the W_h field with coefficients u [N]."""
        m = self.mesh
        d = m.dim
        out = np.zeros((m.E, d, self.npb))
        Cr = self.C.reshape(d, self.npb, -1)  # [a, m, j]
        for t in range(m.E):
            ids, P = self.local_map(t)
            ref = np.einsum("amj,j->am", Cr, P @ u[ids])  # reference field's coefficients
            out[t] = np.einsum("ia,am->im", m.J[t], ref) / m.detJ[t]
        return out

    def transpose(self, F):
        """I^T F for F [E, d, Np] (a functional's values on the DG basis) -> [N]."""
        m = self.mesh
        d = m.dim
        out = np.zeros(self.N)
        Cr = self.C.reshape(d, self.npb, -1)
        for t in range(m.E):
            ids, P = self.local_map(t)
            G = np.einsum("ia,im->am", m.J[t], F[t]) / m.detJ[t]
            np.add.at(out, ids, P.T @ np.einsum("amj,am->j", Cr, G))
        return out

    def dofs(self, v, qn=None):
        """The global dof functionals applied to a DG field v [E, d, Np] directly in physical
        coordinates (facet moments from the owner element's side in the canonical facet
        parameter; interior moments with the covariant map).  Returns [N]."""
        m, k = self.mesh, self.k
        d, nfd = m.dim, self.nfd
        qn = qn or k + 3
        out = np.zeros(self.N)
        s, ws = R.facet_rule(d, qn)
        q = facet_tests(d, k, s)
        for t in range(m.E):
            for f in range(d + 1):
                nb = m.nbr[t, f]
                if not (nb < 0 or t < nb):
                    continue  # the owner's side computes the facet's moments
                A = m.canon[t, f, 0]
                x = A[None, :] + sum(s[:, a:a + 1] * (m.canon[t, f, a + 1] - A)[None, :]
                                     for a in range(d - 1))
                xi = np.linalg.solve(m.J[t], (x - m.X[t, 0]).T).T
                vals = np.einsum("qm,im->qi", R.eval_basis(d, k, xi), v[t])
                vn = vals @ m.normal[t, f]
                base = self.facet_id[t, f] * nfd
                out[base:base + nfd] = m.area[t, f] * np.einsum("q,q,ql->l", ws, vn, q)
        p, w = R.collapsed_rule(d, qn)
        psi = _nedelec_basis(d, k, p)  # [R, Q, d] at reference points
        phi = R.eval_basis(d, k, p)
        for t in range(m.E):
            vals = np.einsum("qm,im->qi", phi, v[t])
            cov = np.einsum("ji,rqj->rqi", m.Jinv[t], psi)  # J^-T psi
            base = self.n_facets * nfd + t * self.n_int
            out[base:base + self.n_int] = np.sign(m.detJ[t]) * m.absdetJ[t] * np.einsum(
                "q,qi,rqi->r", w, vals, cov)
        return out
