"""The H(div)-conforming velocity space W_h and the transfer operators between it and the
DG space V_h (2D), written out plainly.

Test infrastructure (see ``oracle/__init__``).

W_h (Sec. 2.2, the space of element-wise [P^k]^d fields whose normal components are
continuous across facets, e.g. Brezzi-Douglas-Marini) is given the BDM degrees of freedom
(Brezzi-Fortin), k >= 1:
  facet    l_{F,l}(v) = int_F (v . n_F) q_l(s) ds,          l = 0..k,
           n_F the unit outward normal of the lower-numbered element sharing F (a boundary
           facet: of its element), s in [0, 1] along F from its lexicographically first
           vertex, q_l(s) = sqrt(2l+1) P_l(2s-1);
  interior l_{T,r}(v) = sign(det J_T) int_T v . (J_T^-T psi_r(F_T^-1 x)) dx,
           psi_r over a basis of the first-kind Nedelec space N_{k-1} of the reference
           triangle: (x^a y^b, 0), (0, x^a y^b) for a+b <= k-2, and (-y, x) x^a y^b for
           a+b = k-2  (k^2 - 1 functions).
The basis of W_h is dual to these functionals.  Global numbering: the k+1 dofs of each
facet (facets in the order of their lower-numbered element, then local facet), then the
k^2 - 1 interior dofs of each element in element order.

Transfer (Sec. 2.4, eq. l2I): I = (M^V)^-1 M^{U,V} gives the DG coefficients of a W_h field
(exact: W_h is a subspace of V_h on affine meshes); I^T is its transpose, which maps a
functional on V_h (values on the DG basis) to one on W_h.

Construction, per element T with the contravariant Piola map v = J v^(F_T^-1 x) / det J:
a W_h basis function restricted to T is s * Piola(psi^_j), psi^_j the reference dual basis
(inverse of the reference moment matrix over the DG basis e_a phi^_m), s = +-1 from the
facet's normal and parameter orientations and, for facet dofs, sign(det J) (the signed Piola
map carries normal fluxes over with that sign), so
  c_T[i][m] = (1/det J) sum_a J_ia sum_j s_j u_J(j) C[(a, m), j],   C = G^-1.
"""
import numpy as np
from scipy.special import eval_legendre

from . import refelem as R


def n_local(k):
    return (k + 1) * (k + 2)


def _nedelec_basis(k, pts):
    """psi_r at reference points [Q, 2] -> [R, Q, 2] (first-kind Nedelec N_{k-1})."""
    x, y = pts[:, 0], pts[:, 1]
    out = []
    for deg in range(k - 1):
        for a in range(deg, -1, -1):
            b = deg - a
            mono = x ** a * y ** b
            out.append(np.stack([mono, 0 * mono], -1))
            out.append(np.stack([0 * mono, mono], -1))
    for a in range(k - 2, -1, -1):
        b = k - 2 - a
        mono = x ** a * y ** b
        out.append(np.stack([-y * mono, x * mono], -1))
    return np.array(out).reshape(-1, pts.shape[0], 2)


def _legendre01(l, s):
    return np.sqrt(2 * l + 1) * eval_legendre(l, 2 * s - 1)


def reference_dual(k):
    """C = G^-1 with G[j, (a, m)] = the reference dof j of e_a phi^_m: the coefficients
    C[(a, m), j] of the reference dual basis psi^_j on the DG basis.  Reference facet dofs use
    each local facet's ascending local vertices (A -> B) and the reference outward normal."""
    assert k >= 1
    npb = R.n_basis(2, k)
    ndof = n_local(k)
    G = np.zeros((ndof, 2 * npb))
    s, ws = R.facet_rule(2, k + 2)
    s = s[:, 0]
    V = R.ref_vertices(2)
    row = 0
    for f in range(3):
        a, b = [v for v in range(3) if v != f]
        A, B = V[a], V[b]
        t = B - A
        length = np.linalg.norm(t)
        n = np.array([t[1], -t[0]]) / length
        if np.dot(n, V[f] - A) > 0:
            n = -n
        x = A[None, :] + s[:, None] * t[None, :]
        phi = R.eval_basis(2, k, x)  # [Q, Np]
        for l in range(k + 1):
            q = _legendre01(l, s)
            for ai in range(2):
                G[row, ai * npb:(ai + 1) * npb] = length * np.einsum("q,q,qm->m", ws, n[ai] * q, phi)
            row += 1
    p, w = R.collapsed_rule(2, k + 2)
    phi = R.eval_basis(2, k, p)
    psi = _nedelec_basis(k, p)
    for r in range(psi.shape[0]):
        for ai in range(2):
            G[row, ai * npb:(ai + 1) * npb] = np.einsum("q,q,qm->m", w, psi[r, :, ai], phi)
        row += 1
    assert row == ndof
    return np.linalg.inv(G)


class HdivSpace:
    """W_h on a 2D mesh (degree k >= 1), global dof numbering and the transfer operators."""

    def __init__(self, mesh, k):
        assert mesh.dim == 2 and k >= 1
        self.mesh, self.k = mesh, k
        E = mesh.E
        self.npb = R.n_basis(2, k)
        # global facets: owned by the lower-numbered element (or the only one)
        fid = -np.ones((E, 3), dtype=np.int64)
        nf = 0
        for t in range(E):
            for f in range(3):
                nb = mesh.nbr[t, f]
                if nb < 0 or t < nb:
                    fid[t, f] = nf
                    nf += 1
        for t in range(E):
            for f in range(3):
                nb = mesh.nbr[t, f]
                if nb >= 0 and t > nb:
                    fid[t, f] = fid[nb, mesh.nbr_facet[t, f]]
        self.facet_id = fid
        self.n_facets = nf
        self.n_int = k * k - 1
        self.N = nf * (k + 1) + E * self.n_int
        # signs: normal (owner +1) and parameter orientation (local ascending = canonical)
        owner = (mesh.nbr < 0) | (np.arange(E)[:, None] < mesh.nbr)
        self.sig_n = np.where(owner, 1.0, -1.0)
        asc0 = np.array([[v for v in range(3) if v != f][0] for f in range(3)])
        self.sig_t = np.where(mesh.canon_idx[:, :, 0] == asc0[None, :], 1.0, -1.0)
        self.C = reference_dual(k)

    def local_dofs(self, t):
        """Global ids and signs of the local dofs of element t (reference dof order)."""
        k = self.k
        ids, sg = [], []
        # the signed Piola map carries normal fluxes over with sign(det J): the divergence
        # theorem on T and on the reference element give v.n ds = sign(det J) v^.n^ ds^
        sd = np.sign(self.mesh.detJ[t])
        for f in range(3):
            for l in range(k + 1):
                ids.append(self.facet_id[t, f] * (k + 1) + l)
                sg.append(sd * self.sig_n[t, f] * self.sig_t[t, f] ** l)
        base = self.n_facets * (k + 1) + t * self.n_int
        ids += list(range(base, base + self.n_int))
        sg += [1.0] * self.n_int
        return np.array(ids), np.array(sg)

    def to_dg(self, u):
        """I u: DG coefficients [E, 2, Np] of the W_h field with coefficients u [N]."""
        m = self.mesh
        out = np.zeros((m.E, 2, self.npb))
        Cr = self.C.reshape(2, self.npb, -1)  # [a, m, j]
        for t in range(m.E):
            ids, sg = self.local_dofs(t)
            ref = np.einsum("amj,j->am", Cr, sg * u[ids])  # reference field's coefficients
            out[t] = np.einsum("ia,am->im", m.J[t], ref) / m.detJ[t]
        return out

    def transpose(self, F):
        """I^T F for F [E, 2, Np] (a functional's values on the DG basis) -> [N]."""
        m = self.mesh
        out = np.zeros(self.N)
        Cr = self.C.reshape(2, self.npb, -1)
        for t in range(m.E):
            ids, sg = self.local_dofs(t)
            G = np.einsum("ia,im->am", m.J[t], F[t]) / m.detJ[t]
            np.add.at(out, ids, sg * np.einsum("amj,am->j", Cr, G))
        return out

    def dofs(self, v, qn=None):
        """The global dof functionals applied to a DG field v [E, 2, Np] directly in physical
        coordinates (facet moments from the owner element's side; interior moments with the
        covariant map).  Returns [N]."""
        m, k = self.mesh, self.k
        qn = qn or k + 3
        out = np.zeros(self.N)
        s, ws = R.facet_rule(2, qn)
        s = s[:, 0]
        for t in range(m.E):
            for f in range(3):
                nb = m.nbr[t, f]
                if not (nb < 0 or t < nb):
                    continue  # the owner's side computes the facet's moments
                A, B = m.canon[t, f, 0], m.canon[t, f, 1]
                x = A[None, :] + s[:, None] * (B - A)[None, :]
                xi = np.linalg.solve(m.J[t], (x - m.X[t, 0]).T).T
                vals = np.einsum("qm,im->qi", R.eval_basis(2, k, xi), v[t])
                vn = vals @ m.normal[t, f]
                for l in range(k + 1):
                    out[self.facet_id[t, f] * (k + 1) + l] = m.area[t, f] * np.sum(
                        ws * vn * _legendre01(l, s))
        p, w = R.collapsed_rule(2, qn)
        psi = _nedelec_basis(k, p)  # [R, Q, 2] at reference points
        phi = R.eval_basis(2, k, p)
        for t in range(m.E):
            vals = np.einsum("qm,im->qi", phi, v[t])
            cov = np.einsum("ji,rqj->rqi", m.Jinv[t], psi)  # J^-T psi
            base = self.n_facets * (k + 1) + t * self.n_int
            out[base:base + self.n_int] = np.sign(m.detJ[t]) * m.absdetJ[t] * np.einsum(
                "q,qi,rqi->r", w, vals, cov)
        return out
