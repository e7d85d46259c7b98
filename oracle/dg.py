"""The upwind-DG convection operator, its SSP-RK3 substeps and helpers, written out plainly.

Test infrastructure (see ``oracle/__init__``).

State layout: coefficients c[T, i, m] (element T, velocity component i, basis function m of the
orthonormal Dubiner basis pulled back through the element map), FP64.

Operator (Sec. 2.3, upwind trilinear form; Sec. 2.4, discrete operator C^V; Sec. 3.2,
propagation problem):

    C_h(u; w, z) = sum_T [ - int_T (w (x) u) : grad z dx + int_{dT} (u.n) w^ z ds ]
    r = -(M^V)^-1 C^V(u) w          (the time derivative in  ds w + (M^V)^-1 C^V w = 0)

with w^ the upwind value (the trace of w taken from the side the flow comes from) and M^V the
DG mass matrix, diagonal for an L2-orthogonal basis (Sec. 2.3).

Readings where the paper leaves the hot path open:
  * The paper's convecting velocity is H(div)-conforming, so u.n is single-valued.  For a
    discontinuous convecting field we use the facet-averaged normal velocity
    beta = 1/2 (u^- + u^+) . n^-, and w^ = w^- if beta > 0 else w^+ (at beta = 0 the flux is 0
    for either choice).
  * "Self" mode u := w gives the nonlinear div(w (x) w); a caller-given u gives the linear
    operator C^V(u) of the propagation problem with frozen convection.
  * The upwind value is taken pointwise at the facet quadrature points, so the facet rule
    (refelem.operator_facet_rule, canonical orientation from mesh.Mesh) is part of the
    definition: Gauss-Legendre points on an edge; on a triangle, the symmetric rule of degree
    3k (k = 2, 3: 12 and 19 points) where it needs fewer points than the collapsed rule.
  * Time integrator: three-stage SSP-RK3 (Shu-Osher form); the paper leaves the explicit
    integrator of the propagation problem generic.
"""
import numpy as np

from . import refelem as R


class Space:
    """Vector DG space V_h = prod_T [P^k(T)]^d on a mesh, with the oracle's quadrature."""

    def __init__(self, mesh, k, chunk=8192):
        self.mesh = mesh
        self.k = k
        self.dim = d = mesh.dim
        self.np = R.n_basis(d, k)
        self.vq, self.vw = R.collapsed_rule(d, R.volume_points_for_oracle(k))
        self.phi_v = R.eval_basis(d, k, self.vq)  # [Q, Np]
        self.dphi_v = R.eval_grad(d, k, self.vq)  # [Q, Np, d]
        self.fq, self.fw = R.operator_facet_rule(d, k)  # [Qf, d-1], weights sum to 1
        self.chunk = chunk
        # the diagonal of M^V: int_T phi_m phi_m dx, by quadrature on every element
        self.mass = mesh.absdetJ[:, None] * np.einsum("q,qm,qm->m", self.vw, self.phi_v,
                                                      self.phi_v)[None, :]
        self._cache = {}
        self._cached_bytes = 0

    @property
    def shape(self):
        return (self.mesh.E, self.dim, self.np)

    # ---- facet points ------------------------------------------------------------------
    def facet_points_phys(self, T, f):
        """Physical facet quadrature points of local facet f of elements T (own frame)."""
        V = self.mesh.canon[T, f]  # [n, d, d], canonical vertex order
        x = V[:, None, 0, :] + np.einsum("qc,ncj->nqj", self.fq, V[:, 1:, :] - V[:, None, 0, :])
        return x  # [n, Qf, d]

    def facet_ref_points(self, T, f):
        """The facet quadrature points of local facet f of elements T in their reference
        coordinates: the affine map sends reference vertices to element vertices, so the
        point A + s(B-A) [+ t(C-A)] of the canonically ordered facet vertices is the same
        combination of the corresponding reference vertices (no rounding from J^-1)."""
        vref = R.ref_vertices(self.dim)
        ci = self.mesh.canon_idx[T, f]  # [n, d] local ids in canonical order
        A = vref[ci[:, 0]]
        return A[:, None, :] + np.einsum("qc,ncj->nqj", self.fq, vref[ci[:, 1:]] - A[:, None, :])

    def facet_basis(self, T):
        """phi_m at the facet points, own side and neighbour side: two [n, d+1, Qf, Np]."""
        key = hash(np.ascontiguousarray(T).tobytes())
        if key in self._cache:
            return self._cache[key]
        m, d = self.mesh, self.dim
        own, nbr = [], []
        for f in range(d + 1):
            # boundary facets have no neighbour: the own element stands in (values unused)
            bnd = m.nbr[T, f] < 0
            N = np.where(bnd, T, m.nbr[T, f])
            Nf = np.where(bnd, f, m.nbr_facet[T, f])
            own.append(R.eval_basis(d, self.k, self.facet_ref_points(T, f)))
            nbr.append(R.eval_basis(d, self.k, self.facet_ref_points(N, Nf)))
        out = (np.stack(own, axis=1), np.stack(nbr, axis=1))
        nbytes = len(T) * (d + 1) * len(self.fw) * self.np * 16
        if nbytes < 1e9 and self._cached_bytes + nbytes < 4e9:
            self._cache[key] = out
            self._cached_bytes += nbytes
        return out

    # ---- the operator ------------------------------------------------------------------
    def boundary_points(self):
        """Physical quadrature points of the boundary facets, canonical order: [nb, Qf, d]."""
        bf = self.mesh.bfacets
        if len(bf) == 0:
            return np.zeros((0, len(self.fw), self.dim))
        out = np.empty((len(bf), len(self.fw), self.dim))
        for f in range(self.dim + 1):
            sel = bf[:, 1] == f
            out[sel] = self.facet_points_phys(bf[sel, 0], f)
        return out

    def _outer(self, T, f, pnbr, w, vb):
        """Outer-side values at the points of local facet f of elements T: the neighbour's
        trace, or on boundary facets the given values vb [nb, Qf, d]."""
        m = self.mesh
        N = m.nbr[T, f]
        bnd = N < 0
        vals = np.einsum("tqm,tim->tqi", pnbr[:, f], w[np.where(bnd, T, N)])
        if bnd.any():
            if vb is None:
                raise ValueError("the mesh has boundary facets: boundary values are required")
            vals[bnd] = vb[m.bf_id[T[bnd], f]]
        return vals

    def form(self, w, u=None, elems=None, wb=None, ub=None):
        """C_h(u; w, phi_{T,i,m}) for the test functions of elements `elems` -> [n, d, Np].

        Boundary facets (Sec. 2.3: on the inflow part of the boundary the upwind value comes
        from outside the domain) take the outer values from wb (and the outer convecting
        velocity from ub in frozen mode, from wb in self mode), given at boundary_points();
        the flux formula is the interior one with these outer values."""
        elems = np.arange(self.mesh.E) if elems is None else np.asarray(elems)
        out = np.empty((len(elems), self.dim, self.np))
        for s in range(0, len(elems), self.chunk):
            vol, facs = self._terms(w, u, elems[s:s + self.chunk], wb, ub)
            fac = np.zeros_like(vol)
            for ff in facs:
                fac += ff
            out[s:s + self.chunk] = vol + fac
        return out

    def form_parts(self, w, u=None, elems=None, wb=None, ub=None):
        """The terms of C_h(u; w, phi_{T,i,m}) (Sec. 2.3) separately: the volume term
        -int_T (w (x) u) : grad phi [n, d, Np] and the facet terms int_F (u.n) w^ phi of the
        local facets F [d+1, n, d, Np]; form() is their sum."""
        elems = np.arange(self.mesh.E) if elems is None else np.asarray(elems)
        parts = [self._terms(w, u, elems[s:s + self.chunk], wb, ub)
                 for s in range(0, len(elems), self.chunk)]
        return (np.concatenate([p[0] for p in parts]),
                np.concatenate([np.stack(p[1]) for p in parts], axis=1))

    def _terms(self, w, u, T, wb, ub):
        """Volume term and the list of facet terms of C_h on the elements T (one chunk)."""
        m, d = self.mesh, self.dim
        uu = w if u is None else u
        ubb = wb if u is None else ub
        # volume term: - int_T w_i u_j d_j phi_m dx
        wq = np.einsum("qm,tim->tqi", self.phi_v, w[T])
        uq = np.einsum("qm,tim->tqi", self.phi_v, uu[T])
        grad = np.einsum("tkj,qmk->tqmj", m.Jinv[T], self.dphi_v)  # physical gradients
        conv = np.einsum("tqj,tqmj->tqm", uq, grad)  # u . grad phi_m
        vol = -np.einsum("t,q,tqi,tqm->tim", m.absdetJ[T], self.vw, wq, conv)
        # facet terms: int_F (u.n) w^ phi_m ds with the pointwise upwind value
        pown, pnbr = self.facet_basis(T)
        facs = []
        for f in range(d + 1):
            wm = np.einsum("tqm,tim->tqi", pown[:, f], w[T])
            wp = self._outer(T, f, pnbr, w, wb)
            um = np.einsum("tqm,tim->tqi", pown[:, f], uu[T])
            up = self._outer(T, f, pnbr, uu, ubb)
            beta = 0.5 * np.einsum("tqj,tj->tq", um + up, m.normal[T, f])
            what = np.where(beta[..., None] > 0.0, wm, wp)
            facs.append(np.einsum("t,q,tq,tqi,tqm->tim", m.area[T, f], self.fw, beta, what,
                                  pown[:, f]))
        return vol, facs

    def apply(self, w, u=None, elems=None, wb=None, ub=None):
        """r = -(M^V)^-1 C^V(u) w on elements `elems` (all by default); u=None means u := w.
        wb, ub: boundary values (see form)."""
        elems = np.arange(self.mesh.E) if elems is None else np.asarray(elems)
        return -self.form(w, u, elems, wb, ub) / self.mass[elems][:, None, :]

    def ssprk3(self, w, dt, n, u=None, wb=None, ub=None):
        """n substeps of three-stage SSP-RK3 for ds w = apply(w) (Shu-Osher form), with
        boundary values held fixed over the substeps."""
        w = np.array(w, dtype=np.float64, copy=True)
        for _ in range(n):
            w1 = w + dt * self.apply(w, u, None, wb, ub)
            w2 = 0.75 * w + 0.25 * (w1 + dt * self.apply(w1, u, None, wb, ub))
            w = w / 3.0 + 2.0 / 3.0 * (w2 + dt * self.apply(w2, u, None, wb, ub))
        return w

    def ssprk3_extrap(self, w, dt, n, t0, ua, ta, ub, tb):
        """n SSP-RK3 substeps of the propagation problem (Sec. 3.2, "The propagation
        operator", eq. explproblem) with the convecting velocity extrapolated linearly in time
        from two stored fields: u(s) = ua + (s - ta) / (tb - ta) (ub - ua).  Substep j starts
        at s_j = t0 + j dt; the Shu-Osher stages evaluate the operator at s_j, s_j + dt and
        s_j + dt / 2."""
        ua = np.asarray(ua, dtype=np.float64)
        dub = np.asarray(ub, dtype=np.float64) - ua

        def u_at(s):
            return ua + ((s - ta) / (tb - ta)) * dub

        w = np.array(w, dtype=np.float64, copy=True)
        for j in range(n):
            s = t0 + j * dt
            w1 = w + dt * self.apply(w, u_at(s))
            w2 = 0.75 * w + 0.25 * (w1 + dt * self.apply(w1, u_at(s + dt)))
            w = w / 3.0 + 2.0 / 3.0 * (w2 + dt * self.apply(w2, u_at(s + 0.5 * dt)))
        return w

    def richardson(self, g, u, tau, ds, rtol, max_it, v0=None):
        """Pseudo-time iteration for the implicit convection problem with frozen convection
        (Sec. 3.3, eq. implconv):  v + tau (M^V)^-1 C^V(u) v = g.  Explicit Euler steps of size
        ds in pseudo time (eq. implconvit, read with the sign that makes the residual of
        eq. implconv vanish at the fixed point):

            res_i   = g - v_i + tau r(v_i),   r = -(M^V)^-1 C^V(u) v  (= self.apply)
            v_{i+1} = v_i + ds res_i

        from v_0 (default g), until ||res_i|| <= rtol ||res_0|| (L2 norm), at most max_it
        updates.  Returns (v_n, n, [||res_0||, ..., ||res_{n'}||]) with n the number of updates
        (v_n is the first iterate meeting the criterion, or v_max_it) and the residual norms of
        the iterates v_0 .. v_n' that were evaluated."""
        g = np.asarray(g, dtype=np.float64)
        v = np.array(g if v0 is None else v0, dtype=np.float64, copy=True)
        hist = []
        for i in range(max_it):
            res = g - v + tau * self.apply(v, u)
            hist.append(self.l2_norm(res))
            if hist[-1] <= rtol * hist[0]:
                return v, i, hist
            v = v + ds * res
        return v, max_it, hist

    # ---- projection and functionals ----------------------------------------------------
    def quad_points(self, n):
        """Physical points of a collapsed rule with n points per direction: [E, Q, d]."""
        p, _ = R.collapsed_rule(self.dim, n)
        return self.mesh.X[:, None, 0, :] + np.einsum("tij,qj->tqi", self.mesh.J, p)

    def project(self, vals, n):
        """L2 projection onto V_h of a field given at quad_points(n): vals [E, Q, d]."""
        p, wq = R.collapsed_rule(self.dim, n)
        phi = R.eval_basis(self.dim, self.k, p)
        rhs = np.einsum("t,q,tqi,qm->tim", self.mesh.absdetJ, wq, vals, phi)
        return rhs / self.mass[:, None, :]

    def evaluate(self, w, pts_ref):
        """w at reference points [Q, d] of every element -> [E, Q, d]."""
        phi = R.eval_basis(self.dim, self.k, pts_ref)
        return np.einsum("qm,tim->tqi", phi, w)

    def energy(self, w):
        """1/2 int |w|^2 dx by quadrature."""
        wq = np.einsum("qm,tim->tqi", self.phi_v, w)
        return 0.5 * np.einsum("t,q,tqi,tqi->", self.mesh.absdetJ, self.vw, wq, wq)

    def momentum(self, w):
        """int w dx (vector) by quadrature."""
        wq = np.einsum("qm,tim->tqi", self.phi_v, w)
        return np.einsum("t,q,tqi->i", self.mesh.absdetJ, self.vw, wq)

    def l2_norm(self, w):
        return np.sqrt(2.0 * self.energy(w))

    def rel_l2(self, a, b):
        """||a - b||_L2 / ||b||_L2."""
        return self.l2_norm(a - b) / self.l2_norm(b)

    def max_speed(self, w, n=None):
        """max over the points of a volume rule of the Euclidean norm of w."""
        n = R.volume_points_for_oracle(self.k) if n is None else n
        p, _ = R.collapsed_rule(self.dim, n)
        return float(np.max(np.linalg.norm(self.evaluate(w, p), axis=-1)))

    def dissipation(self, w, u, wb=None, ub=None):
        """1/2 sum_F int_F |beta| |w^- - w^+|^2 ds (each facet once), the upwind dissipation;
        on boundary facets w^+, u^+ are the boundary values wb, ub."""
        m, d = self.mesh, self.dim
        T = np.arange(m.E)
        pown, pnbr = self.facet_basis(T)
        tot = 0.0
        for f in range(d + 1):
            wm = np.einsum("tqm,tim->tqi", pown[:, f], w[T])
            wp = self._outer(T, f, pnbr, w, wb)
            um = np.einsum("tqm,tim->tqi", pown[:, f], u[T])
            up = self._outer(T, f, pnbr, u, ub)
            beta = 0.5 * np.einsum("tqj,tj->tq", um + up, m.normal[T, f])
            jump2 = np.sum((wm - wp) ** 2, axis=-1)
            # interior facets are visited from both sides (weight 1/2 each), boundary facets once
            wgt = np.where(m.nbr[T, f] < 0, 1.0, 0.5)
            tot += np.einsum("t,t,q,tq,tq->", wgt, m.area[T, f], self.fw, np.abs(beta), jump2)
        return 0.5 * tot


def cfl_dt(h, k, umax, c=0.1):
    """dt = c h / (k^2 max|u|), the substep size of the benchmark configurations."""
    return c * h / (max(k, 1) ** 2 * umax)
