"""The learned macro-step of the propagation problem and its a-posteriori check, in FP64.

Test infrastructure (see ``oracle/__init__``).  The macro-step is not in the paper: it replaces
M explicit SSP-RK3 substeps of the propagation problem ds w + (M^V)^-1 C^V w = 0 (Sec. 3.2,
eq. explproblem; self-convection u := w) by one network evaluation, checked a posteriori, with
the plain substeps as fallback.  Everything here is built from ``dg.Space.apply`` (the
operator), ``dg.Space.l2_norm`` (quadrature norms) and ``mlp.forward`` (the FP64 network).

Definitions, for a state w, substep dt, M substeps, tau = M dt, mesh size h:

  scale      s = max |w(x)| over the points of a collapsed Gauss rule with n points per
             direction (the network's convention; the library uses n = ceil((3k+1)/2))
  sign       sigma_T = sign of the x component of v_1 - v_0 (the point reflection of a split
             square swaps its two triangles and maps the flow to itself with w -> -w)
  candidate  w~ = w + tau r(w) + sigma_T (s^3 tau^2 / h) y_T,   y = net(features of w)
             (the network gives the remainder of the macro-step beyond forward Euler over tau,
             in units of s^3 tau^2 / h)
  defect     rho = ||w~ - w - (tau / 2) (r(w) + r(w~))|| / ||w~ - w||   (L2 norms over the mesh)
             the residual of the trapezoid rule for ds w = r(w) over [0, tau], relative to the
             macro increment; rho = 0 for the exact trapezoid step of a linear operator.  Edge
             cases: rho is NaN when either norm is not finite; with w~ = w it is 0 if the
             residual vanishes too, else infinite
  decision   accept w~ when rho <= tol (a NaN defect is never accepted); otherwise the M plain
             SSP-RK3 substeps of size dt from w

Reading (the benchmark configuration asks for a "residual check against one plain substep"):
the check costs two operator applications, less than one SSP-RK3 substep (three), and the
trapezoid defect is what that cost buys; the 8 plain substeps are the fallback and the judge.
"""
import numpy as np

from . import mlp


def orientation_sign(mesh):
    """sigma_T = sign of the x component of v_1 - v_0 for every element (+1 at 0)."""
    X = mesh.X
    return np.where(X[:, 1, 0] - X[:, 0, 0] < 0, -1.0, 1.0)


def scale(sp, w, n):
    """s = max |w| over a collapsed Gauss rule with n points per direction."""
    return sp.max_speed(w, n=n)


def candidate(sp, w, y, sign, s, tau, h, r0=None):
    """w~ = w + tau r(w) + sigma_T (s^3 tau^2 / h) y_T; y [E, d Np] (or the state's shape);
    r0 = r(w) when already known."""
    r0 = sp.apply(w) if r0 is None else r0
    unit = s ** 3 * tau ** 2 / h
    return w + tau * r0 + (sign * unit)[:, None, None] * np.asarray(y, dtype=np.float64).reshape(w.shape)


def defect(sp, w, wt, tau, u=None, r0=None, r1=None):
    """rho = ||w~ - w - (tau/2)(r(w) + r(w~))|| / ||w~ - w|| with r = sp.apply(., u) (u None:
    self-convection); r0, r1 = r(w), r(w~) when already known."""
    r0 = sp.apply(w, u) if r0 is None else r0
    r1 = sp.apply(wt, u) if r1 is None else r1
    inc = wt - w
    num = sp.l2_norm(inc - 0.5 * tau * (r0 + r1))
    den = sp.l2_norm(inc)
    if not (np.isfinite(num) and np.isfinite(den)):
        return float("nan")
    if den > 0:
        return float(num / den)
    return float("inf") if num > 0 else 0.0


def macro_step(sp, params, w, dt, M, tol, h, n_scale, y=None):
    """One macro-step from w: returns (new state, accepted, rho, candidate).

    y: the network output [E, d Np] to use (e.g. the one a BF16 implementation produced, so
    that everything after the network can be compared exactly); None evaluates the FP64
    network oracle on the features of w."""
    w = np.asarray(w, dtype=np.float64)
    tau = M * dt
    sign = orientation_sign(sp.mesh)
    s = scale(sp, w, n_scale)
    if y is None:
        x = mlp.features(w, sp.mesh.nbr, sign, s, np.arange(sp.mesh.E))
        y = mlp.forward(params, x)
    r0 = sp.apply(w)
    wt = candidate(sp, w, y, sign, s, tau, h, r0=r0)
    rho = defect(sp, w, wt, tau, r0=r0)
    if np.isfinite(rho) and rho <= tol:
        return wt, True, rho, wt
    return sp.ssprk3(w, dt, M), False, rho, wt
