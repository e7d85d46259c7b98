"""Pins of the macro-step oracle (oracle/macro.py): the candidate, the trapezoid defect and the
accept decision, checked against what linear algebra and the symmetries of the flow fix.

* The defect vanishes for the exact trapezoid step of a linear operator, and equals
  (tau / 2) ||L^2 w|| / ||L w|| for the forward-Euler candidate; L is the frozen-velocity
  operator assembled by exact rational integration (oracle/bruteforce.py), which shares
  nothing with the operator the defect calls.
* Self-convection is quadratic, so the macro-map is homogeneous: w -> a w with tau -> tau / a
  maps candidate and defect onto themselves (catches a wrong power of s or tau in the unit
  s^3 tau^2 / h, or a missing term).
* The point reflection x -> (1, 1) - x maps the split-square mesh onto itself with the
  flow w -> -w: the candidate commutes with it (catches a missing or misplaced orientation
  sign).
* The decision takes the candidate at tol >= rho and the plain substeps otherwise; a
  non-finite network output is never accepted; a zero network gives the Euler candidate.
"""
import numpy as np
import pytest

from oracle import macro, mlp
from oracle import refelem as R
from oracle.bruteforce import assemble_frozen_constant
from oracle.dg import Space
from oracle.mesh import box_mesh


def frozen_setup(N=2, k=1, u=(1.0, 1.0 / 3.0), jit=0.0):
    m = box_mesh(2, N, jitter=jit, seed=11)
    sp = Space(m, k)
    L = assemble_frozen_constant(m.X, m.period, k, u, m.nbr, m.nbr_facet, m.shift)
    U = np.zeros(sp.shape)
    U[:, :, 0] = np.array(u) / R.eval_basis(2, 0, np.zeros((1, 2)))[0, 0]
    return m, sp, L, U


def per_component(L, w, fn):
    """Apply fn (a dense map on one component's flattened coefficients) to each component."""
    out = np.empty_like(w)
    E, d, Np = w.shape
    for i in range(d):
        out[:, i, :] = fn(w[:, i, :].ravel()).reshape(E, Np)
    return out


def l2(m, c):
    """L2 norm of a coefficient array in the orthonormal basis: sqrt(sum_T |J_T| |c_T|^2)."""
    return np.sqrt(np.einsum("t,tim->", m.absdetJ, c * c))


@pytest.mark.parametrize("k,jit", [(1, 0.0), (2, 0.0), (1, 0.1)])
def test_defect_vanishes_for_the_exact_trapezoid_step(k, jit):
    m, sp, L, U = frozen_setup(N=2 if jit == 0 else 3, k=k, jit=jit)
    w = np.random.default_rng(3).normal(size=sp.shape)
    tau = 0.4 / np.linalg.norm(L, 2)
    n = L.shape[0]
    A = np.eye(n) - 0.5 * tau * L
    B = np.eye(n) + 0.5 * tau * L
    wt = per_component(L, w, lambda v: np.linalg.solve(A, B @ v))
    rho = macro.defect(sp, w, wt, tau, u=U)
    assert rho < 1e-12, rho
    # and it does not vanish for a candidate that is off by a little
    assert macro.defect(sp, w, wt * (1 + 1e-6), tau, u=U) > 1e-8


@pytest.mark.parametrize("k", [1, 2])
def test_defect_of_the_euler_candidate(k):
    m, sp, L, U = frozen_setup(k=k)
    w = np.random.default_rng(4).normal(size=sp.shape)
    tau = 0.3 / np.linalg.norm(L, 2)
    Lw = per_component(L, w, lambda v: L @ v)
    LLw = per_component(L, w, lambda v: L @ (L @ v))
    # w~ - w - tau/2 (L w + L (w + tau L w)) = -tau^2/2 L^2 w  and  w~ - w = tau L w
    ref = 0.5 * tau * l2(m, LLw) / l2(m, Lw)
    got = macro.defect(sp, w, w + tau * Lw, tau, u=U)
    assert abs(got - ref) <= 1e-12 * ref, (got, ref)


def test_defect_is_homogeneous_in_self_mode():
    sp = Space(box_mesh(2, 3, jitter=0.15, seed=2), 2)
    rng = np.random.default_rng(5)
    w = rng.normal(size=sp.shape)
    tau = 0.01
    wt = w + tau * sp.apply(w) + 1e-4 * rng.normal(size=sp.shape)
    rho = macro.defect(sp, w, wt, tau)
    for a in (2.0, 3.7):
        assert abs(macro.defect(sp, a * w, a * wt, tau / a) - rho) <= 1e-12 * rho
    # not invariant if tau is left alone (the check above is not vacuous)
    assert abs(macro.defect(sp, 3.7 * w, 3.7 * wt, tau) - rho) > 1e-3 * rho


def small_net(seed, gain=0.3):
    return mlp.init_params(seed) * gain


def test_candidate_is_homogeneous():
    N, k = 4, 3
    sp = Space(box_mesh(2, N), k)
    w = np.random.default_rng(6).normal(size=sp.shape)
    p = small_net(7)
    dt, h, n = 2e-3, 1.0 / N, (3 * k + 1) // 2
    _, _, _, wt = macro.macro_step(sp, p, w, dt, 8, np.inf, h, n)
    for a in (2.0, 3.0):
        _, _, _, wta = macro.macro_step(sp, p, a * w, dt / a, 8, np.inf, h, n)
        e = np.abs(wta - a * wt).max() / np.abs(a * (wt - w)).max()
        assert e < 1e-12, (a, e)
    # the network term itself scales like the state (its unit is s^3 tau^2 / h)
    _, _, _, wt2 = macro.macro_step(sp, p, 2 * w, dt / 2, 8, np.inf, h, n)
    _, _, _, w0 = macro.macro_step(sp, np.zeros_like(p), w, dt, 8, np.inf, h, n)
    _, _, _, w02 = macro.macro_step(sp, np.zeros_like(p), 2 * w, dt / 2, 8, np.inf, h, n)
    net, net2 = wt - w0, wt2 - w02
    assert np.abs(net).max() > 1e-6 * np.abs(wt - w).max()
    assert np.abs(net2 - 2.0 * net).max() <= 1e-12 * np.abs(net2).max()


def reflect(N, w):
    """Coefficients of the reflected field -w((1,1) - x) on the split-square box mesh: the
    element 2(jN+i)+b goes to 2((N-1-j)N + N-1-i) + 1-b with the same local frame and minus
    its coefficients."""
    out = np.empty_like(w)
    for j in range(N):
        for i in range(N):
            for b in range(2):
                out[2 * ((N - 1 - j) * N + N - 1 - i) + 1 - b] = -w[2 * (j * N + i) + b]
    return out


def test_candidate_commutes_with_the_point_reflection():
    N, k = 4, 3
    sp = Space(box_mesh(2, N), k)
    w = np.random.default_rng(8).normal(size=sp.shape)
    p = small_net(9)
    dt, h, n = 2e-3, 1.0 / N, (3 * k + 1) // 2
    Rw = reflect(N, w)
    # the operator itself commutes with the reflection
    assert np.abs(sp.apply(Rw) - reflect(N, sp.apply(w))).max() <= 1e-12 * np.abs(sp.apply(w)).max()
    _, _, rho, wt = macro.macro_step(sp, p, w, dt, 8, np.inf, h, n)
    _, _, rho_r, wt_r = macro.macro_step(sp, p, Rw, dt, 8, np.inf, h, n)
    assert np.abs(wt_r - reflect(N, wt)).max() <= 1e-12 * np.abs(wt - w).max()
    assert abs(rho_r - rho) <= 1e-12 * rho
    # without the orientation sign the network term would not commute with the reflection
    sign = macro.orientation_sign(sp.mesh)
    assert set(np.unique(sign)) == {-1.0, 1.0}
    s = macro.scale(sp, w, n)
    y = mlp.forward(p, mlp.features(w, sp.mesh.nbr, np.ones(sp.mesh.E), s, np.arange(sp.mesh.E)))
    yr = mlp.forward(p, mlp.features(Rw, sp.mesh.nbr, np.ones(sp.mesh.E), s, np.arange(sp.mesh.E)))
    c = macro.candidate(sp, w, y, np.ones(sp.mesh.E), s, 8 * dt, h)
    cr = macro.candidate(sp, Rw, yr, np.ones(sp.mesh.E), s, 8 * dt, h)
    assert np.abs(cr - reflect(N, c)).max() > 1e-6 * np.abs(c - w).max()


def test_decision_and_fallback():
    N, k = 3, 3
    sp = Space(box_mesh(2, N, jitter=0.1, seed=3), k)
    w = np.random.default_rng(10).normal(size=sp.shape)
    p = small_net(11)
    dt, h, n = 1e-3, 1.0 / N, (3 * k + 1) // 2
    _, acc, rho, wt = macro.macro_step(sp, p, w, dt, 8, np.inf, h, n)
    assert acc and rho > 0 and np.isfinite(rho)
    out, acc, _, _ = macro.macro_step(sp, p, w, dt, 8, rho, h, n)
    assert acc and np.array_equal(out, wt)
    out, acc, _, _ = macro.macro_step(sp, p, w, dt, 8, rho * (1 - 1e-9), h, n)
    assert not acc and np.array_equal(out, sp.ssprk3(w, dt, 8))
    # a non-finite network output gives a NaN defect, which is rejected at any tolerance
    y = np.zeros((sp.mesh.E, 2 * sp.np))
    y[1, 3] = np.nan
    out, acc, rho_nan, _ = macro.macro_step(sp, p, w, dt, 8, np.inf, h, n, y=y)
    assert not acc and np.isnan(rho_nan) and np.array_equal(out, sp.ssprk3(w, dt, 8))
    # a zero network gives the forward-Euler candidate over tau
    _, _, rho0, wt0 = macro.macro_step(sp, np.zeros_like(p), w, dt, 8, np.inf, h, n)
    tau = 8 * dt
    assert np.abs(wt0 - (w + tau * sp.apply(w))).max() <= 1e-15 * np.abs(w).max()
    assert rho0 == macro.defect(sp, w, w + tau * sp.apply(w), tau)


def test_defect_edge_cases():
    sp = Space(box_mesh(2, 2), 1)
    w = np.random.default_rng(12).normal(size=sp.shape)
    # no change predicted: infinite defect unless the operator vanishes as well
    assert macro.defect(sp, w, w, 0.1) == np.inf
    z = np.zeros(sp.shape)  # the zero state: r = 0 exactly
    assert macro.defect(sp, z, z, 0.1) == 0.0
