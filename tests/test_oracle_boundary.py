"""Pins of the oracle's boundary facets (bounded box directions, no CPU GPU split here).

Sec. 2.3: the upwind value on the inflow part of the boundary comes from outside the domain;
here the outer values are given at the boundary facet points and enter the interior flux
formula.  Pinned by the upwind energy identity with zero outer data, free-stream
preservation, the textbook k = 0 finite-volume update with inflow data, and order k + 1
convergence on an exact travelling wave entering through the inflow boundary.
"""
import numpy as np
import pytest

from oracle import refelem as R
from oracle.dg import Space
from oracle.mesh import box_mesh


def rand_state(sp, seed=0, scale=1.0):
    return np.random.default_rng(seed).normal(0, scale, size=sp.shape)


def const_field(sp, v):
    U = np.zeros(sp.shape)
    U[:, :, 0] = np.array(v) / R.eval_basis(sp.dim, 0, np.zeros((1, sp.dim)))[0, 0]
    return U


def const_bvals(sp, v):
    return np.broadcast_to(np.array(v, dtype=np.float64),
                           (len(sp.mesh.bfacets), len(sp.fw), sp.dim)).copy()


CHANNELS = [(2, 4, (False, True), 0.2), (3, 2, (False, True, False), 0.1)]


def test_boundary_facet_count():
    m = box_mesh(2, 5, periodic=(False, True))
    assert len(m.bfacets) == 2 * 5
    m = box_mesh(3, 3, periodic=(False, True, False))
    assert len(m.bfacets) == 4 * 2 * 9
    # boundary facets lie on the bounded sides, and their points do
    sp = Space(m, 2)
    x = sp.boundary_points()
    on = (np.abs(x[..., 0]) < 1e-12) | (np.abs(x[..., 0] - 1) < 1e-12) | \
         (np.abs(x[..., 2]) < 1e-12) | (np.abs(x[..., 2] - 1) < 1e-12)
    assert on.all()


@pytest.mark.parametrize("dim,N,per,jit", CHANNELS)
@pytest.mark.parametrize("k", [1, 3])
def test_energy_identity_with_zero_outer_data(dim, N, per, jit, k):
    """Frozen constant u (divergence-free, continuous): <w, M r> = -1/2 sum_F int |u.n| |[w]|^2
    with [w] = w^- - 0 on boundary facets: interior facets dissipate as before, outflow facets
    carry 1/2 (u.n)|w|^2 out, and zero inflow data takes 1/2 |u.n| |w|^2 away."""
    m = box_mesh(dim, N, jitter=jit, seed=4, periodic=per)
    sp = Space(m, k)
    v = [0.8, -0.45, 0.3][:dim]
    U = const_field(sp, v)
    w = rand_state(sp, 5)
    wb = const_bvals(sp, [0.0] * dim)
    ub = const_bvals(sp, v)
    r = sp.apply(w, U, wb=wb, ub=ub)
    lhs = np.einsum("t,tim,tim->", m.absdetJ, w, r)
    diss = sp.dissipation(w, U, wb=wb, ub=ub)
    assert diss > 0
    assert abs(lhs + diss) < 1e-12 * diss


@pytest.mark.parametrize("dim,N,per,jit", CHANNELS)
def test_free_stream_preservation(dim, N, per, jit):
    m = box_mesh(dim, N, jitter=jit, seed=2, periodic=per)
    sp = Space(m, 2)
    c = [1.0, -0.5, 0.25][:dim]
    w = const_field(sp, c)
    r = sp.apply(w, wb=const_bvals(sp, c))
    assert np.abs(r).max() < 1e-13
    u = const_field(sp, [0.3, 0.7, -0.2][:dim])
    r = sp.apply(w, u, wb=const_bvals(sp, c), ub=const_bvals(sp, [0.3, 0.7, -0.2][:dim]))
    assert np.abs(r).max() < 1e-13


def test_boundary_values_are_required():
    sp = Space(box_mesh(2, 3, periodic=(False, True)), 1)
    with pytest.raises(ValueError):
        sp.apply(rand_state(sp, 1))


@pytest.mark.parametrize("dim,per", [(2, (False, True)), (3, (False, True, False))])
def test_k0_upwind_finite_volume_with_inflow_data(dim, per):
    """k = 0: r_T = -(1/|T|) sum_F |F| beta_F W_upwind with cell values W, where a boundary
    facet's outer value is the given datum (textbook first-order upwind FV)."""
    m = box_mesh(dim, 3, jitter=0.2, seed=9, periodic=per)
    sp = Space(m, 0)
    w = rand_state(sp, 3)
    rng = np.random.default_rng(7)
    data = rng.normal(size=(len(m.bfacets), dim))  # one outer value per boundary facet
    wb = np.repeat(data[:, None, :], len(sp.fw), axis=1)
    phi0 = np.sqrt(1.0 / R.ref_volume(dim))
    W = w[:, :, 0] * phi0
    vol = m.absdetJ * R.ref_volume(dim)
    dW = np.zeros_like(W)
    for t in range(m.E):
        for f in range(dim + 1):
            nb = m.nbr[t, f]
            outer = W[nb] if nb >= 0 else data[m.bf_id[t, f]]
            beta = 0.5 * (W[t] + outer) @ m.normal[t, f]
            up = W[t] if beta > 0 else outer
            dW[t] -= m.area[t, f] * beta * up / vol[t]
    r = sp.apply(w, wb=wb)
    assert np.abs(r[:, :, 0] * phi0 - dW).max() < 1e-12 * np.abs(dW).max()


def _wave(x, t, A=0.3):
    """w = (1, 1/2 + A sin(2 pi (x - t))): w_t + div(w (x) w) = 0 exactly (w_1 = 1 carries
    the profile of w_2 to the right)."""
    out = np.empty(x.shape)
    out[..., 0] = 1.0
    out[..., 1] = 0.5 + A * np.sin(2 * np.pi * (x[..., 0] - t))
    return out


def _wave_error(k, N, T, n):
    m = box_mesh(2, N, periodic=(False, True))
    sp = Space(m, k)
    q = k + 6
    w = sp.project(_wave(sp.quad_points(q), 0.0), q)
    xb = sp.boundary_points()
    dt = T / n
    for j in range(n):
        s = j * dt
        L = lambda v, t: sp.apply(v, wb=_wave(xb, t))  # outer values at the stage's time
        w1 = w + dt * L(w, s)
        w2 = 0.75 * w + 0.25 * (w1 + dt * L(w1, s + dt))
        w = w / 3.0 + 2.0 / 3.0 * (w2 + dt * L(w2, s + 0.5 * dt))
    ex = sp.project(_wave(sp.quad_points(q), T), q)
    return sp.l2_norm(w - ex)


def test_inflow_wave_converges_at_order_k_plus_one():
    """The wave enters through the inflow side (u.n = -1 at x = 0): the error after crossing
    a third of the channel falls at order k + 1 only if the inflow data enters correctly."""
    k, T = 2, 0.3
    errs = [_wave_error(k, N, T, 12 * N) for N in (4, 8, 16)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > k + 0.5, (errs, rates)
