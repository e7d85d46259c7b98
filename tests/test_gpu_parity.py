"""GPU parity: the HIP library against the FP64 oracle on the same seeded inputs.

Bar (FP64 path): relative L2 error <= 1e-12 and max coefficient error <= 1e-12 max|ref|.
Every test prints its case before touching the GPU.
"""
import numpy as np
import pytest

from gpu_common import (C1, C2, C3, C4, C5, initial_state, operator_scales, oracle_rk_on_sample,
                        oracle_space, reduced_bars, rel_l2, rel_l2_rows, say)
from oracle.dg import cfl_dt

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def dg():
    import paper_1508_04245_amd as dg
    assert torch.cuda.is_available(), "GPU tests need a device"
    dg.lib()
    return dg


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def check(sp, got, ref, tol=TOL):
    e = rel_l2(sp, got, ref)
    emax = np.abs(got - ref).max() / np.abs(ref).max()
    say("   rel_l2 %.3e  max %.3e" % (e, emax))
    assert e <= tol and emax <= 10 * tol, (e, emax)


def lib_mesh(dg, sp, dim, N, k, jitter):
    if jitter == 0.0:
        return dg.Mesh.box(dim, N, k)
    # the oracle's jittered mesh, handed over as per-element vertices (no shared vertices)
    X = sp.mesh.X
    E = X.shape[0]
    xyz = X.reshape(-1, dim)
    elem = np.arange(E * (dim + 1)).reshape(E, dim + 1)
    return dg.Mesh.from_arrays(dim, k, xyz, elem, np.ones(dim))


# every compiled (dim, k) on a small mesh with a ragged last tile, self and frozen mode
CASES = [(2, k, 5, 0.2) for k in range(7)] + [(3, k, 3, 0.15) for k in range(5)]


@pytest.mark.parametrize("dim,k,N,jit", CASES)
def test_apply_all_degrees(dg, dim, k, N, jit):
    say("case apply dim=%d k=%d N=%d jitter=%g" % (dim, k, N, jit))
    sp = oracle_space(dim, N, k, jit, seed=k)
    m = lib_mesh(dg, sp, dim, N, k, jit)
    w = initial_state(sp, seed=1, sd=0.05)
    u = initial_state(sp, field="fourier", seed=2)
    for uu in (None, u):
        got = m.apply(dev(w), None if uu is None else dev(uu)).cpu().numpy()
        check(sp, got, sp.apply(w, uu))


def test_c1_apply_and_100_substeps(dg):
    dim, N, k = C1
    say("case c1 apply + 100 SSP-RK3 substeps")
    sp = oracle_space(dim, N, k)
    m = dg.Mesh.box(dim, N, k)
    w = initial_state(sp, seed=0)
    check(sp, m.apply(dev(w)).cpu().numpy(), sp.apply(w))
    dt = cfl_dt(1.0 / N, k, sp.max_speed(w))
    wd = dev(w)
    m.rk_substeps(wd, dt, 100)
    ref = sp.ssprk3(w, dt, 100)
    check(sp, wd.cpu().numpy(), ref)


def test_c5_apply_and_substeps(dg):
    dim, N, k = C5
    say("case c5 apply + 2 substeps (self) + 1 substep (frozen)")
    sp = oracle_space(dim, N, k)
    m = dg.Mesh.box(dim, N, k)
    w = initial_state(sp, field="fourier", seed=3)
    check(sp, m.apply(dev(w)).cpu().numpy(), sp.apply(w))
    dt = cfl_dt(1.0 / N, k, sp.max_speed(w))
    wd = dev(w)
    m.rk_substeps(wd, dt, 2)
    check(sp, wd.cpu().numpy(), sp.ssprk3(w, dt, 2))
    u = initial_state(sp, field="fourier", seed=4)
    wd = dev(w)
    m.rk_substeps(wd, dt, 1, u=dev(u))
    check(sp, wd.cpu().numpy(), sp.ssprk3(w, dt, 1, u))


_FULL = {}


def full_case(cfg, field):
    """Full-size mesh, its initial state, sampled elements and the oracle's values there (one
    configuration is kept at a time: the 3D 64^3 x 6 mesh alone holds 1.5M elements)."""
    key = (cfg, field)
    if key not in _FULL:
        _FULL.clear()
        dim, N, k = cfg
        sp = oracle_space(dim, N, k)
        w = initial_state(sp, field=field, seed=0)
        rng = np.random.default_rng(7)
        sample = np.unique(np.concatenate([rng.choice(sp.mesh.E, 300, replace=False),
                                           [0, sp.mesh.E - 1]]))
        ref_apply, amp, rate = operator_scales(sp, w, elems=sample)
        dt = cfl_dt(1.0 / N, k, 3.0)  # any positive step: a bound on max|w| for these fields
        inc = dt * rate  # one step's increment relative to the state
        S, ref_rk = oracle_rk_on_sample(sp, w, dt, sample[:60])
        _FULL[key] = (sp, w, sample, ref_apply, dt, S, ref_rk, amp, inc)
    return _FULL[key]


# (configuration, field, precision)
FULL_CASES = [
    (C2, "tg", "fp64"), (C2, "tg", "fp32"), (C2, "tg", "mixf32"), (C2, "tg", "f16x2"),
    (C2, "tg", "bf16x3"),
    (C3, "tg", "fp64"), (C3, "tg", "f16x2"), (C3, "tg", "bf16x3"),
    (C4, "fourier", "fp64"), (C4, "fourier", "fp32"), (C4, "fourier", "mixf32"),
    (C4, "fourier", "f16x2"), (C4, "fourier", "bf16x3"),
]


@pytest.mark.parametrize("cfg,field,prec", FULL_CASES)
def test_full_size_sampled(dg, cfg, field, prec):
    """Full-size meshes: one apply and one fused SSP-RK3 substep (the benchmark launch
    configuration), checked on sampled elements the oracle evaluates one by one, for the FP64
    path and for the FP32, FP32-contraction and split-product variants the configurations name
    (bars: gpu_common.reduced_bars, with the cancellation factor measured on the sample)."""
    dim, N, k = cfg
    say("case full-size sampled dim=%d N=%d k=%d %s" % (dim, N, k, prec))
    sp, w, sample, ref, dt, S, ref1, amp, inc = full_case(cfg, field)
    bar_apply, bar_rk = reduced_bars(prec, amp, inc, n=1, tol=TOL)
    say("   cancellation factor %.1f, step increment %.2e" % (amp, inc))
    ty = torch.float32 if prec == "fp32" else torch.float64
    m = dg.Mesh.box(dim, N, k)
    wd = dev(w, ty)
    r = m.apply(wd, precision=prec).double().cpu().numpy()
    J = sp.mesh.absdetJ[sample]
    e = rel_l2_rows(J, r[sample], ref)
    say("   apply sampled rel_l2 %.3e (bar %.1e)" % (e, bar_apply))
    assert e <= bar_apply
    if prec == "fp64":
        # properties that hold at any size: conservation of the discrete momentum
        mom = m.reduce("momentum", torch.tensor(r, device="cuda", dtype=torch.float64)).cpu().numpy()
        assert np.abs(mom[:dim]).max() <= 1e-12 * np.abs(r).max()
    m.rk_substeps(wd, dt, 1, precision=prec)
    got = wd.double().cpu().numpy()
    e = rel_l2_rows(sp.mesh.absdetJ[S], got[S], ref1)
    say("   substep sampled rel_l2 %.3e (bar %.1e)" % (e, bar_rk))
    assert e <= bar_rk


def test_reductions(dg):
    dim, N, k = 2, 7, 3
    say("case reductions")
    sp = oracle_space(dim, N, k, 0.2, seed=1)
    m = lib_mesh(dg, sp, dim, N, k, 0.2)
    a = initial_state(sp, seed=1, sd=0.1)
    b = initial_state(sp, seed=2, sd=0.1)
    ad, bd = dev(a), dev(b)
    en = m.reduce("energy", ad).cpu().numpy()[0]
    assert abs(en - sp.energy(a)) <= 1e-13 * sp.energy(a)
    mo = m.reduce("momentum", ad).cpu().numpy()[:dim]
    assert np.abs(mo - sp.momentum(a)).max() <= 1e-13
    l2 = m.reduce("l2diff", ad, bd).cpu().numpy()[:2]
    assert abs(l2[0] / l2[1] - sp.rel_l2(a, b)) <= 1e-12
    mv = m.reduce("maxvel", ad).cpu().numpy()[0]
    # the speed reduction is defined on the collapsed rule with ceil(3k/2) points per direction
    assert abs(mv - sp.max_speed(a, n=(3 * k + 1) // 2)) <= 1e-13 * mv
    bad = a.copy()
    bad[3, 1, 2] = np.nan
    bad[5, 0, 0] = np.inf
    assert m.reduce("nonfinite", dev(bad)).cpu().numpy()[0] == 2


def test_deterministic_and_stream(dg):
    dim, N, k = C1
    say("case determinism")
    sp = oracle_space(dim, N, k)
    m = dg.Mesh.box(dim, N, k)
    w = dev(initial_state(sp, seed=5))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        r1 = m.apply(w)
        r2 = m.apply(w)
    s.synchronize()
    assert torch.equal(r1, r2)
    w1, w2 = w.clone(), w.clone()
    m.rk_substeps(w1, 1e-3, 5)
    m.rk_substeps(w2, 1e-3, 5, work=torch.empty((2,) + tuple(w.shape), dtype=torch.float64,
                                                   device="cuda"))
    assert torch.equal(w1, w2)


def test_fp32_path(dg):
    """FP32 state and arithmetic against the FP64 oracle on the 2D 128^2 x 2 P3 workload (bar:
    gpu_common.reduced_bars)."""
    dim, N, k = C5
    say("case fp32 c5")
    sp = oracle_space(dim, N, k)
    m = dg.Mesh.box(dim, N, k)
    w = initial_state(sp, field="fourier", seed=3)
    ref, amp, _ = operator_scales(sp, w)
    bar = reduced_bars("fp32", amp)[0]
    r = m.apply(dev(w, torch.float32), precision="fp32").double().cpu().numpy()
    e = rel_l2(sp, r, ref)
    say("   fp32 apply rel_l2 %.3e (bar %.1e, %.1f u amp)" % (e, bar, e / (2.0 ** -24 * amp)))
    assert e <= bar


def test_argument_errors(dg):
    say("case argument errors")
    m = dg.Mesh.box(2, 4, 2)
    w = torch.zeros((m.E, 2, m.np), dtype=torch.float64, device="cuda")
    with pytest.raises(dg.DGError):
        m.rk_substeps(w, -1.0, 1)
    with pytest.raises(dg.DGError):
        m.rk_substeps(w, float("nan"), 1)
    with pytest.raises(dg.DGError):
        m.apply(w, out=w)
    flat = torch.zeros(w.numel() + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(dg.DGError):  # 8-byte misaligned state
        m.apply(flat[1:].view(w.shape))
