"""GPU parity of the matrix-core operator paths against the FP64 oracle.

* FP64 on the matrix cores (v_mfma_f64_16x16x4): the same 1e-12 relative L2 bar as the VALU
  path.
* Mixed precision (FP64 state, flux, facet sums and RK; basis contractions as split FP16x2 or
  BF16x3 products with FP32 accumulation, or FP32 on the vector units): the error against the
  FP64 oracle is measured and held below the bars of gpu_common.reduced_bars (the pieces'
  unit roundoff times the cancellation factor of the operator, which the oracle measures).
"""
import os

import numpy as np
import pytest

from gpu_common import (C1, C5, UNIT, initial_state, operator_scales, oracle_space, reduced_bars,
                        rel_l2, say)
from oracle.dg import cfl_dt

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import paper_1508_04245_amd as dg
    assert torch.cuda.is_available()
    dg.lib()
    return dg


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def mesh_with(dg, env, factory):
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return factory()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def lib_mesh(dg, sp, dim, N, k, jit, env):
    if jit == 0.0:
        return mesh_with(dg, env, lambda: dg.Mesh.box(dim, N, k))
    X = sp.mesh.X
    E = X.shape[0]
    return mesh_with(dg, env, lambda: dg.Mesh.from_arrays(
        dim, k, X.reshape(-1, dim), np.arange(E * (dim + 1)).reshape(E, dim + 1), np.ones(dim)))


CASES = [(2, k, 5, 0.2) for k in range(7)] + [(3, k, 3, 0.15) for k in range(5)]
MFMA64 = {"DGCONV_FP64_KERNEL": "mfma"}


@pytest.mark.parametrize("dim,k,N,jit", CASES)
def test_fp64_mfma_apply_all_degrees(dg, dim, k, N, jit):
    say("case fp64-mfma apply dim=%d k=%d" % (dim, k))
    sp = oracle_space(dim, N, k, jit, seed=k)
    m = lib_mesh(dg, sp, dim, N, k, jit, MFMA64)
    w = initial_state(sp, seed=1, sd=0.05)
    u = initial_state(sp, field="fourier", seed=2)
    for uu in (None, u):
        got = m.apply(dev(w), None if uu is None else dev(uu)).cpu().numpy()
        ref = sp.apply(w, uu)
        e = rel_l2(sp, got, ref)
        say("   rel_l2 %.3e" % e)
        assert e <= 1e-12


def test_fp64_mfma_c1_substeps(dg):
    dim, N, k = C1
    say("case fp64-mfma c1 100 substeps")
    sp = oracle_space(dim, N, k)
    m = mesh_with(dg, MFMA64, lambda: dg.Mesh.box(dim, N, k))
    w = initial_state(sp, seed=0)
    dt = cfl_dt(1.0 / N, k, sp.max_speed(w))
    wd = dev(w)
    m.rk_substeps(wd, dt, 100)
    e = rel_l2(sp, wd.cpu().numpy(), sp.ssprk3(w, dt, 100))
    say("   rel_l2 %.3e" % e)
    assert e <= 1e-12


@pytest.mark.parametrize("prec", ["f16x2", "bf16x3"])
@pytest.mark.parametrize("dim,k,N,jit", [(2, 2, 5, 0.2), (2, 4, 4, 0.0), (3, 2, 3, 0.15),
                                         (3, 3, 2, 0.0)])
def test_mixed_apply_error(dg, prec, dim, k, N, jit):
    say("case mixed %s apply dim=%d k=%d" % (prec, dim, k))
    sp = oracle_space(dim, N, k, jit, seed=k)
    m = lib_mesh(dg, sp, dim, N, k, jit, {})
    w = initial_state(sp, seed=1, sd=0.05)
    got = m.apply(dev(w), precision=prec).cpu().numpy()
    ref, amp, _ = operator_scales(sp, w)
    e = rel_l2(sp, got, ref)
    bar = reduced_bars(prec, amp)[0]
    say("   rel_l2 %.3e (bar %.1e, %.2f u amp)" % (e, bar, e / (UNIT[prec] * amp)))
    assert e <= bar


def c5_apply_and_substeps(dg, prec, n=4):
    """The 2D 128^2 x 2 P3 workload (random Fourier field): one application and n substeps of
    variant prec against the oracle, with their bars (gpu_common.reduced_bars)."""
    dim, N, k = C5
    sp = oracle_space(dim, N, k)
    m = dg.Mesh.box(dim, N, k)
    w = initial_state(sp, field="fourier", seed=3)
    r = m.apply(dev(w), precision=prec).cpu().numpy()
    ref, amp, rate = operator_scales(sp, w)
    e_apply = rel_l2(sp, r, ref)
    dt = cfl_dt(1.0 / N, k, sp.max_speed(w))
    wd = dev(w)
    m.rk_substeps(wd, dt, n, precision=prec)
    e_state = rel_l2(sp, wd.cpu().numpy(), sp.ssprk3(w, dt, n))
    b_apply, b_state = reduced_bars(prec, amp, dt * rate, n=n)
    say("   apply rel_l2 %.3e (bar %.1e)  state after %d substeps rel_l2 %.3e (bar %.1e)"
        % (e_apply, b_apply, n, e_state, b_state))
    assert e_apply <= b_apply
    assert e_state <= b_state


@pytest.mark.parametrize("prec", ["f16x2", "bf16x3"])
def test_mixed_c5_substeps(dg, prec):
    say("case mixed %s c5 apply + 4 substeps" % prec)
    c5_apply_and_substeps(dg, prec)


@pytest.mark.parametrize("dim,k,N,jit", CASES)
def test_mixf32_apply_all_degrees(dg, dim, k, N, jit):
    """FP64 state, flux, facet sums and update around FP32 contractions (the vector-unit
    kernel), self and frozen mode, every compiled degree, against the FP64 oracle (bars:
    gpu_common.reduced_bars)."""
    say("case mixf32 apply dim=%d k=%d" % (dim, k))
    sp = oracle_space(dim, N, k, jit, seed=k)
    m = lib_mesh(dg, sp, dim, N, k, jit, {})
    w = initial_state(sp, seed=1, sd=0.05)
    u = initial_state(sp, field="fourier", seed=2)
    for uu in (None, u):
        got = m.apply(dev(w), None if uu is None else dev(uu), precision="mixf32").cpu().numpy()
        ref, amp, _ = operator_scales(sp, w, uu)
        e = rel_l2(sp, got, ref)
        bar = reduced_bars("mixf32", amp)[0]
        say("   %s rel_l2 %.3e (bar %.1e, %.2f u amp)"
            % ("frozen" if uu is not None else "self", e, bar, e / (UNIT["mixf32"] * amp)))
        assert e <= bar


def test_mixf32_c5_substeps(dg):
    say("case mixf32 c5 apply + 4 substeps")
    c5_apply_and_substeps(dg, "mixf32")
