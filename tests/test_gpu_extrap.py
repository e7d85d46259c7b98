"""GPU parity of the propagation substeps with a convecting velocity extrapolated linearly in
time (dg_rk_substeps_extrap) against the oracle's stepper, on jittered meshes with ragged
tiles, for the VALU and matrix-core FP64 kernels and the reduced-precision variants.
Every test prints its case before touching the GPU.
"""
import os

import numpy as np
import pytest

from gpu_common import initial_state, operator_scales, oracle_space, reduced_bars, rel_l2, say
from oracle.dg import cfl_dt

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import paper_1508_04245_amd as dg
    assert torch.cuda.is_available(), "GPU tests need a device"
    dg.lib()
    return dg


def lib_mesh(dg, sp, dim, k):
    X = sp.mesh.X
    E = X.shape[0]
    elem = np.arange(E * (dim + 1)).reshape(E, dim + 1)
    return dg.Mesh.from_arrays(dim, k, X.reshape(-1, dim), elem, np.ones(dim))


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


# (dim, k, N, jitter): 338 and 162 elements -> several tiles and a ragged last one
CASES = [(2, 2, 13, 0.2), (2, 4, 7, 0.2), (3, 2, 3, 0.15), (3, 3, 3, 0.15)]
# precision, FP64 kernel (bar of the final state: gpu_common.reduced_bars, with the scales of the
# operator frozen at the later field, which the extrapolation starts from)
VARIANTS = [("fp64", "valu"), ("fp64", "mfma"), ("fp32", None), ("bf16x3", None),
            ("f16x2", None), ("mixf32", None)]


@pytest.mark.parametrize("dim,k,N,jit", CASES)
def test_extrap_substeps_vs_oracle(dg, dim, k, N, jit):
    say("case extrap dim=%d k=%d N=%d jitter=%g" % (dim, k, N, jit))
    sp = oracle_space(dim, N, k, jit, seed=3)
    w = initial_state(sp, seed=4, sd=0.05)
    ua = 0.5 * initial_state(sp, field="fourier", seed=5)
    ub = 0.5 * initial_state(sp, field="fourier", seed=6)
    umax = max(sp.max_speed(ua), sp.max_speed(ub))
    n = 6
    dt = cfl_dt(1.0 / N, k, 3.0 * umax)  # |u(s)| <= |ub| + |ub - ua| over the substeps
    t0, ta, tb = 0.0, -n * dt, 0.0  # extrapolation forward from the fields at -n dt and 0
    ref = sp.ssprk3_extrap(w, dt, n, t0, ua, ta, ub, tb)
    frozen = sp.ssprk3(w, dt, n, ub)
    assert sp.rel_l2(frozen, ref) > 1e-4  # the time dependence matters at this size
    _, amp, rate = operator_scales(sp, w, ub)
    for prec, kern in VARIANTS:
        tol = reduced_bars(prec, amp, dt * rate, n=n)[1]
        if kern:
            os.environ["DGCONV_FP64_KERNEL"] = kern
        else:
            os.environ.pop("DGCONV_FP64_KERNEL", None)
        say("   %s %s" % (prec, kern or ""))
        m = lib_mesh(dg, sp, dim, k)
        ty = torch.float32 if prec == "fp32" else torch.float64
        wd = dev(w, ty)
        m.rk_substeps_extrap(wd, dt, n, t0, dev(ua, ty), ta, dev(ub, ty), tb, precision=prec)
        got = wd.double().cpu().numpy()
        e = rel_l2(sp, got, ref)
        say("      rel_l2 %.3e (bar %.1e)" % (e, tol))
        assert e <= tol, (prec, kern, e)
    os.environ.pop("DGCONV_FP64_KERNEL", None)
