"""GPU parity on meshes with boundary facets (bounded box directions) against the oracle:
single applications in self and frozen mode and SSP-RK3 substeps with fixed outer values,
for the VALU and matrix-core FP64 kernels and the reduced-precision variants, on jittered
channel meshes with ragged tiles.  Every test prints its case before touching the GPU.
"""
import os

import numpy as np
import pytest

from gpu_common import UNIT, initial_state, operator_scales, reduced_bars, rel_l2, say
from oracle.dg import Space, cfl_dt
from oracle.mesh import box_mesh

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import paper_1508_04245_amd as dg
    assert torch.cuda.is_available(), "GPU tests need a device"
    dg.lib()
    return dg


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def wave(x, A=0.3):
    out = np.empty(x.shape)
    out[..., 0] = 1.0
    out[..., 1] = 0.5 + A * np.sin(2 * np.pi * x[..., 0])
    for c in range(2, x.shape[-1]):
        out[..., c] = 0.2 * np.cos(2 * np.pi * x[..., 1])
    return out


# (dim, k, N, periodic flags, jitter): 2D channel 338 elements, 3D duct 162 elements
CASES = [(2, 2, 13, (False, True), 0.2), (2, 4, 7, (False, True), 0.2),
         (3, 2, 3, (False, True, False), 0.1), (3, 3, 3, (False, True, False), 0.1)]
# precision, FP64 kernel (bars: gpu_common.reduced_bars)
VARIANTS = [("fp64", "valu"), ("fp64", "mfma"), ("fp32", None), ("bf16x3", None),
            ("f16x2", None), ("mixf32", None)]


@pytest.mark.parametrize("dim,k,N,per,jit", CASES)
def test_boundary_apply_and_substeps_vs_oracle(dg, dim, k, N, per, jit):
    say("case boundary dim=%d k=%d N=%d periodic=%s" % (dim, k, N, per))
    om = box_mesh(dim, N, jitter=jit, seed=5, periodic=per)
    sp = Space(om, k)
    q = k + 4
    w = sp.project(wave(sp.quad_points(q)), q) + np.random.default_rng(1).normal(0, 0.02, sp.shape)
    u = initial_state(sp, field="fourier", seed=2)
    xb = sp.boundary_points()
    wb = wave(xb)
    ub = 0.5 * wave(xb)
    r_self, amp_s, rate = operator_scales(sp, w, wb=wb)
    r_frozen, amp_f, _ = operator_scales(sp, w, u, wb=wb, ub=ub)
    dt = cfl_dt(1.0 / N, k, max(sp.max_speed(w), 1.0))
    ref_rk = sp.ssprk3(w, dt, 3, wb=wb)
    say("   cancellation factor self %.1f frozen %.1f, step increment %.2e"
        % (amp_s, amp_f, dt * rate))
    E = om.E
    for prec, kern in VARIANTS:
        if kern:
            os.environ["DGCONV_FP64_KERNEL"] = kern
        else:
            os.environ.pop("DGCONV_FP64_KERNEL", None)
        say("   %s %s" % (prec, kern or ""))
        m = dg.Mesh.from_arrays(dim, k, om.X.reshape(-1, dim),
                                np.arange(E * (dim + 1)).reshape(E, dim + 1),
                                np.where(per, 1.0, 0.0))
        ty = torch.float32 if prec == "fp32" else torch.float64
        got = m.apply_bc(dev(w, ty), dev(wb, ty), precision=prec).double().cpu().numpy()
        e1 = rel_l2(sp, got, r_self)
        got = m.apply_bc(dev(w, ty), dev(wb, ty), u=dev(u, ty), ub=dev(ub, ty),
                         precision=prec).double().cpu().numpy()
        e2 = rel_l2(sp, got, r_frozen)
        wd = dev(w, ty)
        m.rk_substeps_bc(wd, dt, 3, dev(wb, ty), precision=prec)
        e3 = rel_l2(sp, wd.double().cpu().numpy(), ref_rk)
        b1, b3 = reduced_bars(prec, amp_s, dt * rate, n=3)
        b2 = reduced_bars(prec, amp_f)[0]
        say("      self %.3e  frozen %.3e  substeps %.3e  (bars %.1e %.1e %.1e)"
            % (e1, e2, e3, b1, b2, b3))
        assert e1 <= b1 and e2 <= b2 and e3 <= b3, (prec, kern, e1, e2, e3)
    os.environ.pop("DGCONV_FP64_KERNEL", None)
