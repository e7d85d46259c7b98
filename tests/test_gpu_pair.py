"""The two-lanes-per-element FP64 kernel (2D self-convection, P2-P4) against the oracle and
against the one-lane kernel on the same mesh.

The library takes it on 2D periodic meshes of fewer than 1024 tiles; DGCONV_PAIR=0 selects
the one-lane kernel.  Cases: meshes of several tiles (two element classes, so both lanes of
a pair and both halves of a tile are busy) and a mesh whose only tile is partly empty
(padded lane pairs redo an element and store nothing).  One application and three SSP-RK3
substeps (the fused stage epilogue, in place), FP64 bar 1e-12 against the oracle; the two
kernels agree to 1e-13 (same arithmetic, different rounding order of the normal speed and
of J^-1 w).
"""
import os

import numpy as np
import pytest

from gpu_common import initial_state, rel_l2, say
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


def mesh_with(dg, pair, N, k):
    os.environ["DGCONV_PAIR"] = "1" if pair else "0"
    try:
        return dg.Mesh.box(2, N, k)
    finally:
        os.environ.pop("DGCONV_PAIR", None)


@pytest.mark.parametrize("N,k", [(24, 2), (20, 3), (16, 4), (5, 4)])
def test_pair_kernel_against_oracle_and_one_lane_kernel(dg, N, k):
    say("case pair kernel 2D N=%d k=%d" % (N, k))
    sp = Space(box_mesh(2, N), k)
    w = initial_state(sp, field="fourier", seed=11, sd=1e-3)
    assert dg.Mesh.box(2, N, k).info["n_tiles"] < 1024  # the default takes the pair kernel
    mp, m1 = mesh_with(dg, True, N, k), mesh_with(dg, False, N, k)
    wd = torch.tensor(w, device="cuda")
    rp = mp.apply(wd).cpu().numpy()
    r1 = m1.apply(wd).cpu().numpy()
    ref = sp.apply(w)
    e_or, e_11 = rel_l2(sp, rp, ref), rel_l2(sp, rp, r1)
    say("   apply: pair vs oracle %.3e, pair vs one-lane %.3e" % (e_or, e_11))
    assert e_or <= 1e-12 and e_11 <= 1e-13
    dt = cfl_dt(1.0 / N, k, sp.max_speed(w))
    a, b = wd.clone(), wd.clone()
    mp.rk_substeps(a, dt, 3)
    m1.rk_substeps(b, dt, 3)
    sref = sp.ssprk3(w, dt, 3)
    a, b = a.cpu().numpy(), b.cpu().numpy()
    e_or, e_11 = rel_l2(sp, a, sref), rel_l2(sp, a, b)
    say("   3 substeps: pair vs oracle %.3e, pair vs one-lane %.3e" % (e_or, e_11))
    assert e_or <= 1e-12 and e_11 <= 1e-13
    assert np.all(np.isfinite(a))
