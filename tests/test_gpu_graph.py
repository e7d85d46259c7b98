"""SSP-RK3 substeps captured in a HIP graph (torch's graph capture on its capture stream: the
library launches on the stream it is given, here the capturing one) must replay exactly like
the eager calls.  The graph is replayed several times with the program's own eager work and
synchronisations between the replays, and every replay is compared with the eager result from
the same state, bit for bit (the kernels are deterministic).  The substeps record no memset
or allocation, so nothing but kernel nodes enters the graph; every table upload and work
buffer exists before the capture.
"""
import numpy as np
import pytest

from gpu_common import initial_state, oracle_space, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import paper_1508_04245_amd as dg
    assert torch.cuda.is_available(), "GPU tests need a device"
    dg.lib()
    return dg


@pytest.mark.parametrize("prec", ["fp64", "mixf32", "bf16x3", "fp32"])
def test_graph_replay_matches_eager(dg, prec):
    dim, N, k = 2, 32, 4
    say("case graph replay %s 2D %dx%dx2 P%d" % (prec, N, N, k))
    sp = oracle_space(dim, N, k)
    ty = torch.float32 if prec == "fp32" else torch.float64
    w0 = torch.tensor(initial_state(sp, seed=2), dtype=ty, device="cuda")
    m = dg.Mesh.box(dim, N, k)
    dt = 1e-4
    work_g = torch.empty((2,) + tuple(w0.shape), dtype=ty, device="cuda")
    work_e = torch.empty_like(work_g)
    # first calls upload the mesh tables and the matrix-core fragments (synchronous)
    m.rk_substeps(w0.clone(), dt, 1, work=work_e, precision=prec)
    torch.cuda.synchronize()
    wg = w0.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        m.rk_substeps(wg, dt, 3, work=work_g, precision=prec)
    torch.cuda.synchronize()
    assert torch.equal(wg, w0)  # capture runs nothing
    we = w0.clone()
    for rep in range(4):
        m.rk_substeps(we, dt, 3, work=work_e, precision=prec)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(wg, we), rep
        # eager work between replays, on the same buffers the graph does not own
        r = m.apply(we, precision=prec)
        assert torch.isfinite(r).all()
        torch.cuda.synchronize()
    say("   4 replays equal to the eager substeps")
