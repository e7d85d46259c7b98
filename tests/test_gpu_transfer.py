"""GPU parity of the H(div) <-> DG transfer operators (Sec. 2.4) against the oracle:
I u (dg_transfer_to_dg) and I^T f (dg_transfer_transpose) on jittered, shuffled-frame and
bounded 2D meshes with ragged last blocks, degrees 1..6, and on a 64x64x2 box; in 3D on
jittered, shuffled-frame (every facet orientation) and bounded tetrahedral meshes, degrees
1..4, and on an 8x8x8x6 box.
Every test prints its case before touching the GPU.
"""
import numpy as np
import pytest

from gpu_common import say
from oracle.hdiv import HdivSpace
from oracle.mesh import Mesh, box_mesh

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import paper_1508_04245_amd as dg
    assert torch.cuda.is_available(), "GPU tests need a device"
    dg.lib()
    return dg


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def mesh(kind, N, seed, dim=2):
    if dim == 2:
        per = (False, True) if kind == "bounded" else (True, True)
    else:
        per = (False, True, False) if kind == "bounded" else (True, True, True)
    base = box_mesh(dim, N, jitter=0.0 if kind == "box" else 0.15, seed=seed, periodic=per)
    if kind in ("shuffled", "bounded"):
        rng = np.random.default_rng(seed)
        X = base.X.copy()
        for t in range(base.E):
            X[t] = X[t][rng.permutation(dim + 1)]
        return Mesh(X, base.period)
    return base


CASES = [(2, "jittered", 9, k) for k in (1, 2, 3)] + [(2, "shuffled", 7, k) for k in (4, 5, 6)] + \
        [(2, "bounded", 7, 2), (2, "bounded", 6, 4), (2, "box", 64, 4)] + \
        [(3, "jittered", 3, 1), (3, "shuffled", 3, 2), (3, "shuffled", 2, 3), (3, "bounded", 3, 3),
         (3, "bounded", 2, 1), (3, "box", 8, 3), (3, "shuffled", 2, 4), (3, "bounded", 2, 4)]


@pytest.mark.parametrize("dim,kind,N,k", CASES)
def test_transfer_vs_oracle(dg, dim, kind, N, k):
    say("case transfer %dD %s N=%d k=%d" % (dim, kind, N, k))
    om = mesh(kind, N, seed=k, dim=dim)
    H = HdivSpace(om, k)
    E = om.E
    m = dg.Mesh.from_arrays(dim, k, om.X.reshape(-1, dim),
                            np.arange(E * (dim + 1)).reshape(E, dim + 1), om.period)
    assert m.hdiv_size() == (H.N, H.n_facets)
    rng = np.random.default_rng(11 + k)
    u = rng.normal(size=H.N)
    F = rng.normal(size=(E, dim, m.np))
    ref = H.to_dg(u)
    got = m.to_dg(dev(u)).cpu().numpy()
    e1 = np.abs(got - ref).max() / np.abs(ref).max()
    reft = H.transpose(F)
    gott = m.transfer_transpose(dev(F)).cpu().numpy()
    e2 = np.abs(gott - reft).max() / np.abs(reft).max()
    say("   I: max rel %.3e   I^T: max rel %.3e" % (e1, e2))
    assert e1 <= 1e-12 and e2 <= 1e-12
