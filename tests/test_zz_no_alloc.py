"""dg_reduce_noalloc (the reductions with their partial results in the library's static device
array, no allocation) against dg_reduce on the same inputs, through the C ABI.

Both run the same kernels in the same order, so the results must agree bit for bit.  Two
meshes in a row, the second smaller, so the second call finds the first call's partial results
still in the shared array and must not read them.
"""
import numpy as np
import pytest
import torch

import paper_1508_04245_amd as dg

pytestmark = pytest.mark.gpu

NOUT = {"maxvel": 1, "energy": 1, "momentum": None, "l2diff": 2, "nonfinite": 1}


def _case(dim, n, k, seed):
    m = dg.Mesh.box(dim, n, k)
    rng = np.random.default_rng(seed)
    a = torch.tensor(rng.normal(size=m.shape), device="cuda")
    b = torch.tensor(rng.normal(size=m.shape), device="cuda")
    bad = a.clone()
    bad.view(-1)[:: max(1, bad.numel() // 7)] = float("nan")
    return m, a, b, bad


@pytest.mark.parametrize("first,second", [((2, 64, 4), (2, 8, 2)), ((3, 10, 2), (3, 2, 1))])
def test_noalloc_matches_dg_reduce(first, second):
    torch.cuda.set_device(0)
    for seed, (dim, n, k) in enumerate((first, second)):
        m, a, b, bad = _case(dim, n, k, seed)
        print("case dim %d n %d k %d" % (dim, n, k), flush=True)
        m.reduce("energy", a)  # uploads the mesh tables (the no-alloc call does not)
        for what, nout in NOUT.items():
            nout = nout or dim
            x = bad if what == "nonfinite" else a
            y = b if what == "l2diff" else None
            ref = m.reduce(what, x, y)
            out = torch.full((4,), float("inf"), dtype=torch.float64, device="cuda")
            m.reduce_noalloc(what, x, y, out)
            torch.cuda.synchronize()
            r, o = ref.cpu().numpy()[:nout], out.cpu().numpy()[:nout]
            assert np.all(np.isfinite(r)), (what, r)
            assert np.array_equal(r, o), (what, r, o)
            assert np.all(out.cpu().numpy()[nout:] == np.inf)  # nothing written beyond
            if what == "nonfinite":
                assert o[0] > 0
