"""What the trained macro-step network gains over the plain method on the 2D 128x128x2 P3
workload (32768 triangles, M = 8 substeps per macro-step).

The network is trained on the GPU by the library's own kernels (BF16 forward and backward,
Adam on FP32 master weights) on trajectories of the plain SSP-RK3 substeps (seeds 1..96), and
evaluated on unseen seeds (10001..10004) from states of the plain trajectory:

* acceptance rate of the a-posteriori check at tol = 2x the plain method's own median
  trapezoid defect;
* time per macro-step (network path, every candidate accepted) against the 8 plain substeps,
  HIP events on one stream, and the network's forward pass alone over every element;
* error of the network's increment against the plain judge, beside the two baselines of the
  same cost class: forward Euler over tau = M dt and one SSP-RK3 step of size tau.

Only what holds is asserted: the fallback is the plain substeps bit for bit, a rejected
macro-step leaves the plain result, and every number is finite.  The numbers are printed as
one JSON line (the measured gain, whatever it is).
"""
import json

import numpy as np
import pytest

from gpu_common import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_trained_macro_step_gain():
    import paper_1508_04245_amd as dg
    from paper_1508_04245_amd import surrogate as S
    assert torch.cuda.is_available()
    say("case macro-step gain, 2D 128x128x2 P3, M = 8")
    mesh = dg.Mesh.box(2, 128, 3)
    sur = dg.Surrogate(mesh, M=8)
    sur.load(S.init_params(0, sur.n_params))
    X, T = S.generate(mesh, sur, range(1, 97), 8, 1024)
    torch.cuda.synchronize()
    say("   %d training samples" % X.shape[0])
    hist = S.train(sur, X, T, epochs=3)
    assert all(np.isfinite(l) for _, l in hist)
    probe = S.evaluate(mesh, sur, range(10001, 10005), 2, tol=np.inf)
    tol = 2.0 * float(np.median(probe["rho_plain"]))
    res = S.evaluate(mesh, sur, range(10001, 10005), 2, tol=tol)
    h = 1.0 / 128
    w0 = torch.tensor(S.initial_state(mesh, 10001), device="cuda")
    s0 = float(mesh.reduce("maxvel", w0)[0].item())
    dt = 0.1 * h / (9 * s0)
    # fallback at tol = 0: the plain substeps, bit for bit
    ref = w0.clone()
    mesh.rk_substeps(ref, dt, 8)
    ws = w0.clone()
    acc, rho = sur.macro_step(ws, dt, 0.0)
    assert not acc and torch.equal(ws, ref)
    # timing: 8 plain substeps against one network macro-step (accepted), same stream
    work = torch.empty((2,) + tuple(w0.shape), dtype=torch.float64, device="cuda")
    mwork = torch.empty((3,) + tuple(w0.shape), dtype=torch.float64, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    wa, wb = w0.clone(), w0.clone()
    for _ in range(3):
        mesh.rk_substeps(wa, dt, 8, work=work)
        sur.macro_step(wb, dt, np.inf, work=mwork)
    reps = 20
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        mesh.rk_substeps(wa, dt, 8, work=work)
    ev[1].record()
    torch.cuda.synchronize()
    ev[2].record()
    for _ in range(reps):
        sur.macro_step(wb, dt, np.inf, work=mwork)
    ev[3].record()
    torch.cuda.synchronize()
    t_plain = ev[0].elapsed_time(ev[1]) / reps
    t_net = ev[2].elapsed_time(ev[3]) / reps
    # the network alone on every element (inputs of w0), the inference path of the macro-step
    scale = mesh.reduce("maxvel", w0)[:1].contiguous()
    xin = sur.features(w0, scale)
    for _ in range(3):
        sur.forward(xin)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        sur.forward(xin)
    ev[1].record()
    torch.cuda.synchronize()
    t_mlp = ev[0].elapsed_time(ev[1]) / reps
    mlp_flops = 2.0 * (80 * 256 + 2 * 256 * 256 + 256 * 20) * mesh.E
    acc_rate = res["accepted"] / res["macro_steps"]
    out = {"study": "macro-step gain", "workload": "2D periodic 128x128x2 triangles, P3, M=8",
           "train_samples": int(X.shape[0]), "loss_first": hist[0][1], "loss_last": hist[-1][1],
           "tol": tol, "acceptance": acc_rate,
           "rho_network_median": float(np.median(probe["rho"])),
           "rho_plain_median": float(np.median(probe["rho_plain"])),
           "err_increment_network_median": float(np.median(probe["err_increment"])),
           "err_increment_euler_median": float(np.median(probe["err_increment_euler"])),
           "err_increment_rk3_coarse_median": float(np.median(probe["err_increment_rk3_coarse"])),
           "ms_plain_8_substeps": t_plain, "ms_network_macro_step": t_net,
           "ms_network_forward_all_elements": t_mlp,
           "network_forward_tflops": mlp_flops / (t_mlp * 1e-3) / 1e12,
           "speedup_if_all_accepted": t_plain / t_net,
           "speedup_at_measured_acceptance": t_plain / (t_net + (1 - acc_rate) * t_plain)}
    say("   " + json.dumps(out))
    for v in out.values():
        if isinstance(v, float):
            assert np.isfinite(v)
    assert 0.0 <= acc_rate <= 1.0
