"""Benchmark: SSP-RK3 substeps of the upwind-DG convection operator on one MI355X.

Workload (default): 2D periodic unit square, 256x256 squares x 2 triangles (131072 affine
triangles), vector P4 DG (15 basis functions per component), FP64, self-convection
div(w (x) w); initial field = L2 projection of the Taylor-Green field plus seeded N(0, 1e-3)
coefficient noise; dt = 0.1 h / (k^2 max|u|).  One step = one SSP-RK3 substep (three fused
operator-plus-stage launches).  Inputs are resident in device memory when timing starts.

The timed substeps run as one HIP graph (captured through torch's graph capture on the stream
the library launches on; the W warm-up substeps run between the capture and the timed replay),
so the launches of the 3 K kernels are submitted at once; `--no-graph` times the eager launches
instead.  The line's other measurements run before the headline's warm-up.  Beside the headline the line
carries the mixed variants on the same workload (the workload's own run length, 1000 substeps
for the 2D 256^2 x 2 P4 one, from the same state in FP64 and in each variant: time per substep,
final-state relative L2 error against FP64, the cheapest within 1e-6), the FP64 rate of the 3D
64^3 x 6 P2 workload, and the FP64 oracle on the host (all cores and one).

Prints one JSON line.  `--gpus N` with N > 1 is not supported (this benchmark runs on one GPU).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12  # MI355X FP64 vector (= FP64 matrix) peak, flop/s
PEAK_FP32 = 157.3e12
PEAK_HBM = 8.0e12

# HBM bytes per launch of the dominant kernel, from two rocprofv3 --pmc runs (FETCH_SIZE x2.00,
# WRITE_SIZE x1.00: the factors a plain 512 MiB device copy gives), mean over the stage
# launches of SSP-RK3 substeps (all three stages; not the single applications a profiled run
# makes afterwards, which read no base state); keyed by (config, precision, kernel) with the
# SHA-256 of the kernel sources the counters were taken on.  Reported as null once those
# sources change.
TRAFFIC_SOURCES = ("paper_1508_04245_amd/csrc/conv_kernels.hpp",
                   "paper_1508_04245_amd/csrc/mfma_kernels.hpp",
                   "paper_1508_04245_amd/csrc/dgconv.hip",
                   "paper_1508_04245_amd/csrc/sym_rules.hpp")
MEASURED_TRAFFIC = {
    ("c2", "fp64", "valu"): (98.3e6, "4459bb64d6ea016d"),
}


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for p in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def kernel_label(cfg, precision, fp64_kernel, n_tiles=None):
    """Which operator kernel the library runs (its default: matrix cores for FP64 when the
    element has >= 20 basis functions per component, and for 2D P3; on the VALU, two lanes per
    element for 2D P2-P4 meshes of fewer than 1024 tiles)."""
    NP, _, _ = shape_counts(cfg["dim"], cfg["k"])
    if precision == "fp64":
        kind = fp64_kernel or ("mfma" if NP >= 20 or (cfg["dim"], cfg["k"]) == (2, 3) else "valu")
    else:
        kind = "valu" if precision in ("fp32", "mixf32") else "mfma"
    if kind == "valu" and precision == "fp64":
        if cfg["dim"] == 2 and 2 <= cfg["k"] <= 4 and n_tiles is not None and n_tiles < 1024:
            return kind, "conv_pair_kernel<2,%d>" % cfg["k"]
        return kind, "conv_self_kernel<%d,%d>" % (cfg["dim"], cfg["k"])  # the pipelined path
    name = "conv_kernel" if kind == "valu" else "mconv_kernel"
    return kind, "%s<%d,%d,%s,self>" % (name, cfg["dim"], cfg["k"], precision)

CONFIGS = {
    "c1": dict(dim=2, n=16, k=2, field="tg"),
    "c2": dict(dim=2, n=256, k=4, field="tg"),
    "c3": dict(dim=3, n=32, k=3, field="tg"),
    "c4": dict(dim=3, n=64, k=2, field="fourier"),
    "c5": dict(dim=2, n=128, k=3, field="fourier"),
}


def shape_counts(dim, k):
    """Basis functions, volume points and facet points of the library's rules."""
    import paper_1508_04245_amd as dg
    np_ = (k + 1) * (k + 2) // 2 if dim == 2 else (k + 1) * (k + 2) * (k + 3) // 6
    nq = len(dg.volume_rule(dim, k)[1])
    nfq = len(dg.facet_rule(dim, k)[1])
    return np_, nq, nfq


def alg_flops_per_elem(dim, k):
    """Algorithmic flops of one fused operator+stage application per element (dense
    per-element contractions, minimal exact volume rule, each facet trace once per side)."""
    NP, NQ, NFQ = shape_counts(dim, k)
    NF = dim + 1
    interp = 2 * dim * NP * NQ
    uhat = 2 * dim * dim * NQ
    test = 4 * dim * NP * NQ          # P_m = uh . Dv_m, then R_im += w_i P_m
    trace = 2 * dim * NP * NFQ * NF   # own-side traces
    lift = 2 * dim * NP * NFQ * NF
    flux = (8 * dim + 3) * NFQ * NF
    rk = 4 * dim * NP
    return interp + uhat + test + trace + lift + flux + rk


def alg_bytes_per_elem(dim, k, esz=8):
    """Algorithmic HBM bytes per element of one fused stage launch, averaged over the three
    SSP-RK3 stages: read x (neighbour states counted once), write out, read w0 in stages 2
    and 3 only (8/3 states on average), plus geometry (J^-1, neighbour ids, element list)."""
    NP, _, _ = shape_counts(dim, k)
    state = dim * NP * esz
    geo = dim * dim * esz + 4 * (dim + 1) + 4
    return state * 8.0 / 3.0 + geo


def make_state(dg, cfg, seed=0, mesh="box"):
    from paper_1508_04245_amd import synth
    if mesh == "box":
        m = dg.Mesh.box(cfg["dim"], cfg["n"], cfg["k"])
    else:
        # the same box with jittered vertices and, for "shuffled", arbitrary element frames
        X = synth.box_elements(cfg["dim"], cfg["n"], jitter=0.15, seed=seed + 1,
                               shuffle=mesh == "shuffled")
        E, nv, d = X.shape
        m = dg.Mesh.from_arrays(d, cfg["k"], X.reshape(-1, d), np.arange(E * nv).reshape(E, nv),
                                np.ones(d))
    n = cfg["k"] + 3
    x = m.project_points(n)
    if cfg["field"] == "tg":
        f = synth.taylor_green_2d(x) if cfg["dim"] == 2 else synth.taylor_green_3d(x)
    else:
        f = synth.FourierField(cfg["dim"], seed=seed)(x)
    w = m.project(f, n) + synth.noise(m.shape, seed=seed)
    return m, w


def _oracle_worker(sp, w, elems, n, barrier, out):
    """One process of the all-cores oracle run: a warm application on its elements, then n
    timed ones after every process is ready."""
    sp.apply(w, elems=elems)
    barrier.wait()
    t0, c0 = time.perf_counter(), time.process_time()
    for _ in range(n):
        sp.apply(w, elems=elems)
    out.put((time.perf_counter() - t0, time.process_time() - c0))


def cpu_baseline(cfg, budget_s=30.0):
    """The FP64 oracle, as it stands, on the same mesh, on the host cores of this machine.

    One core: one untimed warm application, then timed applications of the full operator for
    about budget_s / 2.  All cores: the same operator applied by P processes at once (P = the
    CPUs this process may run on, at most 16), each taking a fixed contiguous share of the
    elements through the oracle's own element selection, after a warm application; timed from
    the moment all are ready to the last one's end, for about budget_s / 3.  DOF-updates/s with
    one SSP-RK3 substep = 3 applications."""
    import multiprocessing as mp
    from oracle.dg import Space
    from oracle.mesh import box_mesh
    from paper_1508_04245_amd import synth
    sp = Space(box_mesh(cfg["dim"], cfg["n"]), cfg["k"])
    w = synth.noise(sp.shape, seed=0, sd=1.0)
    ndof = int(np.prod(sp.shape))
    sp.apply(w)
    t0, c0 = time.perf_counter(), time.process_time()
    n = 0
    while True:
        sp.apply(w)
        n += 1
        if time.perf_counter() - t0 > budget_s / 2:
            break
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    one = {"value": ndof * n / 3.0 / wall, "unit": "DOF-updates/s",
           "cores": max(1, int(round(cpu / wall))), "kind": "oracle",
           "sample": "%d full operator application(s) of the FP64 NumPy oracle on the same mesh "
                     "after one warm call (%.1f s), scaled to SSP-RK3 substeps" % (n, wall)}
    visible = len(os.sched_getaffinity(0))
    P = max(1, min(16, visible))
    per_apply = wall / n
    reps = max(1, int(round(budget_s / 3 / (per_apply / P))))
    ctx = mp.get_context("fork")
    barrier, q = ctx.Barrier(P + 1), ctx.Queue()
    parts = np.array_split(np.arange(sp.mesh.E), P)
    procs = [ctx.Process(target=_oracle_worker, args=(sp, w, parts[i], reps, barrier, q))
             for i in range(P)]
    for pr in procs:
        pr.start()
    barrier.wait()
    t0 = time.perf_counter()
    res = [q.get() for _ in range(P)]
    wall_all = time.perf_counter() - t0
    for pr in procs:
        pr.join()
    cpu_all = sum(c for _, c in res)
    return {"value": ndof * reps / 3.0 / wall_all, "unit": "DOF-updates/s",
            "cores": max(1, int(round(cpu_all / wall_all))), "kind": "oracle",
            "sample": "%d full operator applications of the FP64 NumPy oracle on the same mesh by "
                      "%d processes at once (each a fixed share of the elements, after a warm "
                      "call; %.1f s), scaled to SSP-RK3 substeps (3 applications each); %d "
                      "logical CPUs visible" % (reps, P, wall_all, visible),
            "processes": P, "one_core": one}


STUDY_STEPS = {"c1": 100, "c2": 1000, "c3": 40, "c4": 200, "c5": 200}


def precision_study(dg, cfgs, tol=1e-6):
    """Each precision variant against FP64 from the same initial state: final-state relative
    L2 error after a fixed number of substeps, time per substep, and the speedup of the
    cheapest variant within `tol` (one JSON line per configuration)."""
    import torch
    dev = torch.device("cuda", 0)
    variants = [("fp64", None), ("fp64", "valu"), ("fp64", "mfma"), ("fp32", None),
                ("mixf32", None), ("f16x2", None), ("bf16x3", None)]
    for name in cfgs:
        cfg = CONFIGS[name]
        steps = STUDY_STEPS[name]
        rows = []
        ref = None
        w_host = None
        for prec, kern in variants:
            if kern:
                os.environ["DGCONV_FP64_KERNEL"] = kern
            else:
                os.environ.pop("DGCONV_FP64_KERNEL", None)
            if w_host is None:
                m, w_host = make_state(dg, cfg)
            else:
                m = dg.Mesh.box(cfg["dim"], cfg["n"], cfg["k"])  # kernel choice is per mesh
            w64 = torch.tensor(w_host, dtype=torch.float64, device=dev)
            umax = float(m.reduce("maxvel", w64)[0].item())
            dt = 0.1 / cfg["n"] / (max(cfg["k"], 1) ** 2 * umax)
            ty = torch.float32 if prec == "fp32" else torch.float64
            w = w64.to(ty)
            work = torch.empty((2,) + tuple(w.shape), dtype=ty, device=dev)
            m.rk_substeps(w.clone(), dt, 2, work=work, precision=prec)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            m.rk_substeps(w, dt, steps, work=work, precision=prec)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / 1e3 / steps
            wf = w.to(torch.float64)
            if ref is None:
                ref = wf.clone()
            d = m.reduce("l2diff", wf, ref)
            err = float(d[0].item() / d[1].item())
            rows.append({"precision": prec, "kernel": kern or "default", "rel_l2_vs_fp64": err,
                         "s_per_substep": t})
            print("%s %s/%s: %.1f us per substep" % (name, prec, kern or "default", t * 1e6),
                  file=sys.stderr, flush=True)
            del m
        os.environ.pop("DGCONV_FP64_KERNEL", None)
        t64 = rows[0]["s_per_substep"]
        for r in rows:
            r["speedup_vs_fp64_default"] = t64 / r["s_per_substep"]
        ok = [r for r in rows[1:] if r["rel_l2_vs_fp64"] <= tol]
        best = max(ok, key=lambda r: r["speedup_vs_fp64_default"]) if ok else None
        print(json.dumps({"config": name, "substeps": steps, "tol": tol, "variants": rows,
                          "best_within_tol": best}), flush=True)


def rows_study(dg, reps=50):
    """Timing of the rows beside the self-convection substeps, on the 2D 256x256x2 P4 mesh
    (FP64, inputs resident): frozen-velocity substeps, substeps with the velocity extrapolated
    in time, the pseudo-time (Richardson) update, substeps on the bounded channel, and the
    H(div) <-> DG transfers (also on the 3D 32^3 x 6 P3 mesh).  One JSON line per row, with its HBM-byte equivalent (algorithmic
    bytes: state reads and writes, neighbour states counted once, geometry)."""
    import torch
    from paper_1508_04245_amd import synth
    dev = torch.device("cuda", 0)
    cfg = CONFIGS["c2"]
    m, wh = make_state(dg, cfg)
    w = torch.tensor(wh, device=dev)
    u = torch.tensor(0.5 * wh, device=dev)
    u2 = torch.tensor(0.6 * wh, device=dev)
    E, ndof = m.info["n_elem"], m.info["n_dof"]
    st = ndof * 8
    geo = E * 48
    dt = 0.1 / cfg["n"] / (cfg["k"] ** 2 * float(m.reduce("maxvel", w)[0].item()))
    work = torch.empty((2,) + tuple(w.shape), dtype=torch.float64, device=dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(n):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / 1e3 / n

    def emit(row, sec, launches, byts, extra=None,
             workload="2D periodic 256x256x2 triangles, P4, FP64"):
        out = {"row": row, "workload": workload,
               "s_per_call": sec, "us_per_launch": sec / launches * 1e6,
               "hbm_equiv_GBps": byts / (sec / launches) / 1e9}
        out.update(extra or {})
        print(json.dumps(out), flush=True)

    t = timed(lambda: m.rk_substeps(w, dt, 1, u=u, work=work), reps)
    emit("frozen-velocity SSP-RK3 substep", t, 3, st * (8.0 / 3 + 1) + geo,
         {"dof_updates_per_s": ndof / t})
    t = timed(lambda: m.rk_substeps_extrap(w, dt, 1, 0.0, u, -dt, u2, 0.0, work=work), reps)
    emit("extrapolated-velocity SSP-RK3 substep", t, 3, st * (8.0 / 3 + 2) + geo,
         {"dof_updates_per_s": ndof / t})
    g = w.clone()
    v = w.clone()
    h = 1.0 / cfg["n"]
    tau = 0.5 * h
    ds = 1.0 / (1.0 + tau * 25 / h)
    n_it = 40
    t = timed(lambda: m.richardson(v.copy_(g), g, u, tau, ds, 0.0, n_it, work=work), 5)
    emit("pseudo-time (Richardson) update", t, n_it, st * 4 + geo,
         {"updates_per_s": n_it / t, "updates_per_call": n_it})
    # bounded channel of the same size: x bounded, inflow data on its two sides
    X = synth.box_elements(2, cfg["n"])
    mc = dg.Mesh.from_arrays(2, cfg["k"], X.reshape(-1, 2), np.arange(X.shape[0] * 3).reshape(-1, 3),
                             np.array([0.0, 1.0]))
    xb = mc.boundary_points()
    wb = torch.tensor(np.stack([np.ones(xb.shape[:2]), 0.5 * np.sin(2 * np.pi * xb[..., 1])], -1),
                      device=dev)
    wc = w.clone()
    t = timed(lambda: mc.rk_substeps_bc(wc, dt, 1, wb, work=work), reps)
    emit("bounded-channel SSP-RK3 substep", t, 3, st * 8.0 / 3 + geo,
         {"dof_updates_per_s": ndof / t, "n_bfacet": mc.info["n_bfacet"]})
    n_w, n_f = m.hdiv_size()
    uh = torch.randn(n_w, dtype=torch.float64, device=dev)
    out = torch.empty_like(w)
    t = timed(lambda: m.to_dg(uh, out=out), reps)
    emit("transfer I (W_h -> V_h)", t, 1, n_w * 8 + st + E * 44, {"n_hdiv": n_w})
    gt = torch.empty(n_w, dtype=torch.float64, device=dev)
    t = timed(lambda: m.transfer_transpose(w, out=gt), reps)
    # bytes of both passes, reported per launch as their mean
    emit("transfer I^T (V_h' -> W_h')", t, 2, (st + 2 * E * 2 * m.np * 8 + n_w * 8 + E * 44) / 2,
         {"n_hdiv": n_w})
    # the same transfers in 3D on the 32^3 x 6 tetrahedra P3 mesh (facet codes 16 B and J^-1
    # 72 B per element)
    m3 = dg.Mesh.box(3, 32, 3)
    E3 = m3.info["n_elem"]
    st3 = m3.info["n_dof"] * 8
    n_w3, _ = m3.hdiv_size()
    uh3 = torch.randn(n_w3, dtype=torch.float64, device=dev)
    out3 = torch.empty((E3, 3, m3.np), dtype=torch.float64, device=dev)
    wl3 = "3D periodic 32^3 x 6 tetrahedra, P3, FP64"
    t = timed(lambda: m3.to_dg(uh3, out=out3), reps)
    emit("transfer I (W_h -> V_h)", t, 1, n_w3 * 8 + st3 + E3 * 88, {"n_hdiv": n_w3},
         workload=wl3)
    gt3 = torch.empty(n_w3, dtype=torch.float64, device=dev)
    t = timed(lambda: m3.transfer_transpose(out3, out=gt3), reps)
    emit("transfer I^T (V_h' -> W_h')", t, 2, (st3 + 2 * st3 + n_w3 * 8 + E3 * 88) / 2,
         {"n_hdiv": n_w3}, workload=wl3)
    del m3, uh3, out3, gt3
    # the learned macro-step on the 2D 128^2 x 2 P3 workload (32768 elements; the network
    # untrained: the timing does not depend on its weights): the network's forward pass over
    # every element (BF16 inputs in, FP32 outputs), a macro-step on the network path (accepted,
    # defect check included, host decision) and the 8 plain substeps it replaces
    from paper_1508_04245_amd import surrogate as S
    m5 = dg.Mesh.box(2, 128, 3)
    sur = dg.Surrogate(m5, M=8)
    sur.load(S.init_params(0, sur.n_params))
    w5 = torch.tensor(S.initial_state(m5, 1), device=dev)
    scale5 = m5.reduce("maxvel", w5)[:1].contiguous()
    x5 = sur.features(w5, scale5)
    E5 = m5.info["n_elem"]
    wl5 = "2D periodic 128x128x2 triangles, P3, FP64 state; network 80-256-256-256-20 BF16"
    t = timed(lambda: sur.forward(x5), reps)
    mlp_flops = 2.0 * (80 * 256 + 2 * 256 * 256 + 256 * 20) * E5
    emit("network forward (every element)", t, 1, E5 * (80 * 4 + 20 * 4) + sur.n_params * 2,
         {"tflops": mlp_flops / t / 1e12, "frac_bf16_peak": mlp_flops / t / 2.5e15},
         workload=wl5)
    dt5 = 0.1 / 128 / (9 * float(scale5[0].item()))
    mwork = torch.empty((3,) + tuple(w5.shape), dtype=torch.float64, device=dev)
    w5b = w5.clone()
    t = timed(lambda: sur.macro_step(w5b, dt5, float("inf"), work=mwork), 20)
    emit("macro-step, network path (M = 8)", t, 1, 0, {"ms": t * 1e3}, workload=wl5)
    work5 = torch.empty((2,) + tuple(w5.shape), dtype=torch.float64, device=dev)
    t = timed(lambda: m5.rk_substeps(w5b, dt5, 8, work=work5), 20)
    emit("8 plain SSP-RK3 substeps", t, 24, m5.info["n_dof"] * 8 * 8.0 / 3 + E5 * 48 * 3,
         {"ms": t * 1e3}, workload=wl5)

def timed_substeps(m, w, dt, steps, work, prec, graph=True, warm=0, warm_state=None):
    """Time `steps` SSP-RK3 substeps in place on w with HIP events on the current stream (the
    one the library launches on).  graph: capture the substeps into one HIP graph first
    (nothing runs during a capture) and time its replay.  warm: untimed substeps enqueued
    after the capture and right before the timed region, so that it starts on a busy device,
    on warm_state (a state of the same shape and type; w itself when None).  The library's
    first-call set-up must have happened before (any call on this mesh and precision).
    Returns (GPU seconds, wall)."""
    import torch
    stream = torch.cuda.current_stream()
    g = None
    if graph and steps > 0:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            m.rk_substeps(w, dt, steps, work=work, precision=prec)
        torch.cuda.synchronize()
    if warm > 0:
        m.rk_substeps(w if warm_state is None else warm_state, dt, warm, work=work,
                      precision=prec)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    if g is not None:
        g.replay()
    else:
        m.rk_substeps(w, dt, steps, work=work, precision=prec)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    del g
    return ev0.elapsed_time(ev1) / 1e3, wall


def mixed_variants(m, w_start, dt, steps, graph=True, tol=1e-6):
    """`steps` substeps (the workload's own run length) from the same state in FP64 and in
    every lower-precision variant: time per substep, final-state relative L2 error against
    the FP64 result, speedup over FP64, and the cheapest variant within tol."""
    import torch
    w_ref = w_start.to(torch.float64).clone()
    work64 = torch.empty((2,) + tuple(w_ref.shape), dtype=torch.float64, device=w_ref.device)
    # every run starts from w_start; the warm-up substeps before each timed region run on a
    # copy (the same work buffer, which each run overwrites before reading)
    t64, _ = timed_substeps(m, w_ref, dt, steps, work64, "fp64", graph, warm=20,
                            warm_state=w_ref.clone())
    del work64
    rows = []
    for prec in ("fp32", "mixf32", "bf16x3", "f16x2"):
        ty = torch.float32 if prec == "fp32" else torch.float64
        w = w_start.to(ty).clone()
        work = torch.empty((2,) + tuple(w.shape), dtype=ty, device=w.device)
        m.rk_substeps(w.clone(), dt, 1, work=work, precision=prec)  # first-call setup
        torch.cuda.synchronize()
        t, _ = timed_substeps(m, w, dt, steps, work, prec, graph, warm=20, warm_state=w.clone())
        d = m.reduce("l2diff", w.to(torch.float64).contiguous(), w_ref)
        err = float(d[0].item() / d[1].item())
        rows.append({"precision": prec, "s_per_substep": t / steps, "rel_l2_vs_fp64": err,
                     "speedup_vs_fp64": t64 / t})
    ok = [r for r in rows if r["rel_l2_vs_fp64"] <= tol]
    best = max(ok, key=lambda r: r["speedup_vs_fp64"]) if ok else None
    return {"substeps": steps, "fp64_s_per_substep": t64 / steps, "tol": tol,
            "variants": rows, "best_within_tol": best}


def c4_rate(dg, graph=True, steps=20):
    """FP64 rate of the 3D periodic 64^3 x 6 tetrahedra P2 workload (random Fourier field,
    projected with 3 points per direction: the timing does not depend on the values)."""
    import torch
    from paper_1508_04245_amd import synth
    cfg = CONFIGS["c4"]
    m = dg.Mesh.box(cfg["dim"], cfg["n"], cfg["k"])
    x = m.project_points(3)
    w = torch.tensor(m.project(synth.FourierField(3, seed=0)(x), 3), device="cuda")
    del x
    umax = float(m.reduce("maxvel", w)[0].item())
    dt = 0.1 / cfg["n"] / (cfg["k"] ** 2 * umax)
    work = torch.empty((2,) + tuple(w.shape), dtype=torch.float64, device="cuda")
    m.rk_substeps(w, dt, 1, work=work)
    torch.cuda.synchronize()
    t, _ = timed_substeps(m, w, dt, steps, work, "fp64", graph, warm=10)
    E = m.info["n_elem"]
    per_launch = t / (3 * steps)
    flops = alg_flops_per_elem(3, 2) * E
    return {"workload": "3D periodic 64^3 x6 tetrahedra (1572864), vector P2, FP64",
            "substeps": steps, "us_per_launch": per_launch * 1e6,
            "dof_updates_per_s": m.info["n_dof"] * steps / t,
            "roofline_frac": flops / per_launch / PEAK_FP64,
            "hbm_equiv_GBps": alg_bytes_per_elem(3, 2) * E / per_launch / 1e9}



def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--precision", default="fp64",
                    choices=["fp64", "fp32", "mixf32", "f16x2", "bf16x3"])
    ap.add_argument("--fp64-kernel", default=None, choices=["valu", "mfma"],
                    help="FP64 operator kernel (default: the library's choice)")
    ap.add_argument("--n", type=int, default=None, help="override the mesh size (experiments)")
    ap.add_argument("--mesh", default="box", choices=["box", "jittered", "shuffled"],
                    help="jittered: the box with moved vertices; shuffled: also arbitrary "
                         "element vertex orders (unstructured element frames)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="time eager launches instead of one captured HIP graph")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline (no mixed variants, no 3D P2 rate)")
    ap.add_argument("--cpu-budget", type=float, default=30.0)
    ap.add_argument("--rows", action="store_true",
                    help="time the rows beside the self-convection substeps (one JSON line each)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only a plain 512 MiB device copy, three times (the reference "
                         "dispatch for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--precision-study", default=None, metavar="CFGS",
                    help="comma-separated configs: final-state error and speedup of every "
                         "precision variant against FP64 (one JSON line per config)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the path's sharding over several GPUs (element "
              "slabs with one boundary exchange per stage) is designed, not built; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    if args.fp64_kernel:
        os.environ["DGCONV_FP64_KERNEL"] = args.fp64_kernel
    import torch
    import paper_1508_04245_amd as dg
    dg.lib()
    if args.copy_calibration:
        x = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 8, "copies": 3}), flush=True)
        return
    if args.precision_study:
        precision_study(dg, args.precision_study.split(","))
        return
    if args.rows:
        rows_study(dg)
        return
    cfg = dict(CONFIGS[args.config])
    if args.n:
        cfg["n"] = args.n
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    m, w_host = make_state(dg, cfg, mesh=args.mesh)
    ty = torch.float32 if args.precision == "fp32" else torch.float64
    w = torch.tensor(w_host, dtype=ty, device=dev)
    w64 = torch.tensor(w_host, dtype=torch.float64, device=dev)
    umax = float(m.reduce("maxvel", w64)[0].item())
    h = 1.0 / cfg["n"]
    dt = 0.1 * h / (max(cfg["k"], 1) ** 2 * umax)
    stream = torch.cuda.current_stream()
    work = torch.empty((2,) + tuple(w.shape), dtype=ty, device=dev)
    prec = args.precision
    # the library's first-call set-up (device tables) by one application, outside the graph
    # capture; the W warm-up substeps run after the capture, right before the timed region
    m.apply(w, out=torch.empty_like(w), precision=prec)
    torch.cuda.synchronize()
    w_start = w.clone()
    # the other measurements of the line run first (the 3D workload's rate, then the mixed
    # variants over the workload's own run length), so that the headline's timed substeps,
    # like the profiler's mean over many launches, see the device at its working clocks
    extra = {}
    if not args.no_extra and prec == "fp64" and not args.n and args.mesh == "box":
        if args.config != "c4":
            extra["c4_fp64"] = c4_rate(dg, not args.no_graph)
        extra["mixed"] = mixed_variants(m, w_start, dt, STUDY_STEPS[args.config],
                                        not args.no_graph)
    gpu_s, wall = timed_substeps(m, w, dt, args.steps, work, prec, not args.no_graph,
                                 warm=args.warmup)
    ndof = m.info["n_dof"]
    value = ndof * args.steps / gpu_s
    launches = 3 * args.steps
    per_launch = gpu_s / max(1, launches)
    E = m.info["n_elem"]
    flops = alg_flops_per_elem(cfg["dim"], cfg["k"]) * E
    byts = alg_bytes_per_elem(cfg["dim"], cfg["k"], esz=8 if ty == torch.float64 else 4) * E
    peak = PEAK_FP64 if ty == torch.float64 else PEAK_FP32
    finite = torch.isfinite(w).all().item()
    # single operator applications (mode r = L(w), no Runge-Kutta stage), same stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    r_out = torch.empty_like(w)
    n_app = max(10, args.steps // 10)
    ev0.record(stream)
    for _ in range(n_app):
        m.apply(w, out=r_out, precision=prec)
    ev1.record(stream)
    torch.cuda.synchronize()
    apply_s = ev0.elapsed_time(ev1) / 1e3 / n_app
    kind, label = kernel_label(cfg, args.precision, args.fp64_kernel, m.info["n_tiles"])
    tr = MEASURED_TRAFFIC.get((args.config, args.precision, kind))
    traffic = (tr[0] if tr and not args.n and args.mesh == "box" and tr[1] == kernel_sources_hash()
               else None)
    out = {
        "metric": "DG convection DOF-updates/s (SSP-RK3 substeps), FP64",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_s * 1e3 / max(1, args.steps),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if ty == torch.float64 else "f32",
        "data": "synthetic",
        "config": {"workload": "2D periodic unit square %dx%d x2 triangles (%d), vector P%d DG "
                               "(%d dofs/component), self-convection, SSP-RK3 dt=%.4g"
                               % (cfg["n"], cfg["n"], E, cfg["k"], m.np, dt)
                   if cfg["dim"] == 2 else
                   "3D periodic unit cube %d^3 x6 tets (%d), vector P%d DG, SSP-RK3 dt=%.4g"
                   % (cfg["n"], E, cfg["k"], dt),
                   "config": args.config, "n_dof": ndof, "precision": args.precision,
                   "mesh": args.mesh},
        "roofline": {"bound": "alu", "achieved": flops / per_launch / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": flops / per_launch / peak, "traffic": traffic,
                     "traffic_unit": "B/launch", "alg_bytes": byts, "kernel": label,
                     "launch_us": per_launch * 1e6,
                     "hbm_equiv_GBps": byts / per_launch / 1e9},
        "dof_applies_per_s": ndof / apply_s,
        "wall_s": wall,
        "final_state_finite": bool(finite),
    }
    out["graph"] = not args.no_graph
    out.update(extra)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_budget)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
