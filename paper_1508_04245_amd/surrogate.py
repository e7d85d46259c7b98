"""Driver of the learned macro-step: data from the plain method, training, evaluation.

All arithmetic runs in libdgconv.so (the plain SSP-RK3 substeps that generate and check the
data, the feature gather, the BF16 network kernels, Adam, the macro-step with its defect check
and fallback); this module only sequences calls and holds the data in device memory.

Workload (2D periodic unit square, 128 x 128 squares x 2 triangles, vector P3 DG): fields
from the seeded random Fourier generator (16 modes, |kappa| <= 4, Leray-projected, |kappa|^-2
amplitudes, unit RMS), projected onto the DG space; dt = 0.1 h / (k^2 max|w0|); one
macro-step replaces M = 8 substeps.

The same network also serves as a learned initial guess of the pseudo-time (Richardson)
iteration for v + tau (M^V)^-1 C^V(u) v = g (Sec. 3.3) with u := g frozen, tau = 0.5 h / max|g|:
trained on the remainder of the converged solution beyond g + tau r(g) (--warm-start).

Usage: python -m paper_1508_04245_amd.surrogate [--train-seeds 2000] ...  (prints JSON)
"""
import argparse
import json
import time

import numpy as np

from . import Mesh, Surrogate, synth


def initial_state(mesh, seed, n_pts=4):
    x = mesh.project_points(n_pts)
    return mesh.project(synth.FourierField(2, seed=seed)(x), n_pts)


def init_params(seed, n_params):
    """He-style initialisation (last layer fan-in scaled), zero biases."""
    rng = np.random.default_rng(seed)
    sizes = [(256, 80), (256, 256), (256, 256), (20, 256)]
    parts = []
    for li, (o, i) in enumerate(sizes):
        sd = np.sqrt((1.0 if li == 3 else 2.0) / i)
        parts.append(rng.normal(0.0, sd, size=o * i))
        parts.append(np.zeros(o))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == n_params
    return p


def initial_states(mesh, seeds, workers=8):
    """Initial states of several seeds, evaluated on host threads (NumPy releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    x = mesh.project_points(4)
    f = lambda s: mesh.project(synth.FourierField(2, seed=s)(x), 4)
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(f, seeds))


def generate(mesh, sur, seeds, n_macro, per_snapshot, M=8, k=3, device="cuda", chunk=64):
    """Samples (x, t) from trajectories of the plain method: for each seed, n_macro macro
    intervals of M substeps; per interval `per_snapshot` random elements."""
    import torch
    h = 1.0 / round(np.sqrt(mesh.E / 2))
    xs, ts = [], []
    gen = torch.Generator(device=device)
    seeds = list(seeds)
    for c0 in range(0, len(seeds), chunk):
        batch = seeds[c0:c0 + chunk]
        for seed, w_host in zip(batch, initial_states(mesh, batch)):
            _trajectory(mesh, sur, seed, w_host, n_macro, per_snapshot, M, k, h, gen, xs, ts,
                        device)
    return torch.cat(xs), torch.cat(ts)


def _trajectory(mesh, sur, seed, w_host, n_macro, per_snapshot, M, k, h, gen, xs, ts, device):
    """One trajectory of the plain method from w_host; appends the samples to xs, ts."""
    import torch
    gen.manual_seed(int(seed))
    w = torch.tensor(w_host, device=device)
    s0 = float(mesh.reduce("maxvel", w)[0].item())
    dt = 0.1 * h / (k * k * s0)
    for _ in range(n_macro):
        scale = mesh.reduce("maxvel", w)
        elems = torch.randint(0, mesh.E, (per_snapshot,), generator=gen, device=device,
                              dtype=torch.int32)
        x = sur.features(w, scale, elems)
        r0 = mesh.apply(w)
        w1 = w.clone()
        mesh.rk_substeps(w1, dt, M)
        xs.append(x)
        ts.append(sur.targets(w, w1, r0, scale, M * dt, elems))
        w = w1


def train(sur, X, T, epochs, batch=4096, lr0=1e-3, lr1=1e-5, seed=0, log=None):
    import torch
    n = X.shape[0]
    steps = epochs * (n // batch)
    gen = torch.Generator(device=X.device)
    gen.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device=X.device)
    hist = []
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen, device=X.device)
        for b in range(n // batch):
            idx = perm[b * batch:(b + 1) * batch]
            lr = lr1 + 0.5 * (lr0 - lr1) * (1 + np.cos(np.pi * step / max(1, steps)))
            sur.train_step(X[idx].contiguous(), T[idx].contiguous(), lr, loss)
            step += 1
            if step % 200 == 0 or step == steps:
                hist.append((step, float(loss.item())))
                if log:
                    log("step %d loss %.4e" % hist[-1])
    return hist


def evaluate(mesh, sur, seeds, n_macro, tol, M=8, k=3, device="cuda"):
    """Run the surrogate and the plain method side by side from the same initial states."""
    import torch
    h = 1.0 / round(np.sqrt(mesh.E / 2))
    res = {"accepted": 0, "macro_steps": 0, "err_state": [], "err_increment": [],
           "rho": [], "rho_plain": [], "err_increment_euler": [], "err_increment_rk3_coarse": []}
    for seed in seeds:
        w0 = torch.tensor(initial_state(mesh, seed), device=device)
        s0 = float(mesh.reduce("maxvel", w0)[0].item())
        dt = 0.1 * h / (k * k * s0)
        ws, wp = w0.clone(), w0.clone()
        for _ in range(n_macro):
            start = wp.clone()
            mesh.rk_substeps(wp, dt, M)
            # the plain method's own trapezoid defect (calibration of tol)
            r0, r1 = mesh.apply(start), mesh.apply(wp)
            d = wp - start
            e = d - 0.5 * M * dt * (r0 + r1)
            res["rho_plain"].append(float(torch.linalg.norm(e) / torch.linalg.norm(d)))
            # baselines of the same cost class: forward Euler over tau (the network's
            # starting point) and one SSP-RK3 step of size tau
            eu = start + M * dt * r0
            res["err_increment_euler"].append(float(torch.linalg.norm(eu - wp) / torch.linalg.norm(d)))
            cr = start.clone()
            mesh.rk_substeps(cr, M * dt, 1)
            res["err_increment_rk3_coarse"].append(float(torch.linalg.norm(cr - wp) / torch.linalg.norm(d)))
            # surrogate from the plain state (one-step error) on a copy
            ws = start.clone()
            acc, rho = sur.macro_step(ws, dt, tol)
            res["accepted"] += int(acc)
            res["macro_steps"] += 1
            res["rho"].append(rho)
            res["err_state"].append(float(torch.linalg.norm(ws - wp) / torch.linalg.norm(wp)))
            res["err_increment"].append(float(torch.linalg.norm(ws - wp) / torch.linalg.norm(d)))
    return res


def timing(mesh, sur, dt, reps=20, M=8, device="cuda"):
    """Per macro-step time of the plain substeps and of the surrogate path (network, defect
    check and the host decision; measured with every candidate accepted)."""
    import torch
    w = torch.tensor(initial_state(mesh, 12345), device=device)
    work = torch.empty((2,) + tuple(w.shape), dtype=torch.float64, device=device)
    tol = np.inf
    for _ in range(3):
        mesh.rk_substeps(w.clone(), dt, M, work=work)
        sur.macro_step(w.clone(), dt, tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        mesh.rk_substeps(w, dt, M, work=work)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / reps
    ws = w.clone()
    t0 = time.perf_counter()
    for _ in range(reps):
        sur.macro_step(ws, dt, tol)
    torch.cuda.synchronize()
    t_sur = (time.perf_counter() - t0) / reps
    return t_plain, t_sur


def richardson_problem(mesh, g, k=3, cfl=0.5):
    """Pseudo-time problem v + tau (M^V)^-1 C^V(u) v = g with u := g frozen: tau = cfl h / s,
    ds = 1 / (1 + tau (k+1)^2 s / h), s = max |g| (the step sizes the Richardson tests use)."""
    h = 1.0 / round(np.sqrt(mesh.E / 2))
    s0 = float(mesh.reduce("maxvel", g)[0].item())
    tau = cfl * h / s0
    ds = 1.0 / (1.0 + tau * (k + 1) ** 2 * s0 / h)
    return tau, ds


def warm_start_data(mesh, sur, seeds, per_seed, rtol=1e-10, max_it=4000, device="cuda"):
    """Samples (x, t) for the learned warm start: inputs from g, targets from the converged
    pseudo-time solution v* (remainder beyond g + tau r(g))."""
    import torch
    xs, ts = [], []
    gen = torch.Generator(device=device)
    work = None
    for seed, g_host in zip(seeds, initial_states(mesh, list(seeds))):
        gen.manual_seed(int(seed))
        g = torch.tensor(g_host, device=device)
        if work is None:
            work = torch.empty_like(g)
        tau, ds = richardson_problem(mesh, g)
        v = g.clone()
        mesh.richardson(v, g, g, tau, ds, rtol, max_it, work=work)
        r0 = mesh.apply(g)
        scale = mesh.reduce("maxvel", g)
        elems = torch.randint(0, mesh.E, (per_seed,), generator=gen, device=device,
                              dtype=torch.int32)
        xs.append(sur.features(g, scale, elems))
        ts.append(sur.targets(g, v, r0, scale, tau, elems))
    return torch.cat(xs), torch.cat(ts)


def warm_start_eval(mesh, sur, seeds, rel_tol=1e-6, max_it=4000, device="cuda"):
    """Updates and time to reach a fixed absolute residual (rel_tol times the residual of the
    plain start v0 = g) from three initial guesses: g, g + tau r(g), and the learned one."""
    import torch
    out = {name: {"updates": [], "err": [], "t_ms": []} for name in ("copy", "euler", "learned")}
    work = None
    for g_host in initial_states(mesh, list(seeds)):
        g = torch.tensor(g_host, device=device)
        if work is None:
            work = torch.empty_like(g)
        tau, ds = richardson_problem(mesh, g)
        ref = g.clone()
        mesh.richardson(ref, g, g, tau, ds, 1e-12, max_it, work=work)
        inc = float(torch.linalg.norm(ref - g))
        # the residual of an initial guess is evaluated with the first update
        _, res_copy, _ = mesh.richardson(g.clone(), g, g, tau, ds, 0.0, 1, work=work)
        atol = rel_tol * res_copy
        starts = {"copy": lambda: g.clone(),
                  "euler": lambda: g + tau * mesh.apply(g),
                  "learned": lambda: sur.warm_start(g, g, tau)}
        for name, make in starts.items():
            v = make()
            _, r0, _ = mesh.richardson(v.clone(), g, g, tau, ds, 0.0, 1, work=work)
            out[name]["err"].append(float(torch.linalg.norm(v - ref)) / inc)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            v = make()
            n, _, _ = mesh.richardson(v, g, g, tau, ds, min(1.0, atol / r0), max_it, work=work)
            torch.cuda.synchronize()
            out[name]["t_ms"].append((time.perf_counter() - t0) * 1e3)
            out[name]["updates"].append(n)
    return {name: {key: float(np.median(val)) for key, val in d.items()} for name, d in out.items()}


def warm_start_main(args):
    """Train the network as a warm start of the pseudo-time iteration and compare initial
    guesses (one JSON line)."""
    import torch
    mesh = Mesh.box(2, args.n, 3)
    sur = Surrogate(mesh, M=8)
    sur.load(init_params(0, sur.n_params))
    log = lambda s: print(s, flush=True)
    t0 = time.perf_counter()
    X, T = warm_start_data(mesh, sur, range(1, args.train_seeds + 1), args.per_snapshot)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    log("generated %d samples in %.1f s" % (X.shape[0], t_gen))
    t0 = time.perf_counter()
    hist = train(sur, X, T, args.epochs, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    res = warm_start_eval(mesh, sur, range(10001, 10001 + args.eval_seeds))
    print(json.dumps({"study": "warm_start", "samples": int(X.shape[0]), "t_generate_s": t_gen,
                      "t_train_s": t_train, "loss_first": hist[0][1] if hist else None,
                      "loss_last": hist[-1][1] if hist else None, "median": res}))


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--train-seeds", type=int, default=2000)
    ap.add_argument("--macro", type=int, default=16)
    ap.add_argument("--per-snapshot", type=int, default=128)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--eval-seeds", type=int, default=20)
    ap.add_argument("--tol", type=float, default=None)
    ap.add_argument("--out", default=None, help="save trained parameters (.npy)")
    ap.add_argument("--warm-start", action="store_true",
                    help="train and evaluate the network as an initial guess of the pseudo-time "
                         "iteration instead (--per-snapshot elements per training seed)")
    args = ap.parse_args()
    if args.warm_start:
        warm_start_main(args)
        return
    mesh = Mesh.box(2, args.n, 3)
    sur = Surrogate(mesh, M=8)
    sur.load(init_params(0, sur.n_params))
    log = lambda s: print(s, flush=True)
    t0 = time.perf_counter()
    X, T = generate(mesh, sur, range(1, args.train_seeds + 1), args.macro, args.per_snapshot)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    log("generated %d samples in %.1f s" % (X.shape[0], t_gen))
    t0 = time.perf_counter()
    hist = train(sur, X, T, args.epochs, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    if args.out:
        np.save(args.out, sur.save())
    eval_seeds = range(10001, 10001 + args.eval_seeds)
    probe = evaluate(mesh, sur, eval_seeds, 2, tol=np.inf)
    tol = args.tol if args.tol is not None else 2.0 * float(np.median(probe["rho_plain"]))
    res = evaluate(mesh, sur, eval_seeds, 2, tol=tol)
    h = 1.0 / args.n
    dt = 0.1 * h / 9.0
    t_plain, t_sur = timing(mesh, sur, dt)
    acc = res["accepted"] / max(1, res["macro_steps"])
    out = {"samples": int(X.shape[0]), "t_generate_s": t_gen, "t_train_s": t_train,
           "loss_first": hist[0][1] if hist else None, "loss_last": hist[-1][1] if hist else None,
           "tol": tol, "acceptance": acc,
           "err_state_median": float(np.median(probe["err_state"])),
           "err_increment_median": float(np.median(probe["err_increment"])),
           "err_increment_euler_median": float(np.median(probe["err_increment_euler"])),
           "err_increment_rk3_coarse_median": float(np.median(probe["err_increment_rk3_coarse"])),
           "rho_median": float(np.median(probe["rho"])),
           "rho_plain_median": float(np.median(probe["rho_plain"])),
           "t_plain_macro_ms": t_plain * 1e3, "t_surrogate_macro_ms": t_sur * 1e3,
           "speedup_if_all_accepted": t_plain / t_sur,
           "speedup_at_acceptance": t_plain / (t_sur + (1 - acc) * t_plain)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
