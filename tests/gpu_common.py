"""Shared helpers of the GPU tests: seeded inputs built with the oracle, comparisons."""
import sys

import numpy as np

from oracle import refelem as R
from oracle.dg import Space, cfl_dt
from oracle.mesh import box_mesh
from paper_1508_04245_amd import synth

# configurations of the workloads (dim, N, k) and their fields
C1 = (2, 16, 2)
C2 = (2, 256, 4)
C3 = (3, 32, 3)
C4 = (3, 64, 2)
C5 = (2, 128, 3)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_space(dim, N, k, jitter=0.0, seed=0):
    return Space(box_mesh(dim, N, jitter=jitter, seed=seed), k)


def initial_state(sp, field="tg", seed=0, sd=1e-3, chunk=65536):
    """L2 projection (oracle basis and rule) of the analytic field plus seeded coefficient
    noise, element chunk by element chunk."""
    d, k, m = sp.dim, sp.k, sp.mesh
    n = k + 8 if m.E <= 200000 else k + 3
    p, wq = R.collapsed_rule(d, n)
    phi = R.eval_basis(d, k, p)
    F = synth.FourierField(d, seed=seed) if field != "tg" else None
    out = np.empty(sp.shape)
    for s in range(0, m.E, chunk):
        T = slice(s, min(m.E, s + chunk))
        x = m.X[T, None, 0, :] + np.einsum("tij,qj->tqi", m.J[T], p)
        if F is None:
            f = synth.taylor_green_2d(x) if d == 2 else synth.taylor_green_3d(x)
        else:
            f = F(x)
        out[T] = np.einsum("q,tqi,qm->tim", wq, f, phi) / np.einsum("q,qm,qm->m", wq, phi, phi)
    return out + synth.noise(sp.shape, seed=seed, sd=sd)


# Reduced-precision variants: unit roundoff of their basis contractions (FP32 coefficients,
# tables and sums; two FP16 pieces carry 22 significant bits; three BF16 pieces hold the FP32
# value exactly and the cross products they drop lie below 2^-24)
UNIT = {"fp32": 2.0 ** -24, "mixf32": 2.0 ** -24, "f16x2": 2.0 ** -22, "bf16x3": 2.0 ** -24}


def operator_scales(sp, w, u=None, elems=None, wb=None, ub=None):
    """(r, amp, rate) from the oracle: r = -(M^V)^-1 C_h(u; w, .) on `elems` (all by default),
    amp = (|vol| + sum_F |fac_F|) / |r|, how much larger the volume term and the facet terms of
    C_h (Sec. 2.3) are than their sum, and rate = |r| / |w|; L2 norms with the element
    measures."""
    elems = np.arange(sp.mesh.E) if elems is None else np.asarray(elems)
    vol, facs = sp.form_parts(w, u, elems, wb, ub)
    mass = sp.mass[elems][:, None, :]
    J = sp.mesh.absdetJ[elems]
    l2 = lambda a: float(np.sqrt(np.einsum("t,tim->", J, a * a)))
    fac = np.zeros_like(vol)
    for ff in facs:  # the order of form()
        fac += ff
    r = -(vol + fac) / mass
    terms = l2(vol / mass) + sum(l2(ff / mass) for ff in facs)
    return r, terms / l2(r), l2(r) / l2(w[elems])


def reduced_bars(prec, amp, inc=0.0, n=0, tol=1e-12):
    """(apply bar, bar of the state after n substeps) for a result of precision variant `prec`
    against the FP64 oracle, in relative L2.

    FP64: the parity bar tol.  Reduced precision: every contraction rounds at the unit
    roundoff u of UNIT, so the volume and the facet term of the operator each carry an error
    of about u times their size, and r, their difference, a relative error of about u amp
    (amp from operator_scales).  A substep adds dt r, of relative size inc = dt |r| / |w|, so
    n substeps carry about n u amp inc, plus the rounding of an FP32 state, s = 2^-24.
    Measured on MI355X over the parity cases (2D and 3D, periodic, bounded and one-cell meshes,
    self and frozen mode, full-size workloads): 0.4 to 3.5 u amp after one application,
    whatever the variant and the contraction length (the FP16 pairs at the low end); after
    substeps 0.25 to 1.2 of n u amp inc + s.  The bars are 5 u amp and 3 (n u amp inc + s)."""
    if prec == "fp64":
        return tol, tol
    u = UNIT[prec]
    s = 2.0 ** -24 if prec == "fp32" else 0.0
    return 5 * u * amp, 3 * (n * u * amp * inc + s)


def rel_l2(sp, a, b):
    """||a - b||_L2 / ||b||_L2 with the element measures (a, b coefficient arrays)."""
    J = sp.mesh.absdetJ
    num = np.einsum("t,tim->", J, (a - b) ** 2)
    den = np.einsum("t,tim->", J, b ** 2)
    return float(np.sqrt(num / den))


def rel_l2_rows(absdet, a, b):
    num = np.einsum("t,tim->", absdet, (a - b) ** 2)
    den = np.einsum("t,tim->", absdet, b ** 2)
    return float(np.sqrt(num / den))


def neighbourhood(mesh, elems):
    """elems and their facet neighbours (sorted unique)."""
    return np.unique(np.concatenate([elems, mesh.nbr[elems].ravel()]))


def oracle_rk_on_sample(sp, w0, dt, sample, u=None):
    """One SSP-RK3 substep of the oracle, evaluated only where `sample` depends on it.

    Stage s at a set S needs the previous stage on S and its facet neighbours, so the stages
    are computed on nested patches S1 > S2 > S3 = sample.  Values outside a patch are never
    read.
    """
    m = sp.mesh
    S3 = np.unique(sample)
    S2 = neighbourhood(m, S3)
    S1 = neighbourhood(m, S2)
    w1 = np.zeros_like(w0)
    w1[S1] = w0[S1] + dt * sp.apply(w0, u, elems=S1)
    w2 = np.zeros_like(w0)
    w2[S2] = 0.75 * w0[S2] + 0.25 * (w1[S2] + dt * sp.apply(w1, u, elems=S2))
    return S3, w0[S3] / 3.0 + 2.0 / 3.0 * (w2[S3] + dt * sp.apply(w2, u, elems=S3))
