"""Seeded synthetic inputs: analytic velocity fields at given points, and coefficient noise.

This module holds none of the discretisation's arithmetic (no basis, no quadrature, no
operator).  It is the only module shared by the GPU path's drivers and the tests' oracle:
each side projects the same analytic field with its own quadrature and adds the same seeded
noise array.

Fields (all periodic on the unit box):
  * 2D Taylor-Green: (sin 2pi x cos 2pi y, -cos 2pi x sin 2pi y).
  * 3D Taylor-Green: (sin X cos Y cos Z, -cos X sin Y cos Z, 0) with X = 2pi x (the vortex on
    [0, 2pi]^3 rescaled to the unit cube).
  * Random Fourier field: 16 distinct wave vectors kappa in Z^d, 0 < |kappa| <= 4 (one of each
    +-pair), complex amplitudes with iid N(0,1) parts, Leray projection a <- a - (a.k)k/|k|^2
    (divergence-free), amplitude scaled by |kappa|^-2, u = Re sum a e^{2 pi i kappa.x}, RMS
    normalised to 1 analytically (distinct, non-opposite modes are L2-orthogonal).
  * Shear wave (exact solution of w_t + div(w (x) w) = 0, div w = 0):
    w(x,t) = c + A sin(2 pi (xi.x - (xi.c) t)) eta, eta . xi = 0.
"""
import numpy as np

TWO_PI = 2.0 * np.pi


def taylor_green_2d(x):
    X, Y = TWO_PI * x[..., 0], TWO_PI * x[..., 1]
    return np.stack([np.sin(X) * np.cos(Y), -np.cos(X) * np.sin(Y)], axis=-1)


def taylor_green_3d(x):
    X, Y, Z = TWO_PI * x[..., 0], TWO_PI * x[..., 1], TWO_PI * x[..., 2]
    return np.stack([np.sin(X) * np.cos(Y) * np.cos(Z), -np.cos(X) * np.sin(Y) * np.cos(Z),
                     np.zeros_like(X)], axis=-1)


class FourierField:
    """Random divergence-free Fourier field; see the module docstring."""

    def __init__(self, dim, seed, n_modes=16, kmax=4):
        rng = np.random.default_rng(seed)
        rng_k = range(-kmax, kmax + 1)
        if dim == 2:
            cand = [(a, b) for a in rng_k for b in rng_k]
        else:
            cand = [(a, b, c) for a in rng_k for b in rng_k for c in rng_k]
        # one representative of each +-pair: first nonzero component positive
        cand = [v for v in cand if 0 < sum(t * t for t in v) <= kmax * kmax
                and next(t for t in v if t != 0) > 0]
        cand = np.array(cand, dtype=np.float64)
        pick = rng.choice(len(cand), size=n_modes, replace=False)
        self.kappa = cand[pick]
        a = rng.normal(size=(n_modes, dim)) + 1j * rng.normal(size=(n_modes, dim))
        kn = self.kappa / np.linalg.norm(self.kappa, axis=1)[:, None]
        a = a - np.sum(a * kn, axis=1)[:, None] * kn  # Leray projection
        a = a / np.sum(self.kappa ** 2, axis=1)[:, None]  # |kappa|^-2
        rms = np.sqrt(0.5 * np.sum(np.abs(a) ** 2))
        self.amp = a / rms

    def __call__(self, x):
        # Re sum_m a_m e^{i ph_m} = cos(ph) Re(a) - sin(ph) Im(a)
        ph = TWO_PI * (x @ self.kappa.T)
        return np.cos(ph) @ self.amp.real - np.sin(ph) @ self.amp.imag


def shear_wave(x, t, c, xi, eta, A=1.0):
    """Exact solution w = c + A sin(2pi(xi.x - (xi.c)t)) eta (xi integer, eta . xi = 0)."""
    c, xi, eta = (np.asarray(v, dtype=np.float64) for v in (c, xi, eta))
    ph = TWO_PI * (x @ xi - np.dot(xi, c) * t)
    return c + A * np.sin(ph)[..., None] * eta


def noise(shape, seed=0, sd=1e-3):
    """Seeded Gaussian noise on the coefficients."""
    return np.random.default_rng(seed).normal(0.0, sd, size=shape)
