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
import os

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

    def _eval(self, x):
        # Re sum_m a_m e^{i ph_m} = cos(ph_m) Re(a_m) - sin(ph_m) Im(a_m), summed mode by mode
        # with elementwise operations only (no BLAS call, so host threads may run it at once)
        n, dim = x.shape
        out = np.zeros((n, self.amp.shape[1]))
        for m in range(self.kappa.shape[0]):
            ph = x[:, 0] * self.kappa[m, 0]
            for a in range(1, dim):
                ph = ph + x[:, a] * self.kappa[m, a]
            ph = TWO_PI * ph
            c, s = np.cos(ph)[:, None], np.sin(ph)[:, None]
            out += c * self.amp[m].real - s * self.amp[m].imag
        return out

    def __call__(self, x, chunk=1 << 18):
        """The field at the points x [..., dim]; large inputs in chunks of points on host
        threads (NumPy's elementwise loops release the GIL), each point evaluated alone."""
        x = np.asarray(x, dtype=np.float64)
        flat = x.reshape(-1, x.shape[-1])
        n, dim = flat.shape[0], self.amp.shape[1]
        if n <= chunk:
            return self._eval(flat).reshape(x.shape[:-1] + (dim,))
        from concurrent.futures import ThreadPoolExecutor
        out = np.empty((n, dim))

        def run(s):
            out[s:s + chunk] = self._eval(flat[s:s + chunk])

        with ThreadPoolExecutor(max(1, min(16, len(os.sched_getaffinity(0))))) as ex:
            list(ex.map(run, range(0, n, chunk)))
        return out.reshape(x.shape[:-1] + (dim,))


def shear_wave(x, t, c, xi, eta, A=1.0):
    """Exact solution w = c + A sin(2pi(xi.x - (xi.c)t)) eta (xi integer, eta . xi = 0)."""
    c, xi, eta = (np.asarray(v, dtype=np.float64) for v in (c, xi, eta))
    ph = TWO_PI * (x @ xi - np.dot(xi, c) * t)
    return c + A * np.sin(ph)[..., None] * eta


def noise(shape, seed=0, sd=1e-3):
    """Seeded Gaussian noise on the coefficients."""
    return np.random.default_rng(seed).normal(0.0, sd, size=shape)


def box_elements(dim, N, jitter=0.0, seed=0, shuffle=False):
    """Per-element vertex coordinates [E, dim+1, dim] of the periodic unit box cut into N^dim
    cells, 2 triangles (lower (v00, v10, v11), upper (v11, v01, v00)) or 6 Kuhn tetrahedra
    (v000, v000+e_s0, v000+e_s0+e_s1, v111) per cell, cells in x-fastest order.  `jitter` > 0
    moves every lattice vertex by a seeded periodic offset of that size times 1/N (copies of
    a vertex move together); `shuffle` permutes each element's vertex order at random (seeded),
    the same mesh with arbitrary element frames.  Input geometry only."""
    import itertools
    rng = np.random.default_rng(seed)
    h = 1.0 / N
    off = rng.uniform(-1, 1, size=(N,) * dim + (dim,)) * jitter * h if jitter else None
    if dim == 2:
        j, i = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
        b = np.stack([i.ravel(), j.ravel()], axis=1)
        lat = np.stack([np.stack([b, b + [1, 0], b + [1, 1]], 1),
                        np.stack([b + [1, 1], b + [0, 1], b], 1)], axis=1).reshape(-1, 3, 2)
    else:
        l, j, i = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
        b = np.stack([i.ravel(), j.ravel(), l.ravel()], axis=1)
        eye = np.eye(3, dtype=np.int64)
        lat = np.stack([np.stack([b, b + eye[s[0]], b + eye[s[0]] + eye[s[1]], b + 1], 1)
                        for s in itertools.permutations(range(3))], axis=1).reshape(-1, 4, 3)
    X = lat * h
    if off is not None:
        w = np.mod(lat, N)
        X = X + off[tuple(w[..., a] for a in range(dim))]
    if shuffle:
        perm = np.argsort(rng.random((X.shape[0], dim + 1)), axis=1)
        X = np.take_along_axis(X, perm[:, :, None], axis=1)
    return X
