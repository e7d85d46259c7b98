"""Python binding of libdgconv.so, the MI355X upwind-DG convection library.

Argument marshalling only: every step of the operator and the Runge-Kutta substeps runs in the
library's HIP kernels.  PyTorch provides device memory and streams.  The library must be built
(``python -m paper_1508_04245_amd.build``); without it every call raises.

Names follow include/dgconv.h.  States are torch tensors of shape [n_elem, dim, n_basis],
contiguous, on the current CUDA(HIP) device, float64 (float32 for precision "fp32").
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgconv.so")

PREC = {"fp64": 0, "fp32": 1, "mixf32": 2, "bf16x3": 4, "f16x2": 5}
RED = {"maxvel": 0, "energy": 1, "momentum": 2, "l2diff": 3, "nonfinite": 4}

_lib = None


class DGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("dgconv error %d: %s" % (status, msg))
        self.status = status


class _Info(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("k", ctypes.c_int), ("n_basis", ctypes.c_int),
                ("n_elem", ctypes.c_int64), ("n_facet", ctypes.c_int64),
                ("n_dof", ctypes.c_int64), ("nq_vol", ctypes.c_int), ("nq_facet", ctypes.c_int),
                ("n_types", ctypes.c_int), ("n_tiles", ctypes.c_int),
                ("h_min", ctypes.c_double), ("volume", ctypes.c_double),
                ("n_bfacet", ctypes.c_int64)]


def lib():
    """Load libdgconv.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libdgconv.so is not built; run: python -m paper_1508_04245_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    sig = {
        "dg_mesh_create": [I, I, I64, P, I64, P, P, P],
        "dg_mesh_create_box": [I, I, I, P],
        "dg_mesh_destroy": [P],
        "dg_mesh_get_info": [P, P],
        "dg_mesh_get_vertices": [P, P],
        "dg_mesh_get_neighbors": [P, P, P],
        "dg_project_points": [P, I, P],
        "dg_project": [P, I, P, P],
        "dg_convection_apply": [P, I, P, P, P, P],
        "dg_rk_substeps": [P, I, P, D, I, P, P, P],
        "dg_rk_substeps_extrap": [P, I, P, D, I, D, P, D, P, D, P, P],
        "dg_boundary_points": [P, P],
        "dg_hdiv_info": [P, P, P],
        "dg_hdiv_reference": [I, I, P],
        "dg_transfer_to_dg": [P, P, P, P],
        "dg_transfer_transpose": [P, P, P, P],
        "dg_convection_apply_bc": [P, I, P, P, P, P, P, P],
        "dg_rk_substeps_bc": [P, I, P, D, I, P, P, P, P, P],
        "dg_richardson": [P, I, P, P, P, D, D, D, I, P, P, P, P],
        "dg_reduce": [P, I, P, P, P, P],
        "dg_reduce_noalloc": [P, I, P, P, P, P],
        "dg_eval_basis": [I, I, I64, P, P, P],
        "dg_volume_rule": [I, I, P, P, P],
        "dg_facet_rule": [I, I, P, P, P],
        "dg_surrogate_n_params": [P],
        "dg_surrogate_create": [P, I, P],
        "dg_surrogate_destroy": [P],
        "dg_surrogate_load": [P, P, I64],
        "dg_surrogate_save": [P, P, I64],
        "dg_surrogate_features": [P, P, P, P, I64, P, P],
        "dg_surrogate_targets": [P, P, P, P, P, D, P, I64, P, P],
        "dg_surrogate_forward": [P, P, I64, P, P],
        "dg_surrogate_grad": [P, P, P, I64, P, P, P],
        "dg_surrogate_train_step": [P, P, P, I64, ctypes.c_float, P, P],
        "dg_macro_step": [P, P, P, D, D, P, P, P, P],
        "dg_surrogate_warm_start": [P, P, P, P, D, P, P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = None if name in ("dg_mesh_destroy", "dg_surrogate_destroy") else ctypes.c_int
    L.dg_last_error.restype = ctypes.c_char_p
    L.dg_version.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status):
    if status != 0:
        raise DGError(status, lib().dg_last_error().decode())


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if isinstance(a, np.ndarray) else ctypes.c_void_p(a)


def _dev(t, dtype=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError("expected dtype %s, got %s" % (dtype, t.dtype))
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def eval_basis(dim, k, pts):
    """The library's reference basis and gradients at pts [n, dim] (host)."""
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    n = pts.shape[0]
    npb = {2: (k + 1) * (k + 2) // 2, 3: (k + 1) * (k + 2) * (k + 3) // 6}[dim]
    vals = np.zeros((n, npb))
    grads = np.zeros((n, npb, dim))
    _check(lib().dg_eval_basis(dim, k, n, _ptr(pts), _ptr(vals), _ptr(grads)))
    return vals, grads


def volume_rule(dim, k):
    """The library's volume quadrature rule: points [n, dim] (reference coordinates) and
    weights [n] (host)."""
    n = ctypes.c_int(0)
    _check(lib().dg_volume_rule(dim, k, ctypes.byref(n), None, None))
    pts = np.zeros((n.value, dim))
    wts = np.zeros(n.value)
    _check(lib().dg_volume_rule(dim, k, ctypes.byref(n), _ptr(pts), _ptr(wts)))
    return pts, wts


def facet_rule(dim, k):
    """The library's facet quadrature rule of the operator: points [n, dim - 1] (facet
    parameters) and weights [n] summing to 1 (host)."""
    n = ctypes.c_int(0)
    _check(lib().dg_facet_rule(dim, k, ctypes.byref(n), None, None))
    pts = np.zeros((n.value, dim - 1))
    wts = np.zeros(n.value)
    _check(lib().dg_facet_rule(dim, k, ctypes.byref(n), _ptr(pts), _ptr(wts)))
    return pts, wts


class Mesh:
    """A periodic affine simplicial mesh with degree-k vector DG space (dg_mesh)."""

    def __init__(self, handle):
        self._h = handle
        info = _Info()
        _check(lib().dg_mesh_get_info(self._h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in _Info._fields_}
        self.dim, self.k, self.np = info.dim, info.k, info.n_basis
        self.E = info.n_elem

    @classmethod
    def box(cls, dim, n, k):
        h = ctypes.c_void_p()
        _check(lib().dg_mesh_create_box(dim, n, k, ctypes.byref(h)))
        return cls(h)

    @classmethod
    def from_arrays(cls, dim, k, xyz, elem, period):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        elem = np.ascontiguousarray(elem, dtype=np.int64)
        period = np.ascontiguousarray(period, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(lib().dg_mesh_create(dim, k, xyz.shape[0], _ptr(xyz), elem.shape[0], _ptr(elem),
                                    _ptr(period), ctypes.byref(h)))
        return cls(h)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.dg_mesh_destroy(self._h)
            self._h = None

    @property
    def shape(self):
        return (self.E, self.dim, self.np)

    def vertices(self):
        out = np.zeros((self.E, self.dim + 1, self.dim))
        _check(lib().dg_mesh_get_vertices(self._h, _ptr(out)))
        return out

    def neighbors(self):
        nb = np.zeros((self.E, self.dim + 1), dtype=np.int32)
        nf = np.zeros((self.E, self.dim + 1), dtype=np.int32)
        _check(lib().dg_mesh_get_neighbors(self._h, _ptr(nb), _ptr(nf)))
        return nb, nf

    def project_points(self, n):
        out = np.zeros((self.E, n ** self.dim, self.dim))
        _check(lib().dg_project_points(self._h, n, _ptr(out)))
        return out

    def project(self, vals, n):
        vals = np.ascontiguousarray(vals, dtype=np.float64)
        out = np.zeros(self.shape)
        _check(lib().dg_project(self._h, n, _ptr(vals), _ptr(out)))
        return out

    def boundary_points(self):
        """Physical quadrature points of the boundary facets: [n_bfacet, nq_facet, dim]."""
        nb = self.info["n_bfacet"]
        out = np.zeros((nb, self.info["nq_facet"], self.dim))
        _check(lib().dg_boundary_points(self._h, _ptr(out) if nb else None))
        return out

    def hdiv_size(self):
        """(dim W_h, number of facets) of the H(div) space (2D: 1 <= k <= 6; 3D: 1 <= k <= 4)."""
        n, nf = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(lib().dg_hdiv_info(self._h, ctypes.byref(n), ctypes.byref(nf)))
        return n.value, nf.value

    # ---- device calls
    def to_dg(self, u, out=None, stream=None):
        """I u: DG coefficients of the W_h field with coefficients u (dev [n_dof])."""
        import torch
        if out is None:
            out = torch.empty((self.E, self.dim, self.np), dtype=torch.float64, device=u.device)
        _check(lib().dg_transfer_to_dg(self._h, _dev(u, torch.float64), _dev(out, torch.float64),
                                       _stream(stream)))
        return out

    def transfer_transpose(self, f, out=None, stream=None):
        """I^T f for a functional f given by its values on the DG basis (dev state)."""
        import torch
        if out is None:
            out = torch.empty(self.hdiv_size()[0], dtype=torch.float64, device=f.device)
        _check(lib().dg_transfer_transpose(self._h, _dev(f, torch.float64),
                                           _dev(out, torch.float64), _stream(stream)))
        return out

    def apply(self, w, u=None, out=None, precision="fp64", stream=None):
        """r = -(M^V)^-1 C^V(u) w on the device (u=None: self-convection)."""
        import torch
        dt = torch.float32 if precision == "fp32" else torch.float64
        if out is None:
            out = torch.empty_like(w)
        _check(lib().dg_convection_apply(self._h, PREC[precision], _dev(w, dt),
                                         None if u is None else _dev(u, dt), _dev(out, dt),
                                         _stream(stream)))
        return out

    def apply_bc(self, w, wb, u=None, ub=None, out=None, precision="fp64", stream=None):
        """apply on a mesh with boundary facets; wb, ub: outer values [n_bfacet, nq_facet, d]."""
        import torch
        dt = torch.float32 if precision == "fp32" else torch.float64
        if out is None:
            out = torch.empty_like(w)
        _check(lib().dg_convection_apply_bc(self._h, PREC[precision], _dev(w, dt),
                                            None if u is None else _dev(u, dt), _dev(wb, dt),
                                            None if ub is None else _dev(ub, dt), _dev(out, dt),
                                            _stream(stream)))
        return out

    def rk_substeps_bc(self, w, dt, n, wb, u=None, ub=None, work=None, precision="fp64",
                       stream=None):
        """n SSP-RK3 substeps in place on a mesh with boundary facets (outer values fixed)."""
        import torch
        ty = torch.float32 if precision == "fp32" else torch.float64
        _check(lib().dg_rk_substeps_bc(self._h, PREC[precision], _dev(w, ty), float(dt), int(n),
                                       None if u is None else _dev(u, ty), _dev(wb, ty),
                                       None if ub is None else _dev(ub, ty),
                                       None if work is None else _dev(work, ty),
                                       _stream(stream)))
        return w

    def rk_substeps(self, w, dt, n, u=None, work=None, precision="fp64", stream=None):
        """n SSP-RK3 substeps in place on w."""
        import torch
        ty = torch.float32 if precision == "fp32" else torch.float64
        _check(lib().dg_rk_substeps(self._h, PREC[precision], _dev(w, ty), float(dt), int(n),
                                    None if u is None else _dev(u, ty),
                                    None if work is None else _dev(work, ty), _stream(stream)))
        return w

    def rk_substeps_extrap(self, w, dt, n, t0, ua, ta, ub, tb, work=None, precision="fp64",
                           stream=None):
        """n SSP-RK3 substeps in place on w with u(s) = ua + (s-ta)/(tb-ta) (ub-ua)."""
        import torch
        ty = torch.float32 if precision == "fp32" else torch.float64
        _check(lib().dg_rk_substeps_extrap(self._h, PREC[precision], _dev(w, ty), float(dt),
                                           int(n), float(t0), _dev(ua, ty), float(ta),
                                           _dev(ub, ty), float(tb),
                                           None if work is None else _dev(work, ty),
                                           _stream(stream)))
        return w

    def richardson(self, v, g, u, tau, ds, rtol, max_it, work=None, precision="fp64",
                   stream=None):
        """Pseudo-time iteration for v + tau (M^V)^-1 C^V(u) v = g in place on v (the initial
        guess); returns (number of updates, ||res_0||, last residual norm)."""
        import torch
        it = ctypes.c_int(0)
        res = (ctypes.c_double * 2)()
        _check(lib().dg_richardson(self._h, PREC[precision], _dev(v, torch.float64),
                                   _dev(g, torch.float64), _dev(u, torch.float64), float(tau),
                                   float(ds), float(rtol), int(max_it),
                                   None if work is None else _dev(work, torch.float64),
                                   _stream(stream), ctypes.byref(it), res))
        return it.value, res[0], res[1]

    def reduce(self, what, a, b=None, out=None, stream=None):
        import torch
        if out is None:
            out = torch.zeros(4, dtype=torch.float64, device=a.device)
        _check(lib().dg_reduce(self._h, RED[what], _dev(a, torch.float64),
                               None if b is None else _dev(b, torch.float64),
                               _dev(out, torch.float64), _stream(stream)))
        return out

    def reduce_noalloc(self, what, a, b, out, stream=None):
        """dg_reduce_noalloc: out (a caller tensor, >= dim doubles) is required."""
        import torch
        _check(lib().dg_reduce_noalloc(self._h, RED[what], _dev(a, torch.float64),
                                       None if b is None else _dev(b, torch.float64),
                                       _dev(out, torch.float64), _stream(stream)))
        return out


class Surrogate:
    """The learned macro-step network of a 2D P3 mesh (dg_surrogate)."""

    def __init__(self, mesh, M=8):
        self.mesh = mesh
        self.M = M
        h = ctypes.c_void_p()
        _check(lib().dg_surrogate_create(mesh._h, M, ctypes.byref(h)))
        self._h = h
        n = ctypes.c_int64()
        _check(lib().dg_surrogate_n_params(ctypes.byref(n)))
        self.n_params = n.value

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.dg_surrogate_destroy(self._h)
            self._h = None

    def load(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(lib().dg_surrogate_load(self._h, _ptr(p), p.size))

    def save(self):
        p = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().dg_surrogate_save(self._h, _ptr(p), p.size))
        return p

    def features(self, w, scale, elems=None, out=None, stream=None):
        import torch
        n = self.mesh.E if elems is None else elems.numel()
        if out is None:
            out = torch.empty((n, 80), dtype=torch.float32, device=w.device)
        _check(lib().dg_surrogate_features(self._h, _dev(w, torch.float64), _dev(scale, torch.float64),
                                           None if elems is None else _dev(elems, torch.int32), n,
                                           _dev(out, torch.float32), _stream(stream)))
        return out

    def targets(self, w0, w1, r0, scale, tau, elems=None, out=None, stream=None):
        import torch
        n = self.mesh.E if elems is None else elems.numel()
        if out is None:
            out = torch.empty((n, 20), dtype=torch.float32, device=w0.device)
        _check(lib().dg_surrogate_targets(self._h, _dev(w0, torch.float64), _dev(w1, torch.float64),
                                          _dev(r0, torch.float64), _dev(scale, torch.float64),
                                          float(tau),
                                          None if elems is None else _dev(elems, torch.int32), n,
                                          _dev(out, torch.float32), _stream(stream)))
        return out

    def forward(self, x, stream=None):
        import torch
        y = torch.empty((x.shape[0], 20), dtype=torch.float32, device=x.device)
        _check(lib().dg_surrogate_forward(self._h, _dev(x, torch.float32), x.shape[0],
                                          _dev(y, torch.float32), _stream(stream)))
        return y

    def grad(self, x, t, stream=None):
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        loss = torch.zeros(1, dtype=torch.float32, device=x.device)
        _check(lib().dg_surrogate_grad(self._h, _dev(x, torch.float32), _dev(t, torch.float32),
                                       x.shape[0], _dev(g, torch.float32), _dev(loss, torch.float32),
                                       _stream(stream)))
        return loss, g

    def train_step(self, x, t, lr, loss=None, stream=None):
        _check(lib().dg_surrogate_train_step(self._h, _dev(x), _dev(t), x.shape[0], float(lr),
                                             None if loss is None else _dev(loss), _stream(stream)))
        return loss

    def macro_step(self, w, dt, tol, work=None, stream=None):
        """One macro-step in place on w; returns (accepted, rho).  work: None (the surrogate's
        buffer) or a dev FP64 tensor of at least 3 states."""
        import torch
        acc = ctypes.c_int()
        rho = ctypes.c_double()
        _check(lib().dg_macro_step(self.mesh._h, self._h, _dev(w, torch.float64), float(dt),
                                   float(tol), None if work is None else _dev(work, torch.float64),
                                   ctypes.byref(acc), ctypes.byref(rho), _stream(stream)))
        return bool(acc.value), rho.value

    def warm_start(self, g, u, tau, out=None, stream=None):
        """Learned initial guess of the pseudo-time problem v + tau (M^V)^-1 C^V(u) v = g
        (u None: u := g); returns out (allocated like g when None)."""
        import torch
        if out is None:
            out = torch.empty_like(g)
        _check(lib().dg_surrogate_warm_start(self.mesh._h, self._h, _dev(g, torch.float64),
                                             None if u is None else _dev(u, torch.float64),
                                             float(tau), _dev(out, torch.float64),
                                             _stream(stream)))
        return out
