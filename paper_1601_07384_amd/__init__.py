"""MI355X (gfx950) staggered space-time DG pressure library: Python binding.

The computation lives in the HIP library ``libstdg.so`` behind the C ABI of
``include/stdg.h``.  This module only marshals arguments: meshes are host
numpy arrays, vectors are torch tensors on the GPU (torch provides device
memory and streams).
"""

import ctypes

import numpy as np

from . import _lib
from ._lib import (Config, MeshInfo, SolveOpts, SolveReport, StepOpts, StepReport, StdgError,
                   ModelConfig, TrainReport,
                   STDG_OK, STDG_NOT_CONVERGED, STDG_FP64, STDG_FP32,
                   STDG_AUTO, STDG_CG, STDG_GMRES, STDG_CG_TIME, STDG_GUESS_ZERO,
                   STDG_GUESS_PREVIOUS, STDG_KRYLOV_ZERO, STDG_KRYLOV_PREVIOUS,
                   STDG_KRYLOV_EXTRAPOLATE, STDG_KRYLOV_LEARNED, STDG_LOSS_MSE, STDG_LOSS_RESIDUAL,
                   STDG_PRECOND_NONE, STDG_PRECOND_BLOCK_JACOBI, STDG_BICGSTAB,
                   STDG_LAYOUT_ELEMENT, STDG_LAYOUT_RUN)

__all__ = ["Mesh", "Model", "StdgError", "STDG_FP64", "STDG_FP32", "STDG_AUTO",
           "STDG_CG", "STDG_GMRES", "STDG_CG_TIME", "STDG_GUESS_ZERO", "STDG_GUESS_PREVIOUS",
           "STDG_KRYLOV_ZERO", "STDG_KRYLOV_PREVIOUS", "STDG_KRYLOV_EXTRAPOLATE",
           "STDG_KRYLOV_LEARNED", "STDG_LOSS_MSE", "STDG_LOSS_RESIDUAL", "STDG_PRECOND_NONE",
           "STDG_PRECOND_BLOCK_JACOBI", "STDG_BICGSTAB", "STDG_LAYOUT_ELEMENT", "STDG_LAYOUT_RUN",
           "solve_opts", "step_opts"]


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(getattr(stream, "cuda_stream", stream))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def solve_opts(**kw):
    o = SolveOpts()
    _lib.load().stdg_solve_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown solve option {k}")
        setattr(o, k, v)
    return o


def step_opts(n_picard=0, pressure_guess=0, pressure=None, viscous=None, krylov_guess=0,
              model=None, hist=None, rec_b=None, rec_x=None, theta=1.0):
    """Step options; tensors given here must stay alive until the step returns."""
    o = StepOpts()
    _lib.load().stdg_step_opts_default(ctypes.byref(o))
    o.n_picard = n_picard
    o.pressure_guess = pressure_guess
    for name, kw in (("pressure", pressure), ("viscous", viscous)):
        for k, v in (kw or {}).items():
            if not hasattr(getattr(o, name), k):
                raise TypeError(f"unknown {name} option {k}")
            setattr(getattr(o, name), k, v)
    o.krylov_guess = krylov_guess
    o.theta = theta
    o.model = model._h.value if model is not None else None
    for name, t in (("hist", hist), ("rec_b", rec_b), ("rec_x", rec_x)):
        setattr(o, name, t.data_ptr() if t is not None else None)
    o._keep = (model, hist, rec_b, rec_x)
    return o


class Mesh:
    """A built mesh handle (owns the library's device tables)."""

    def __init__(self, X, tets, p, p_gamma=0, dt=1e-2, nu=0.0, periodic=False,
                 box_lo=(0.0, 0.0, 0.0), box_hi=(1.0, 1.0, 1.0), anchor_tet=0,
                 anchor_node=0, reorder=True, device=True, nodes=None):
        """nodes: optional (E, N, 3) positions of each element's spatial nodes
        (curved isoparametric elements; only the pressure system is built)."""
        lib = _lib.load()
        X = np.ascontiguousarray(X, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int64)
        cfg = Config()
        cfg.p, cfg.p_gamma, cfg.nu, cfg.dt = p, p_gamma, nu, dt
        cfg.periodic = 1 if periodic else 0
        cfg.box_lo[:] = list(box_lo)
        cfg.box_hi[:] = list(box_hi)
        cfg.anchor_tet, cfg.anchor_node = anchor_tet, anchor_node
        cfg.reorder = 1 if reorder else 0
        h = ctypes.c_void_p()
        if nodes is not None:
            nodes = np.ascontiguousarray(nodes, dtype=np.float64)
            N = (p + 1) * (p + 2) * (p + 3) // 6
            if nodes.shape != (tets.shape[0], N, 3):
                raise ValueError(f"nodes must have shape ({tets.shape[0]}, {N}, 3)")
            _lib.check(lib.stdg_mesh_build_curved(X.ctypes.data, X.shape[0], tets.ctypes.data, tets.shape[0],
                                                  nodes.ctypes.data, 0 if device else 1,
                                                  ctypes.byref(cfg), ctypes.byref(h)))
        else:
            fn = lib.stdg_mesh_build if device else lib.stdg_mesh_build_host
            _lib.check(fn(X.ctypes.data, X.shape[0], tets.ctypes.data, tets.shape[0],
                          ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._lib = lib
        self.device = device
        info = MeshInfo()
        _lib.check(lib.stdg_mesh_info_get(h, ctypes.byref(info)))
        self.E, self.N, self.G, self.Nst = info.n_tet, info.N, info.G, info.Nst
        self.n_face, self.n_interior_face = info.n_face, info.n_interior_face
        self.n_classes = info.n_classes
        self.anchor_internal = info.anchor_internal
        self.inner_layout, self.inner_len = info.inner_layout, info.inner_len
        self.inner_per_element = bool(info.inner_per_element)
        self.p, self.p_gamma, self.dt, self.nu = p, p_gamma, dt, nu

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.stdg_mesh_free(h)
            self._h = None

    # -------------------------------------------------------------- layout
    def permutation(self):
        perm = np.empty(self.E, dtype=np.int64)
        _lib.check(self._lib.stdg_mesh_permutation(self._h, perm.ctypes.data))
        return perm

    def faces(self):
        n = self.n_face
        left = np.empty(n, np.int64); right = np.empty(n, np.int64)
        lf = np.empty(n, np.int32); rf = np.empty(n, np.int32)
        _lib.check(self._lib.stdg_mesh_faces(self._h, left.ctypes.data, lf.ctypes.data,
                                             right.ctypes.data, rf.ctypes.data))
        return left, lf, right, rf

    def blocks(self):
        """(blocks [n_classes,5,N,N], cls [E], nbr [E,4], C [G,G]) host copies."""
        B = np.empty((self.n_classes, 5, self.N, self.N))
        cls = np.empty(self.E, np.int32)
        nbr = np.empty((self.E, 4), np.int32)
        C = np.empty((self.G, self.G))
        _lib.check(self._lib.stdg_mesh_blocks(self._h, B.ctypes.data, cls.ctypes.data,
                                              nbr.ctypes.data, C.ctypes.data))
        return B, cls, nbr, C

    # -------------------------------------------------------------- operator
    def apply(self, x, y, precision=STDG_FP64, stream=None):
        """y = S x on device float64 tensors [E*G*N] (internal element order)."""
        self._check_vec(x, "float64"); self._check_vec(y, "float64")
        _lib.check(self._lib.stdg_pressure_apply(self._h, precision, _ptr(x), _ptr(y),
                                                 _stream_ptr(stream)))

    def apply_f32(self, x, y, stream=None):
        self._check_vec(x, "float32"); self._check_vec(y, "float32")
        _lib.check(self._lib.stdg_pressure_apply_f32(self._h, _ptr(x), _ptr(y),
                                                     _stream_ptr(stream)))

    def apply_spatial_f32(self, x, y, stream=None):
        """y = (B (x) I) x: the spatial operator on every time node, FP32,
        vectors in the inner layout (inner_len entries)."""
        self._check_vec(x, "float32", self.inner_len); self._check_vec(y, "float32", self.inner_len)
        _lib.check(self._lib.stdg_pressure_apply_spatial_f32(self._h, _ptr(x), _ptr(y),
                                                             _stream_ptr(stream)))

    def inner_from_f64(self, x, y, scale=1.0, stream=None):
        """y (FP32, inner layout) = scale x (FP64, [E][G][N])."""
        self._check_vec(x, "float64"); self._check_vec(y, "float32", self.inner_len)
        _lib.check(self._lib.stdg_inner_from_f64(self._h, _ptr(x), float(scale), _ptr(y),
                                                 _stream_ptr(stream)))

    def inner_to_f64(self, y, x, scale=1.0, stream=None):
        """x (FP64, [E][G][N]) = scale y (FP32, inner layout)."""
        self._check_vec(y, "float32", self.inner_len); self._check_vec(x, "float64")
        _lib.check(self._lib.stdg_inner_to_f64(self._h, _ptr(y), float(scale), _ptr(x),
                                               _stream_ptr(stream)))

    def solve(self, b, x, opts=None, stream=None, **kw):
        """Anchored pressure solve; x holds the guess on entry.  Returns the report."""
        self._check_vec(b, "float64"); self._check_vec(x, "float64")
        o = opts if opts is not None else solve_opts(**kw)
        rep = SolveReport()
        code = self._lib.stdg_pressure_solve(self._h, _ptr(b), _ptr(x), ctypes.byref(o),
                                             ctypes.byref(rep), _stream_ptr(stream))
        _lib.check(code, allow=(STDG_OK, STDG_NOT_CONVERGED))
        return rep

    def solve_noalloc(self, b, x, opts=None, stream=None, **kw):
        """The same solve (FP64, STDG_CG or STDG_CG_TIME) on the library's
        fixed device scratch array: no device allocation.  Returns the report."""
        self._check_vec(b, "float64"); self._check_vec(x, "float64")
        o = opts if opts is not None else solve_opts(**kw)
        rep = SolveReport()
        code = self._lib.stdg_pressure_solve_noalloc(self._h, _ptr(b), _ptr(x), ctypes.byref(o),
                                                     ctypes.byref(rep), _stream_ptr(stream))
        _lib.check(code, allow=(STDG_OK, STDG_NOT_CONVERGED))
        return rep

    # -------------------------------------------------------------- Picard
    def picard_step(self, vhat, vbar, p, g_nodal=None, opts=None, stream=None, **kw):
        """One time step (in place on vhat [3,F,G,N], vbar [3,E,G,N], p [E,G,N])."""
        for t, n in ((vhat, 3 * self.n_face * self.Nst), (vbar, 3 * self.E * self.Nst),
                     (p, self.E * self.Nst)):
            self._check_any(t, n)
        if g_nodal is not None:
            self._check_any(g_nodal, 3 * self.E * self.Nst)
        o = opts if opts is not None else step_opts(**kw)
        keep = getattr(o, "_keep", (None, None, None, None))
        n_pic = o.n_picard if o.n_picard > 0 else self.G
        for t, n in zip(keep[1:], (2 * n_pic, 1, 1)):
            if t is not None:
                self._check_any(t, n * self.E * self.Nst)
        rep = StepReport()
        g = _ptr(g_nodal) if g_nodal is not None else None
        code = self._lib.stdg_picard_step(self._h, _ptr(vhat), _ptr(vbar), _ptr(p), g,
                                          ctypes.byref(o), ctypes.byref(rep), _stream_ptr(stream))
        _lib.check(code, allow=(STDG_OK, STDG_NOT_CONVERGED))
        return rep

    def dual_from_main(self, vbar, vhat, stream=None):
        self._check_any(vbar, 3 * self.E * self.Nst)
        self._check_any(vhat, 3 * self.n_face * self.Nst)
        _lib.check(self._lib.stdg_dual_from_main(self._h, _ptr(vbar), _ptr(vhat), _stream_ptr(stream)))

    def main_from_dual(self, vhat, vbar, stream=None):
        self._check_any(vbar, 3 * self.E * self.Nst)
        self._check_any(vhat, 3 * self.n_face * self.Nst)
        _lib.check(self._lib.stdg_main_from_dual(self._h, _ptr(vhat), _ptr(vbar), _stream_ptr(stream)))

    def divergence(self, vhat, div, stream=None):
        self._check_any(vhat, 3 * self.n_face * self.Nst)
        self._check_any(div, self.E * self.Nst)
        _lib.check(self._lib.stdg_divergence(self._h, _ptr(vhat), _ptr(div), _stream_ptr(stream)))

    def _check_any_len(self, t):
        if not t.is_cuda or str(t.dtype) != "torch.float64" or not t.is_contiguous():
            raise ValueError("expected a contiguous CUDA float64 tensor")

    def _check_any(self, t, n):
        if not t.is_cuda or str(t.dtype) != "torch.float64" or not t.is_contiguous():
            raise ValueError("expected a contiguous CUDA float64 tensor")
        if t.numel() != n:
            raise ValueError(f"expected {n} entries, got {t.numel()}")

    def _check_vec(self, t, dtype, n=None):
        if not t.is_cuda or str(t.dtype) != "torch." + dtype or not t.is_contiguous():
            raise ValueError(f"expected a contiguous CUDA {dtype} tensor")
        n = self.E * self.Nst if n is None else n
        if t.numel() != n:
            raise ValueError(f"expected {n} entries, got {t.numel()}")


class Model:
    """Learned Krylov initial guess (MLP) for meshes shaped like `mesh`.

    Tensors are contiguous CUDA float64 in the library's element order:
    pressures and right-hand sides [E*G*N] (or [steps*E*G*N] for training),
    feature rows [n, n_in], outputs [n, n_out].
    """

    def __init__(self, mesh, hidden=128, precision=STDG_FP32, batch=16384, seed=1601, lr=1e-3,
                 beta1=0.9, beta2=0.999, eps=1e-8, init_scale_out=0.0, loss=STDG_LOSS_RESIDUAL):
        lib = _lib.load()
        cfg = ModelConfig()
        lib.stdg_model_config_default(ctypes.byref(cfg))
        cfg.hidden, cfg.precision, cfg.batch, cfg.seed = hidden, precision, batch, seed
        cfg.lr, cfg.beta1, cfg.beta2, cfg.eps = lr, beta1, beta2, eps
        cfg.init_scale_out = init_scale_out
        cfg.loss = loss
        h = ctypes.c_void_p()
        _lib.check(lib.stdg_model_create(mesh._h, ctypes.byref(cfg), ctypes.byref(h)))
        self._h, self._lib, self.mesh = h, lib, mesh
        npar, nin, nout = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _lib.check(lib.stdg_model_info(h, ctypes.byref(npar), ctypes.byref(nin), ctypes.byref(nout)))
        self.n_params, self.n_in, self.n_out = npar.value, nin.value, nout.value
        self.hidden, self.batch = hidden, batch

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.stdg_model_free(h)
            self._h = None

    def params(self):
        out = np.empty(self.n_params)
        _lib.check(self._lib.stdg_model_get_params(self._h, out.ctypes.data))
        return out

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float64)
        if theta.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        _lib.check(self._lib.stdg_model_set_params(self._h, theta.ctypes.data))

    def grads(self):
        out = np.empty(self.n_params)
        _lib.check(self._lib.stdg_model_get_grads(self._h, out.ctypes.data))
        return out

    def _rows(self, t, width):
        self.mesh._check_any_len(t)
        if t.numel() % width:
            raise ValueError(f"expected rows of {width} values")
        return t.numel() // width

    def features(self, P, Pm, B, F, stream=None):
        for t in (P, Pm, B):
            self.mesh._check_any(t, self.mesh.E * self.mesh.Nst)
        self.mesh._check_any(F, self.mesh.E * self.n_in)
        _lib.check(self._lib.stdg_model_features(self._h, self.mesh._h, _ptr(P), _ptr(Pm), _ptr(B),
                                                 _ptr(F), _stream_ptr(stream)))

    def forward(self, F, Y, stream=None):
        n = self._rows(F, self.n_in)
        self.mesh._check_any(Y, n * self.n_out)
        _lib.check(self._lib.stdg_model_forward(self._h, _ptr(F), n, _ptr(Y), _stream_ptr(stream)))

    def loss_grad(self, F, T, stream=None):
        n = self._rows(F, self.n_in)
        self.mesh._check_any(T, n * self.n_out)
        loss = ctypes.c_double()
        _lib.check(self._lib.stdg_model_loss_grad(self._h, _ptr(F), _ptr(T), n, ctypes.byref(loss),
                                                  _stream_ptr(stream)))
        return loss.value

    def residual_loss_grad(self, P, Pm, B, X, stream=None):
        for t in (P, Pm, B, X):
            self.mesh._check_any(t, self.mesh.E * self.mesh.Nst)
        loss = ctypes.c_double()
        _lib.check(self._lib.stdg_model_residual_loss_grad(self._h, self.mesh._h, _ptr(P), _ptr(Pm), _ptr(B),
                                                           _ptr(X), ctypes.byref(loss), _stream_ptr(stream)))
        return loss.value

    def adam_step(self, stream=None):
        _lib.check(self._lib.stdg_model_adam_step(self._h, _stream_ptr(stream)))

    def train(self, P, Pm, B, X, epochs=1, stream=None):
        per = self.mesh.E * self.mesh.Nst
        steps = self._rows(P, per)
        for t in (Pm, B, X):
            self.mesh._check_any(t, steps * per)
        rep = TrainReport()
        _lib.check(self._lib.stdg_model_train(self._h, self.mesh._h, steps, _ptr(P), _ptr(Pm), _ptr(B),
                                              _ptr(X), epochs, ctypes.byref(rep), _stream_ptr(stream)))
        return rep

    def predict(self, P, Pm, B, x0, stream=None):
        for t in (P, Pm, B, x0):
            self.mesh._check_any(t, self.mesh.E * self.mesh.Nst)
        _lib.check(self._lib.stdg_model_predict(self._h, self.mesh._h, _ptr(P), _ptr(Pm), _ptr(B),
                                                _ptr(x0), _stream_ptr(stream)))
