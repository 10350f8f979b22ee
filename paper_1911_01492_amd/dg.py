"""Python binding of libdg (argument marshalling only).

Every step of the operator application and of the solvers runs in the HIP
kernels of ``libdg.so``; this module only passes torch device pointers and the
current HIP stream through the C ABI of ``include/dg.h``.  There is no CPU
fallback: without the built library every call raises.

``DGSolve`` wraps ``dg_cg_solve`` in a ``torch.autograd.Function``: the
backward pass solves the adjoint system A^T lambda = dL/du with the same CG
and returns dL/dtheta_T = -lambda^T (dA/dtheta_T) u (``dg_dA_dtheta``) and
dL/db = lambda.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdg.so")

DG_OK, DG_NOT_CONVERGED, DG_BREAKDOWN = 0, 1, 2
DG_ERR_ARG, DG_ERR_UNSUPPORTED, DG_ERR_DEVICE = -1, -2, -3
PREC = {"f64": 0, "f32": 1, "bf16": 2, "bf16_mfma": 3}
BC = {"dirichlet": 0, "periodic": 1}
PRECOND = {"none": 0, "jacobi": 1, "block_jacobi": 2}
_IN_DTYPE = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "bf16_mfma": torch.bfloat16}
_OUT_DTYPE = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.float32, "bf16_mfma": torch.float32}

#: every function declared in include/dg.h
ABI_FUNCTIONS = ["dg_query_workspace", "dg_setup", "dg_set_theta", "dg_set_reaction", "dg_apply", "dg_apply_transpose", "dg_apply_multi",
                 "dg_dA_dtheta", "dg_dA_dtheta_noalloc", "dg_diagonal", "dg_quadrature_points", "dg_load_vector", "dg_cg_solve",
                 "dg_num_dofs", "dg_num_elements", "dg_nodes_per_dir", "dg_apply_kernel", "dg_destroy",
                 "dg_last_error"]


class DGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libdg error {code}: {msg}")
        self.code = code


class MeshDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("degree", ctypes.c_int32), ("bc", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("penalty_hat", ctypes.c_double), ("vertices", ctypes.c_void_p),
                ("theta", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t)]


DC_MODE = {"restart": 0, "keep": 1}
CG_VARIANT = {"standard": 0, "single_reduction": 1}


class CgOpts(ctypes.Structure):
    _fields_ = [("prec_inner", ctypes.c_int), ("precond", ctypes.c_int), ("transpose", ctypes.c_int),
                ("rtol", ctypes.c_double), ("inner_rtol", ctypes.c_double), ("maxit", ctypes.c_int),
                ("max_outer", ctypes.c_int), ("check_every", ctypes.c_int), ("dc_mode", ctypes.c_int),
                ("cg_variant", ctypes.c_int)]


class CgInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("outer_iters", ctypes.c_int),
                ("restarts", ctypes.c_int), ("rel_true_residual", ctypes.c_double),
                ("seconds", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libdg.so from the package directory (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1911_01492_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, P = ctypes.c_void_p, ctypes.POINTER
    L.dg_query_workspace.argtypes = [P(MeshDesc), P(ctypes.c_size_t)]
    L.dg_setup.argtypes = [P(MeshDesc), P(vp), vp]
    L.dg_set_theta.argtypes = [vp, vp, vp]
    L.dg_set_reaction.argtypes = [vp, vp, vp]
    L.dg_apply.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    L.dg_apply_transpose.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    L.dg_apply_multi.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp]
    L.dg_dA_dtheta.argtypes = [vp, vp, vp, vp, vp]
    L.dg_dA_dtheta_noalloc.argtypes = [vp, vp, vp, vp, vp]
    L.dg_diagonal.argtypes = [vp, vp, vp]
    L.dg_quadrature_points.argtypes = [vp, vp, vp]
    L.dg_load_vector.argtypes = [vp, vp, vp, vp]
    L.dg_cg_solve.argtypes = [vp, P(CgOpts), vp, vp, P(CgInfo), vp]
    L.dg_num_dofs.argtypes = [vp]
    L.dg_num_dofs.restype = ctypes.c_int64
    L.dg_num_elements.argtypes = [vp]
    L.dg_num_elements.restype = ctypes.c_int64
    L.dg_nodes_per_dir.argtypes = [vp]
    L.dg_apply_kernel.argtypes = [vp]
    L.dg_destroy.argtypes = [vp]
    L.dg_destroy.restype = None
    L.dg_last_error.argtypes = [vp]
    L.dg_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream, *keep) -> ctypes.c_void_p:
    """The HIP stream handle for a call.  When the work goes to a stream other
    than the current one, the tensors it uses (``keep``: outputs allocated
    here, contiguous temporaries, the workspace) are recorded on that stream,
    so the caching allocator does not hand their memory out again before the
    library's kernels on it have finished."""
    cur = torch.cuda.current_stream()
    s = stream if stream is not None else cur
    if s != cur:
        for t in keep:
            if t is not None:
                t.record_stream(s)
    return ctypes.c_void_p(s.cuda_stream)


def query_workspace(nx, ny, nz, degree, bc="dirichlet", trilinear=False, penalty_hat=0.0) -> int:
    d = MeshDesc(nx, ny, nz, degree, BC[bc], 0, penalty_hat, 1 if trilinear else None, None, None, 0)
    n = ctypes.c_size_t(0)
    rc = lib().dg_query_workspace(ctypes.byref(d), ctypes.byref(n))
    if rc != DG_OK:
        raise DGError(rc, lib().dg_last_error(None).decode())
    return n.value


class DGOperator:
    """SWIPDG operator on an nx*ny*nz mesh of the unit cube, Q_degree on GLL nodes.

    theta: CUDA float64 tensor (E,) with K = exp(theta) (None: K = 1).
    vertices: CUDA float64 tensor ((nx+1)(ny+1)(nz+1), 3) for trilinear elements
    (None: uniform grid, affine path).  Vectors are element-blocked CUDA tensors."""

    def __init__(self, nx: int, ny: int, nz: int, degree: int, bc: str = "dirichlet",
                 theta: Optional[torch.Tensor] = None, vertices: Optional[torch.Tensor] = None,
                 penalty_hat: float = 0.0, stream=None):
        self.nx, self.ny, self.nz, self.degree, self.bc = nx, ny, nz, degree, bc
        self.n = degree + 1
        self.E = nx * ny * nz
        self.ndof = self.E * self.n ** 3
        self.trilinear = vertices is not None
        L = lib()
        for t in (theta, vertices):
            if t is not None and (not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous()):
                raise ValueError("theta / vertices must be contiguous float64 CUDA tensors")
        nbytes = query_workspace(nx, ny, nz, degree, bc, self.trilinear, penalty_hat)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        desc = MeshDesc(nx, ny, nz, degree, BC[bc], 0, penalty_hat, _ptr(vertices), _ptr(theta),
                        _ptr(self.workspace), nbytes)
        h = ctypes.c_void_p()
        rc = L.dg_setup(ctypes.byref(desc), ctypes.byref(h), _stream(stream))
        if rc != DG_OK:
            raise DGError(rc, L.dg_last_error(None).decode())
        self._h = h

    KERNELS = {0: "affine", 1: "trilinear", 2: "parallelepiped"}

    @property
    def kernel(self) -> str:
        """The apply kernel chosen at setup: "affine", "trilinear" or "parallelepiped"."""
        return self.KERNELS[self._check(lib().dg_apply_kernel(self._h))]

    # -------------------------------------------------------------- helpers
    def _check(self, rc: int):
        if rc < 0:
            raise DGError(rc, lib().dg_last_error(self._h).decode())
        return rc

    def close(self):
        if getattr(self, "_h", None):
            lib().dg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, t: torch.Tensor, dtype) -> torch.Tensor:
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype:
            raise ValueError(f"expected a CUDA tensor of dtype {dtype}")
        if t.numel() != self.ndof or not t.is_contiguous():
            raise ValueError(f"expected a contiguous vector of {self.ndof} entries")
        return t

    # -------------------------------------------------------------- calls
    def set_theta(self, theta: torch.Tensor, stream=None):
        if theta.numel() != self.E or theta.dtype != torch.float64 or not theta.is_cuda:
            raise ValueError("theta must be a CUDA float64 tensor with one entry per element")
        th = theta.contiguous()
        self._check(lib().dg_set_theta(self._h, _ptr(th), _stream(stream, th, self.workspace)))

    def set_reaction(self, c: Optional[torch.Tensor], stream=None):
        """Reaction coefficients c_T (CUDA float64, one per element) or None to remove the term."""
        if c is not None and (c.numel() != self.E or c.dtype != torch.float64 or not c.is_cuda):
            raise ValueError("c must be a CUDA float64 tensor with one entry per element")
        cc = None if c is None else c.contiguous()
        self._check(lib().dg_set_reaction(self._h, _ptr(cc), _stream(stream, cc, self.workspace)))

    def apply(self, x: torch.Tensor, prec: str = "f64", out: Optional[torch.Tensor] = None,
              transpose: bool = False, stream=None) -> torch.Tensor:
        """y = A x (transpose: A^T x).  prec f64 (double in/out), f32 (float in/out),
        bf16 (bfloat16 in, float out), bf16_mfma (as bf16, tangential masses on the
        matrix cores; affine meshes, degree <= 4)."""
        self._vec(x, _IN_DTYPE[prec])
        y = torch.empty(self.ndof, dtype=_OUT_DTYPE[prec], device=x.device) if out is None else out
        self._vec(y, _OUT_DTYPE[prec])
        fn = lib().dg_apply_transpose if transpose else lib().dg_apply
        self._check(fn(self._h, PREC[prec], _ptr(x), _ptr(y), _stream(stream, x, y, self.workspace)))
        return y

    def apply_multi(self, X: torch.Tensor, prec: str = "f64", out: Optional[torch.Tensor] = None,
                    transpose: bool = False, stream=None) -> torch.Tensor:
        """Y = A X for nrhs vectors: X is a contiguous (nrhs, N_dof) tensor, one vector
        per row; returns Y of the same shape (output dtype of `prec`)."""
        if not isinstance(X, torch.Tensor) or not X.is_cuda or X.dtype != _IN_DTYPE[prec] or X.dim() != 2 \
                or X.shape[1] != self.ndof or not X.is_contiguous():
            raise ValueError(f"expected a contiguous CUDA tensor (nrhs, {self.ndof}) of dtype {_IN_DTYPE[prec]}")
        Y = torch.empty(X.shape, dtype=_OUT_DTYPE[prec], device=X.device) if out is None else out
        if Y.shape != X.shape or Y.dtype != _OUT_DTYPE[prec] or not Y.is_contiguous():
            raise ValueError("out has the wrong shape or dtype")
        self._check(lib().dg_apply_multi(self._h, PREC[prec], 1 if transpose else 0, X.shape[0], _ptr(X), _ptr(Y),
                                         _stream(stream, X, Y, self.workspace)))
        return Y

    def dA_dtheta(self, u: torch.Tensor, v: torch.Tensor, out: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
        """g_T = u^T (dA/dtheta_T) v."""
        self._vec(u, torch.float64)
        self._vec(v, torch.float64)
        g = torch.empty(self.E, dtype=torch.float64, device=u.device) if out is None else out
        self._check(lib().dg_dA_dtheta(self._h, _ptr(u), _ptr(v), _ptr(g), _stream(stream, u, v, g, self.workspace)))
        return g

    def dA_dtheta_noalloc(self, u: torch.Tensor, v: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
        """g_T = u^T (dA/dtheta_T) v through dg_dA_dtheta_noalloc (scratch in the library's
        static device array; ``out`` must be given, nothing is allocated)."""
        self._vec(u, torch.float64)
        self._vec(v, torch.float64)
        self._check(lib().dg_dA_dtheta_noalloc(self._h, _ptr(u), _ptr(v), _ptr(out),
                                               _stream(stream, u, v, out, self.workspace)))
        return out

    def diagonal(self, stream=None) -> torch.Tensor:
        d = torch.empty(self.ndof, dtype=torch.float64, device="cuda")
        self._check(lib().dg_diagonal(self._h, _ptr(d), _stream(stream, d, self.workspace)))
        return d

    def quadrature_points(self, stream=None) -> torch.Tensor:
        xq = torch.empty((self.ndof, 3), dtype=torch.float64, device="cuda")
        self._check(lib().dg_quadrature_points(self._h, _ptr(xq), _stream(stream, xq, self.workspace)))
        return xq

    def load_vector(self, fq: torch.Tensor, stream=None) -> torch.Tensor:
        self._vec(fq, torch.float64)
        b = torch.empty(self.ndof, dtype=torch.float64, device="cuda")
        self._check(lib().dg_load_vector(self._h, _ptr(fq), _ptr(b), _stream(stream, fq, b, self.workspace)))
        return b

    def cg_solve(self, b: torch.Tensor, x: Optional[torch.Tensor] = None, prec_inner: str = "f64",
                 precond: str = "jacobi", rtol: float = 1e-10, maxit: int = 100000,
                 inner_rtol: float = 0.0, max_outer: int = 0, transpose: bool = False,
                 check_every: int = 0, dc_mode: str = "restart", variant: str = "standard", stream=None):
        """Solve A x = b (A^T x = b).  Returns (x, info dict).

        prec_inner "f32" / "bf16" selects the FP64 defect correction; dc_mode
        "restart" starts every inner solve afresh, "keep" replaces the inner
        residual by the FP64 one and keeps the search direction.  inner_rtol
        and max_outer <= 0 take the library defaults, check_every <= 0 its default
        interval (32 iterations) between looks at the convergence flag."""
        self._vec(b, torch.float64)
        x = torch.zeros_like(b) if x is None else self._vec(x, torch.float64)
        o = CgOpts(PREC[prec_inner], PRECOND[precond], 1 if transpose else 0, rtol, inner_rtol, maxit,
                   max_outer, check_every, DC_MODE[dc_mode], CG_VARIANT[variant])
        info = CgInfo()
        rc = lib().dg_cg_solve(self._h, ctypes.byref(o), _ptr(b), _ptr(x), ctypes.byref(info),
                               _stream(stream, b, x, self.workspace))
        self._check(rc)
        return x, {"status": info.status, "iters": info.iters, "outer_iters": info.outer_iters,
                   "restarts": info.restarts, "rel_true_residual": info.rel_true_residual,
                   "seconds": info.seconds}


class DGSolve(torch.autograd.Function):
    """u = A(theta)^{-1} b with the adjoint gradient.

    forward(theta, b, op, opts) sets K = exp(theta) on ``op`` and solves with
    ``op.cg_solve(b, **opts)``; backward solves A^T lambda = grad_u and returns
    grad_theta = -dA_dtheta(lambda, u), grad_b = lambda."""

    @staticmethod
    def forward(ctx, theta, b, op, opts):
        op.set_theta(theta.detach().contiguous())
        u, info = op.cg_solve(b.detach().contiguous(), **(opts or {}))
        if info["status"] != DG_OK:
            raise DGError(info["status"], f"forward solve did not converge: {info}")
        ctx.save_for_backward(theta, u)
        ctx.op, ctx.opts = op, dict(opts or {})
        return u

    @staticmethod
    def backward(ctx, grad_u):
        theta, u = ctx.saved_tensors
        op = ctx.op
        op.set_theta(theta.detach().contiguous())
        opts = dict(ctx.opts)
        opts["transpose"] = True
        lam, info = op.cg_solve(grad_u.detach().contiguous(), **opts)
        if info["status"] != DG_OK:
            raise DGError(info["status"], f"adjoint solve did not converge: {info}")
        g = op.dA_dtheta(lam, u)
        return -g, lam, None, None
