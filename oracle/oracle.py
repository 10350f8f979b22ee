"""Python access to the CPU oracle (TEST INFRASTRUCTURE, NOT PRODUCT CODE).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It wraps ``liboracle.so`` (built from ``dg_oracle.cpp`` by
``oracle/build.py``) with numpy/scipy types and adds two plain reference
computations that need no assembly:

* ``fast_diag_solve`` -- the exact solution for K == 1 on a uniform box mesh
  from the Kronecker-sum structure of the operator (1D SWIPDG operators along
  each axis, tangential 1D mass matrices), solved by fast diagonalisation;
* ``pcg`` -- Alg. "PCG" of Sec. 2.4 on the assembled matrix (in C++);
* ``block_jacobi_pcg`` -- the same algorithm with exact element-block inverses
  as the preconditioner (numpy).

The operator, its readings and its notation are those of Sec. 4.1 (SWIPDG
forms b_h and b_h^e); see the header of ``dg_oracle.cpp``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.linalg
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_c_i32 = ctypes.c_int32
_c_i64 = ctypes.c_int64
_c_dbl = ctypes.c_double
_c_vp = ctypes.c_void_p

DIRICHLET = 0
PERIODIC = 1

# planted mistakes (see dg_oracle.cpp); used only by the pin-sensitivity tests
MUTATIONS = {
    "plus_consistency": 1,
    "no_symmetry": 2,
    "no_penalty": 3,
    "no_boundary": 4,
    "jinv_not_transposed": 5,
    "arith_gamma": 6,
    "penalty_no_area": 7,
    "plus_side_at_one": 8,
}


class _CMesh(ctypes.Structure):
    _fields_ = [
        ("nx", _c_i32), ("ny", _c_i32), ("nz", _c_i32), ("degree", _c_i32),
        ("bc", _c_i32), ("quad_extra", _c_i32), ("mutation", _c_i32), ("pad_", _c_i32),
        ("penalty_hat", _c_dbl), ("vertices", _c_vp), ("theta", _c_vp), ("reaction", _c_vp),
    ]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b  # type: ignore
        _b.build()
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_tables.argtypes = [ctypes.c_int, ctypes.c_int, _c_vp, _c_vp, _c_vp]
    lib.oracle_csr_nnz.argtypes = [P(_CMesh)]
    lib.oracle_csr_nnz.restype = _c_i64
    lib.oracle_csr_assemble.argtypes = [P(_CMesh), _c_vp, _c_vp, _c_vp]
    lib.oracle_spmv.argtypes = [_c_i64, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp]
    lib.oracle_apply_rows.argtypes = [P(_CMesh), _c_vp, _c_i64, _c_vp, _c_vp]
    lib.oracle_pcg.argtypes = [_c_i64, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_dbl, ctypes.c_int,
                               ctypes.c_int, P(ctypes.c_int), P(_c_dbl)]
    lib.oracle_rhs.argtypes = [P(_CMesh), ctypes.c_int, _c_vp, _c_vp]
    lib.oracle_l2_error.argtypes = [P(_CMesh), _c_vp, ctypes.c_int, _c_vp]
    lib.oracle_l2_error.restype = _c_dbl
    lib.oracle_dA_dtheta.argtypes = [P(_CMesh), _c_vp, _c_vp, _c_vp]
    lib.oracle_dA_dtheta_cs.argtypes = [P(_CMesh), _c_vp, _c_vp, _c_vp]
    lib.oracle_dA_dtheta_elems.argtypes = [P(_CMesh), _c_vp, _c_vp, _c_i64, _c_vp, _c_vp]
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_c_vp)


@dataclass
class Mesh:
    """Structured hexahedral mesh of [0,1]^3 with per-element K = exp(theta)."""
    nx: int
    ny: int
    nz: int
    k: int
    bc: int = DIRICHLET
    theta: Optional[np.ndarray] = None      # (E,) float64, element order
    vertices: Optional[np.ndarray] = None   # ((nx+1)(ny+1)(nz+1), 3) float64
    quad_extra: int = 0
    mutation: int = 0
    penalty_hat: float = 0.0
    reaction: Optional[np.ndarray] = None   # (E,) float64 reaction coefficients c_T, element order
    _keep: list = field(default_factory=list, repr=False)

    @property
    def n(self) -> int:
        return self.k + 1

    @property
    def n3(self) -> int:
        return self.n ** 3

    @property
    def E(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def ndof(self) -> int:
        return self.E * self.n3

    def c(self) -> _CMesh:
        th = None if self.theta is None else np.ascontiguousarray(self.theta, dtype=np.float64)
        vx = None if self.vertices is None else np.ascontiguousarray(self.vertices, dtype=np.float64)
        if th is not None and th.size != self.E:
            raise ValueError("theta has the wrong length")
        if vx is not None and vx.size != 3 * (self.nx + 1) * (self.ny + 1) * (self.nz + 1):
            raise ValueError("vertices have the wrong length")
        rc = None if self.reaction is None else np.ascontiguousarray(self.reaction, dtype=np.float64)
        if rc is not None and rc.size != self.E:
            raise ValueError("reaction has the wrong length")
        self._keep = [th, vx, rc]
        return _CMesh(self.nx, self.ny, self.nz, self.k, self.bc, self.quad_extra, self.mutation, 0,
                      self.penalty_hat, _ptr(vx), _ptr(th), _ptr(rc))

    def replace(self, **kw) -> "Mesh":
        d = dict(nx=self.nx, ny=self.ny, nz=self.nz, k=self.k, bc=self.bc, theta=self.theta,
                 vertices=self.vertices, quad_extra=self.quad_extra, mutation=self.mutation,
                 penalty_hat=self.penalty_hat, reaction=self.reaction)
        d.update(kw)
        return Mesh(**d)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def tables(n: int, nq: Optional[int] = None):
    """GLL nodes (n), Gauss points and weights (nq, default n), all on [0,1]."""
    nq = n if nq is None else nq
    gll = np.zeros(n)
    gx = np.zeros(nq)
    gw = np.zeros(nq)
    if _load().oracle_tables(n, nq, _ptr(gll), _ptr(gx), _ptr(gw)) != 0:
        raise ValueError("bad table size")
    return gll, gx, gw


def assemble(mesh: Mesh) -> sp.csr_matrix:
    """The global matrix A_ij = b_h(phi_j, phi_i) as CSR (float64, int64 indices)."""
    lib = _load()
    cm = mesh.c()
    nnz = lib.oracle_csr_nnz(ctypes.byref(cm))
    if nnz < 0:
        raise ValueError("invalid mesh")
    rowptr = np.zeros(mesh.ndof + 1, dtype=np.int64)
    cols = np.zeros(nnz, dtype=np.int64)
    vals = np.zeros(nnz, dtype=np.float64)
    if lib.oracle_csr_assemble(ctypes.byref(cm), _ptr(rowptr), _ptr(cols), _ptr(vals)) != 0:
        raise RuntimeError("assembly failed")
    return sp.csr_matrix((vals, cols, rowptr), shape=(mesh.ndof, mesh.ndof))


def spmv(A: sp.csr_matrix, x: np.ndarray) -> np.ndarray:
    """y = A x with the oracle's own OpenMP CSR loop."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros(A.shape[0])
    ip = np.ascontiguousarray(A.indptr, dtype=np.int64)
    ix = np.ascontiguousarray(A.indices, dtype=np.int64)
    dv = np.ascontiguousarray(A.data, dtype=np.float64)
    _load().oracle_spmv(A.shape[0], _ptr(ip), _ptr(ix), _ptr(dv), _ptr(x), _ptr(y))
    return y


def csr_arrays(A: sp.csr_matrix):
    return (np.ascontiguousarray(A.indptr, dtype=np.int64),
            np.ascontiguousarray(A.indices, dtype=np.int64),
            np.ascontiguousarray(A.data, dtype=np.float64))


def apply_rows(mesh: Mesh, x: np.ndarray, elems) -> np.ndarray:
    """Rows of A x for the given elements, shape (len(elems), n^3)."""
    lib = _load()
    cm = mesh.c()
    el = np.ascontiguousarray(np.asarray(elems, dtype=np.int64))
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros((el.size, mesh.n3))
    if lib.oracle_apply_rows(ctypes.byref(cm), _ptr(x), el.size, _ptr(el), _ptr(y)) != 0:
        raise ValueError("invalid mesh or element index")
    return y


def pcg(A: sp.csr_matrix, b: np.ndarray, rtol: float = 1e-10, maxit: int = 10000,
        jacobi: bool = True, x0: Optional[np.ndarray] = None):
    """Alg. PCG (Sec. 2.4) in C++ on the assembled matrix: (x, iterations, true rel. residual)."""
    ip, ix, dv = csr_arrays(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    it = ctypes.c_int(0)
    rr = _c_dbl(0.0)
    _load().oracle_pcg(A.shape[0], _ptr(ip), _ptr(ix), _ptr(dv), _ptr(b), _ptr(x), rtol, maxit,
                       1 if jacobi else 0, ctypes.byref(it), ctypes.byref(rr))
    return x, it.value, rr.value


def block_jacobi_pcg(A: sp.csr_matrix, b: np.ndarray, block: int, rtol: float = 1e-10, maxit: int = 10000,
                     x0: Optional[np.ndarray] = None):
    """Alg. PCG (Sec. 2.4) with the preconditioner M = blockdiag(A)^{-1} over the
    consecutive diagonal blocks of size `block` (the element blocks of Sec. 3.4's
    block preconditioners), in numpy: every block inverted densely.  Steps in
    the order of the algorithm: r0 = b - A x0, p1 = M r0, rho1 = <p1, r0>; per
    iteration q = A p, alpha = <p, q>, x += rho/alpha p, r -= rho/alpha q,
    z = M r, stop when ||r|| <= rtol ||b||, rho' = <z, r>, p = z + rho'/rho p.
    Returns (x, iterations, true relative residual)."""
    nblk = A.shape[0] // block
    Ad = A.tocsr()
    inv = [np.linalg.inv(Ad[e * block:(e + 1) * block, e * block:(e + 1) * block].toarray()) for e in range(nblk)]

    def M(v):
        return np.concatenate([inv[e] @ v[e * block:(e + 1) * block] for e in range(nblk)])

    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    r = b - Ad @ x
    p = M(r)
    rho = p @ r
    it = 0
    done = np.linalg.norm(r) <= rtol * bnorm
    while not done and it < maxit:
        it += 1
        q = Ad @ p
        lam = rho / (p @ q)
        x = x + lam * p
        r = r - lam * q
        z = M(r)
        if np.linalg.norm(r) <= rtol * bnorm:
            break
        rho_new = z @ r
        p = z + (rho_new / rho) * p
        rho = rho_new
    res = np.linalg.norm(b - Ad @ x) / (bnorm if bnorm > 0 else 1.0)
    return x, it, float(res)


def rhs(mesh: Mesh, kind: str = "sine", coef: Optional[np.ndarray] = None) -> np.ndarray:
    """Load vector: kind 'sine' (f = 3 pi^2 sin sin sin, g = 0) or 'poly'
    (u = polynomial with coefficients coef[a,b,c] of x^a y^b z^c, f = -K lap u,
    Dirichlet data g = u added by the weak-Dirichlet lifting terms)."""
    lib = _load()
    cm = mesh.c()
    fk = {"sine": 1, "poly": 2}[kind]
    c = None if coef is None else np.ascontiguousarray(coef, dtype=np.float64).ravel(order="F")
    b = np.zeros(mesh.ndof)
    if lib.oracle_rhs(ctypes.byref(cm), fk, _ptr(c), _ptr(b)) != 0:
        raise ValueError("bad rhs request")
    return b


def l2_error(mesh: Mesh, u: np.ndarray, kind: str = "sine", coef: Optional[np.ndarray] = None) -> float:
    lib = _load()
    cm = mesh.c()
    fk = {"sine": 1, "poly": 2}[kind]
    c = None if coef is None else np.ascontiguousarray(coef, dtype=np.float64).ravel(order="F")
    u = np.ascontiguousarray(u, dtype=np.float64)
    return float(lib.oracle_l2_error(ctypes.byref(cm), _ptr(u), fk, _ptr(c)))


def dA_dtheta(mesh: Mesh, u: np.ndarray, v: np.ndarray, complex_step: bool = False) -> np.ndarray:
    """g_T = u^T (dA/dtheta_T) v for every element T."""
    lib = _load()
    cm = mesh.c()
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    g = np.zeros(mesh.E)
    fn = lib.oracle_dA_dtheta_cs if complex_step else lib.oracle_dA_dtheta
    if fn(ctypes.byref(cm), _ptr(u), _ptr(v), _ptr(g)) != 0:
        raise ValueError("invalid mesh")
    return g


def dA_dtheta_elems(mesh: Mesh, u: np.ndarray, v: np.ndarray, elems) -> np.ndarray:
    """g_T = u^T (dA/dtheta_T) v for the listed elements only."""
    lib = _load()
    cm = mesh.c()
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    el = np.ascontiguousarray(np.asarray(elems, dtype=np.int64))
    g = np.zeros(el.size)
    if lib.oracle_dA_dtheta_elems(ctypes.byref(cm), _ptr(u), _ptr(v), el.size, _ptr(el), _ptr(g)) != 0:
        raise ValueError("invalid mesh or element index")
    return g


# --------------------------------------------------------------------------
# Kronecker-sum structure for K == 1 on uniform box meshes
# --------------------------------------------------------------------------

def swipdg_1d(N: int, k: int, bc: int, penalty_hat: float = 0.0):
    """1D SWIPDG stiffness L and mass M (physical scaling, h = 1/N, K = 1) on
    N elements with the element-blocked GLL basis.  Faces: -1/2 (u'^- + u'^+)[v]
    - 1/2 (v'^- + v'^+)[u] + (sigma_hat/h)[u][v]; Dirichlet ends with outward n."""
    n = k + 1
    h = 1.0 / N
    sh = penalty_hat if penalty_hat > 0 else 2.0 * (k + 1) ** 2
    gll, gx, gw = tables(n, n)
    # Lagrange values/derivatives by the product formula
    def lag(i, x):
        return np.prod([(x - gll[j]) / (gll[i] - gll[j]) for j in range(n) if j != i], axis=0)

    def dlag(i, x):
        s = 0.0
        for m in range(n):
            if m == i:
                continue
            t = 1.0 / (gll[i] - gll[m])
            for j in range(n):
                if j != i and j != m:
                    t = t * (x - gll[j]) / (gll[i] - gll[j])
            s = s + t
        return s

    B = np.array([[lag(i, x) for i in range(n)] for x in gx])
    D = np.array([[dlag(i, x) for i in range(n)] for x in gx])
    Mr = B.T @ np.diag(gw) @ B
    Sr = D.T @ np.diag(gw) @ D
    e0 = np.array([lag(i, 0.0) for i in range(n)])
    e1 = np.array([lag(i, 1.0) for i in range(n)])
    d0 = np.array([dlag(i, 0.0) for i in range(n)]) / h
    d1 = np.array([dlag(i, 1.0) for i in range(n)]) / h
    L = np.zeros((N * n, N * n))
    M = np.zeros((N * n, N * n))
    for e in range(N):
        s = slice(e * n, (e + 1) * n)
        L[s, s] += Sr / h
        M[s, s] += Mr * h
    sig = sh / h
    nfaces = N if bc == PERIODIC else N - 1
    for f in range(nfaces):
        em, ep = f, (f + 1) % N
        idx = np.r_[em * n:(em + 1) * n, ep * n:(ep + 1) * n]
        jump = np.r_[e1, -e0]
        flux = np.r_[d1, d0]
        loc = (-0.5 * np.outer(jump, flux) - 0.5 * np.outer(flux, jump)
               + sig * np.outer(jump, jump))
        L[np.ix_(idx, idx)] += loc
    if bc == DIRICHLET:
        # x = 0: outward normal -1 ; x = 1: outward normal +1
        s = slice(0, n)
        L[s, s] += np.outer(e0, d0) + np.outer(d0, e0) + sig * np.outer(e0, e0)
        s = slice((N - 1) * n, N * n)
        L[s, s] += -np.outer(e1, d1) - np.outer(d1, e1) + sig * np.outer(e1, e1)
    return L, M


def blocked_to_tensor(u: np.ndarray, N, n) -> np.ndarray:
    """Element-blocked vector -> tensor indexed [z, y, x] (global per-axis index)."""
    Nx, Ny, Nz = N
    t = u.reshape(Nz, Ny, Nx, n, n, n)          # ez, ey, ex, i3, i2, i1
    return t.transpose(0, 3, 1, 4, 2, 5).reshape(Nz * n, Ny * n, Nx * n)


def tensor_to_blocked(t: np.ndarray, N, n) -> np.ndarray:
    Nx, Ny, Nz = N
    u = t.reshape(Nz, n, Ny, n, Nx, n).transpose(0, 2, 4, 1, 3, 5)
    return np.ascontiguousarray(u).reshape(-1)


def fast_diag_solve(nx: int, ny: int, nz: int, k: int, bc: int, b: np.ndarray,
                    penalty_hat: float = 0.0) -> np.ndarray:
    """Exact A^{-1} b for K == 1 on the uniform nx*ny*nz mesh:
    A = M_z (x) M_y (x) L_x + M_z (x) L_y (x) M_x + L_z (x) M_y (x) M_x and
    L Q = M Q Lambda, Q^T M Q = I per axis (Dirichlet only: periodic A is singular)."""
    n = k + 1
    Q, lam = [], []
    for N in (nx, ny, nz):
        L, M = swipdg_1d(N, k, bc, penalty_hat)
        w, V = scipy.linalg.eigh(L, M)
        Q.append(V)
        lam.append(w)
    T = blocked_to_tensor(np.asarray(b, dtype=np.float64), (nx, ny, nz), n)
    C = np.einsum("za,zyx->ayx", Q[2], T)
    C = np.einsum("yb,ayx->abx", Q[1], C)
    C = np.einsum("xc,abx->abc", Q[0], C)
    den = lam[2][:, None, None] + lam[1][None, :, None] + lam[0][None, None, :]
    C = C / den
    X = np.einsum("za,abc->zbc", Q[2], C)
    X = np.einsum("yb,zbc->zyc", Q[1], X)
    X = np.einsum("xc,zyc->zyx", Q[0], X)
    return tensor_to_blocked(X, (nx, ny, nz), n)
