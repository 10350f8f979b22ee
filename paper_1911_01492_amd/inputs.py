"""Seeded synthetic inputs shared by the GPU path, the tests and the oracle.

This module holds no arithmetic of the method: it only draws the arrays that
both sides receive (per-element log-coefficients, vectors, vertex
perturbations, observation noise, the elements probed by finite differences)
with ``numpy.random.default_rng(seed)`` (PCG64), in global element-blocked
order, and rounds FP64 data to the storage formats of the low-precision
applies.  The workload definitions mirror the problem families of Sec. 3.3
(axis-parallel grids with a constant coefficient per cell; multilinear
geometries) with the diffusion problem of Sec. 4.1.
"""
from __future__ import annotations

import numpy as np

# seeds of the synthetic workloads
S_X, S_K, S_B, S_OBS, S_NOISE, S_PERT, S_FD = 0, 1, 2, 3, 4, 5, 6
S_REACT = 7

DIRICHLET = 0
PERIODIC = 1

#: the five workloads: mesh, degree, boundary condition, geometry, coefficient
WORKLOADS = {
    "periodic_q2_4": dict(N=4, k=2, bc=PERIODIC, geometry="affine", coeff="one"),
    "dirichlet_q3_32": dict(N=32, k=3, bc=DIRICHLET, geometry="affine", coeff="lognormal"),
    "mixed_q4_64": dict(N=64, k=4, bc=DIRICHLET, geometry="affine", coeff="lognormal"),
    "adjoint_q3_32": dict(N=32, k=3, bc=DIRICHLET, geometry="affine", coeff="lognormal"),
    "trilinear_q7_48": dict(N=48, k=7, bc=DIRICHLET, geometry="trilinear", coeff="lognormal"),
}


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def theta(E: int, seed: int = S_K) -> np.ndarray:
    """theta_T ~ N(0, 1) i.i.d. per element, K_T = exp(theta_T)."""
    return rng(seed).standard_normal(E)


def reaction(E: int, lo: float = 0.5, hi: float = 2.0, seed: int = S_REACT) -> np.ndarray:
    """Per-element reaction coefficients c_T ~ U(lo, hi) (element order)."""
    return rng(seed).uniform(lo, hi, E)


def sheared_vertices(nx: int, ny: int, nz: int, s: float = 0.25) -> np.ndarray:
    """Vertices of the uniform grid under the affine map x -> x + s y + s z / 2,
    y -> y + s z (every element is the same parallelepiped)."""
    V = uniform_vertices(nx, ny, nz).copy()
    x, y, z = V[:, 0].copy(), V[:, 1].copy(), V[:, 2].copy()
    V[:, 0] = x + s * y + 0.5 * s * z
    V[:, 1] = y + s * z
    return V


def layered_shear_vertices(nx: int, ny: int, nz: int, s: float = 0.3, seed: int = 23) -> np.ndarray:
    """Vertices of the uniform grid sheared along x by a different U(-s, s)
    slope in every layer of elements along y: every element is a
    parallelepiped, but not all the same one."""
    V = uniform_vertices(nx, ny, nz).reshape(nz + 1, ny + 1, nx + 1, 3).copy()
    slope = rng(seed).uniform(-s, s, ny)
    V[..., 0] += (np.concatenate([[0.0], np.cumsum(slope)]) / ny)[None, :, None]
    return V.reshape(-1, 3)


def uniform_vector(n: int, seed: int = S_X) -> np.ndarray:
    """x ~ U(-1, 1) i.i.d."""
    return rng(seed).uniform(-1.0, 1.0, n)


def noise(n: int, std: float = 1e-3, seed: int = S_NOISE) -> np.ndarray:
    return std * rng(seed).standard_normal(n)


def fd_elements(E: int, m: int = 16, seed: int = S_FD) -> np.ndarray:
    return np.sort(rng(seed).choice(E, m, replace=False))


def uniform_vertices(nx: int, ny: int, nz: int) -> np.ndarray:
    """Vertex coordinates of the uniform grid of [0,1]^3, x-index fastest, shape ((nx+1)(ny+1)(nz+1), 3)."""
    X = np.zeros((nz + 1, ny + 1, nx + 1, 3))
    X[..., 0] = (np.arange(nx + 1) / nx)[None, None, :]
    X[..., 1] = (np.arange(ny + 1) / ny)[None, :, None]
    X[..., 2] = (np.arange(nz + 1) / nz)[:, None, None]
    return X.reshape(-1, 3)


def perturbed_vertices(N: int, amplitude: float = 0.1, seed: int = S_PERT) -> np.ndarray:
    """Uniform N^3 grid with interior vertices moved by U(-a h, a h) per coordinate
    (h = 1/N); vertices with any index in {0, N} stay in place."""
    h = 1.0 / N
    pert = rng(seed).uniform(-amplitude * h, amplitude * h, ((N + 1) ** 3, 3))
    idx = np.arange(N + 1)
    iz, iy, ix = np.meshgrid(idx, idx, idx, indexing="ij")
    bnd = ((ix == 0) | (ix == N) | (iy == 0) | (iy == N) | (iz == 0) | (iz == N)).reshape(-1)
    pert[bnd] = 0.0
    return uniform_vertices(N, N, N) + pert


def to_f32(x: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even FP64 -> FP32."""
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """FP64 -> FP32 (RNE) -> BF16 (RNE), returned as the uint16 bit patterns."""
    f = np.ascontiguousarray(to_f32(x)).view(np.uint32).astype(np.uint64)
    lsb = (f >> np.uint64(16)) & np.uint64(1)
    r = (f + np.uint64(0x7FFF) + lsb) >> np.uint64(16)
    nan = np.isnan(to_f32(x))
    r = r.astype(np.uint16)
    r[nan] = np.uint16(0x7FC0)
    return r


def bf16_bits_to_f64(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)
