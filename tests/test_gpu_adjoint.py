"""GPU adjoint: the sensitivity kernel u^T (dA/dtheta_T) v against the
oracle, and the adjoint gradient of J(theta) = 1/2 ||u(theta) - u_obs||^2
(u = A(theta)^{-1} b) through torch.autograd against the oracle's gradient and
against central finite differences (tiers (ii)-(iv) of the gradient checks)."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1911_01492_amd import inputs as I  # noqa: E402
from paper_1911_01492_amd.dg import DG_OK, DGOperator, DGSolve  # noqa: E402
from tests.gpu_util import banner, dev, host, rel_l2  # noqa: E402

BCS = {"dirichlet": O.DIRICHLET, "periodic": O.PERIODIC}


def _sine_rhs(op):
    xq = op.quadrature_points()
    fq = 3 * math.pi ** 2 * torch.sin(math.pi * xq[:, 0]) * torch.sin(math.pi * xq[:, 1]) * \
        torch.sin(math.pi * xq[:, 2])
    return op.load_vector(fq.contiguous())


@pytest.mark.parametrize("case", [((2, 2, 2), "dirichlet"), ((3, 2, 2), "periodic"), ((1, 2, 2), "periodic"),
                                  ((2, 1, 1), "periodic"), ((5, 3, 4), "dirichlet")])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_sensitivity_kernel(case, k):
    shape, bc = case
    banner(f"dA/dtheta {shape} {bc} k={k}")
    E = int(np.prod(shape))
    theta = I.theta(E, seed=31)
    m = O.Mesh(*shape, k, bc=BCS[bc], theta=theta)
    op = DGOperator(*shape, k, bc, theta=dev(theta))
    u = I.uniform_vector(m.ndof, seed=32)
    v = I.uniform_vector(m.ndof, seed=33)
    g = host(op.dA_dtheta(dev(u), dev(v)))
    ref = O.dA_dtheta(m, u, v)
    assert np.max(np.abs(g - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("case", [((2, 2, 2), "dirichlet"), ((3, 2, 2), "periodic"), ((1, 2, 2), "periodic"),
                                  ((3, 3, 2), "dirichlet")])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_sensitivity_kernel_trilinear(case, k):
    """Curved (perturbed trilinear) meshes, with a reaction term that the
    sensitivity must ignore."""
    from tests.test_gpu_trilinear import box_vertices
    shape, bc = case
    banner(f"dA/dtheta trilinear {shape} {bc} k={k}")
    E = int(np.prod(shape))
    theta = I.theta(E, seed=41)
    V = box_vertices(*shape, seed=42)
    m = O.Mesh(*shape, k, bc=BCS[bc], theta=theta, vertices=V)
    op = DGOperator(*shape, k, bc, theta=dev(theta), vertices=dev(V))
    op.set_reaction(dev(I.reaction(E)))
    u = I.uniform_vector(m.ndof, seed=43)
    v = I.uniform_vector(m.ndof, seed=44)
    g = host(op.dA_dtheta(dev(u), dev(v)))
    ref = O.dA_dtheta(m, u, v)
    err = np.max(np.abs(g - ref)) / np.max(np.abs(ref))
    print(f"dA/dtheta trilinear {shape} {bc} k={k}: max rel err {err:.3e}")
    assert err <= 1e-12


def test_adjoint_gradient_trilinear():
    """Autograd gradient on a curved 3^3 Q2 mesh against the oracle's adjoint
    gradient from direct solves."""
    from tests.test_gpu_trilinear import box_vertices
    banner("adjoint trilinear")
    N, k = 3, 2
    E = N ** 3
    theta = I.theta(E, seed=51)
    V = box_vertices(N, N, N, seed=52)
    m = O.Mesh(N, N, N, k, theta=theta, vertices=V)
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(theta), vertices=dev(V))
    bs = I.uniform_vector(m.ndof, seed=I.S_B)
    u_obs = I.noise(m.ndof, std=1.0, seed=53)
    th = dev(theta).requires_grad_(True)
    u = DGSolve.apply(th, dev(bs), op, {"rtol": 1e-13})
    loss = 0.5 * torch.sum((u - dev(u_obs)) ** 2)
    loss.backward()
    A = O.assemble(m).tocsc()
    u0 = spla.spsolve(A, bs)
    lam = spla.spsolve(A.T.tocsc(), u0 - u_obs)
    g_ora = -O.dA_dtheta(m, lam, u0)
    e = np.max(np.abs(host(th.grad) - g_ora)) / np.max(np.abs(g_ora))
    print(f"adjoint gradient trilinear 3^3 Q2 vs oracle adjoint: max rel err {e:.3e}")
    assert e <= 1e-8


def test_sensitivity_full_size():
    """32^3 Q3: sampled elements by the oracle, and sum_T g_T = u^T A v."""
    banner("dA/dtheta full size")
    N, k = 32, 3
    theta = I.theta(N ** 3)
    m = O.Mesh(N, N, N, k, theta=theta)
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(theta))
    u = I.uniform_vector(m.ndof, seed=34)
    v = I.uniform_vector(m.ndof, seed=35)
    g = host(op.dA_dtheta(dev(u), dev(v)))
    el = I.fd_elements(N ** 3)
    el = np.unique(np.r_[el, 0, N ** 3 - 1, N - 1])
    ref = O.dA_dtheta_elems(m, u, v, el)
    e = np.max(np.abs(g[el] - ref)) / np.max(np.abs(ref))
    print(f"dA/dtheta 32^3 Q3 sampled elements: max rel err {e:.3e}")
    assert e <= 1e-12
    Av = host(op.apply(dev(v)))
    assert abs(g.sum() - u @ Av) <= 1e-11 * abs(u @ Av)


def _loss_setup(N, k):
    theta = I.theta(N ** 3)
    theta_obs = I.theta(N ** 3, seed=I.S_OBS)
    m = O.Mesh(N, N, N, k, theta=theta)
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(theta))
    b = _sine_rhs(op)
    return theta, theta_obs, m, op, b


def test_adjoint_gradient_small_vs_oracle_and_fd():
    """N = 4, Q3: GPU autograd gradient against the oracle gradient from direct
    solves (adjoint formula) and against central FD of J with direct solves."""
    banner("adjoint small")
    N, k = 4, 3
    theta, theta_obs, m, op, b = _loss_setup(N, k)
    bs = host(b)
    A_obs = O.assemble(m.replace(theta=theta_obs)).tocsc()
    u_obs = spla.spsolve(A_obs, bs) + I.noise(m.ndof)
    th = dev(theta).requires_grad_(True)
    u = DGSolve.apply(th, b, op, {"rtol": 1e-13})
    loss = 0.5 * torch.sum((u - dev(u_obs)) ** 2)
    loss.backward()
    g_gpu = host(th.grad)

    def J(t):
        A = O.assemble(m.replace(theta=t)).tocsc()
        uu = spla.spsolve(A, bs)
        return 0.5 * np.sum((uu - u_obs) ** 2), uu, A

    J0, u0, A0 = J(theta)
    lam = spla.spsolve(A0.T.tocsc(), u0 - u_obs)
    g_ora = -O.dA_dtheta(m, lam, u0)
    assert abs(float(loss.detach()) - J0) <= 1e-10 * J0
    e = np.max(np.abs(g_gpu - g_ora)) / np.max(np.abs(g_ora))
    print(f"adjoint gradient 4^3 Q3 vs oracle adjoint: max rel err {e:.3e}")
    assert e <= 1e-8
    h = 1e-6
    for T in I.fd_elements(N ** 3, m=8):
        tp, tm = theta.copy(), theta.copy()
        tp[T] += h
        tm[T] -= h
        fd = (J(tp)[0] - J(tm)[0]) / (2 * h)
        assert abs(fd - g_gpu[T]) <= 1e-6 * max(abs(g_gpu[T]), 1e-3 * np.max(np.abs(g_gpu))), (T, fd, g_gpu[T])


def test_adjoint_gradient_full_size_fd():
    """32^3 Q3, 16 seeded elements: central FD of J by perturbation solves
    A(theta+-) du = -(A(theta+-) - A(theta)) u (exact far from T because the
    kernel is deterministic), dJ = (u - u_obs).(du+ - du-) + 1/2(|du+|^2 - |du-|^2)."""
    banner("adjoint full size FD")
    N, k = 32, 3
    theta, theta_obs, m, op, b = _loss_setup(N, k)
    opts = {"rtol": 1e-12}
    u_obs = DGSolve.apply(dev(theta_obs), b, op, opts) + dev(I.noise(m.ndof))
    th = dev(theta).requires_grad_(True)
    u = DGSolve.apply(th, b, op, opts)
    loss = 0.5 * torch.sum((u - u_obs) ** 2)
    loss.backward()
    g = host(th.grad)
    u = u.detach()
    r = u - u_obs
    h = 1e-6
    Au = op.apply(u)
    gmax = np.max(np.abs(g))
    worst = 0.0
    for T in I.fd_elements(N ** 3):
        dJ = []
        for sgn in (1.0, -1.0):
            tp = theta.copy()
            tp[T] += sgn * h
            op.set_theta(dev(tp))
            rhs = -(op.apply(u) - Au)
            du, info = op.cg_solve(rhs.contiguous(), rtol=1e-11)
            assert info["status"] == DG_OK
            dJ.append(float(r @ du + 0.5 * du @ du))
        fd = (dJ[0] - dJ[1]) / (2 * h)
        err = abs(fd - g[T]) / max(abs(g[T]), 1e-3 * gmax)
        worst = max(worst, err)
    op.set_theta(dev(theta))
    print(f"full-size FD: worst relative error {worst:.3e}, max|g| {gmax:.3e}")
    assert worst <= 1e-6
