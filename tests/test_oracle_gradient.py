"""P10: the oracle's sensitivity g_T = u^T (dA/dtheta_T) v, K_T = exp(theta_T),
against the complex-step derivative and central finite differences of the
assembled form (no GPU)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1911_01492_amd import inputs as I


@pytest.mark.parametrize("case", [((2, 2, 2), O.DIRICHLET, False), ((3, 2, 2), O.PERIODIC, False),
                                  ((2, 2, 2), O.DIRICHLET, True), ((1, 2, 2), O.PERIODIC, False),
                                  ((2, 1, 1), O.PERIODIC, False)])
@pytest.mark.parametrize("k", [1, 3])
def test_gradient_closed_form_vs_complex_step(case, k):
    (nx, ny, nz), bc, pert = case
    E = nx * ny * nz
    V = None
    if pert:
        V = I.uniform_vertices(2, 2, 2)
        V[13] += np.array([0.06, -0.04, 0.05])
    m = O.Mesh(nx, ny, nz, k, bc=bc, theta=I.theta(E, seed=12), vertices=V)
    u = I.uniform_vector(m.ndof, seed=13)
    v = I.uniform_vector(m.ndof, seed=14)
    g = O.dA_dtheta(m, u, v)
    gc = O.dA_dtheta(m, u, v, complex_step=True)
    assert np.max(np.abs(g - gc)) <= 1e-12 * np.max(np.abs(gc))


def test_gradient_vs_central_fd():
    """Local FD of u^T A(theta) v in one theta_T at a time (the form is linear in K)."""
    m = O.Mesh(2, 2, 2, 2, theta=I.theta(8, seed=15))
    u = I.uniform_vector(m.ndof, seed=16)
    v = I.uniform_vector(m.ndof, seed=17)
    g = O.dA_dtheta(m, u, v)
    h = 1e-5
    for T in range(8):
        tp = m.theta.copy()
        tm = m.theta.copy()
        tp[T] += h
        tm[T] -= h
        fp = u @ (O.assemble(m.replace(theta=tp)) @ v)
        fm = u @ (O.assemble(m.replace(theta=tm)) @ v)
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g[T]) <= 1e-8 * max(abs(g).max(), 1.0)


def test_gradient_sum_is_homogeneity():
    """A(c K) = c A(K): sum_T dA/dtheta_T = A, so sum_T g_T = u^T A v."""
    m = O.Mesh(3, 2, 2, 2, theta=I.theta(12, seed=18), vertices=None)
    u = I.uniform_vector(m.ndof, seed=19)
    v = I.uniform_vector(m.ndof, seed=20)
    g = O.dA_dtheta(m, u, v)
    A = O.assemble(m)
    assert abs(g.sum() - u @ (A @ v)) <= 1e-12 * abs(u @ (A @ v)) + 1e-12
    # homogeneity of the assembled matrix itself
    B = O.assemble(m.replace(theta=m.theta + np.log(3.0)))
    assert abs(B - 3.0 * A).max() <= 1e-13 * abs(B).max()


def test_gradient_element_subset():
    m = O.Mesh(3, 3, 2, 2, theta=I.theta(18, seed=21))
    u = I.uniform_vector(m.ndof, seed=22)
    v = I.uniform_vector(m.ndof, seed=23)
    g = O.dA_dtheta(m, u, v)
    el = [0, 7, 17]
    assert np.array_equal(O.dA_dtheta_elems(m, u, v, el), g[el])
