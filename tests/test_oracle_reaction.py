"""Pins of the reaction term int c_T u v (diffusion-reaction problems of
Sec. 3.3) in the oracle, against facts that do not come from the oracle's
own assembly: the volume of the domain, the Kronecker product of the 1D Gauss
mass matrices (independent numpy tables), and the L2 convergence rate to a
manufactured solution of -div(grad u) + c u = f."""
import numpy as np
import pytest

from oracle import brute as B
from oracle import oracle as O
from paper_1911_01492_amd import inputs as I


@pytest.mark.parametrize("k", [1, 2, 3])
def test_total_mass_is_domain_volume(k):
    """Periodic unit cube, constant c: A 1 = c M 1 and 1^T M 1 = |Omega| = 1,
    so the sum of all entries of A is c (the diffusion part sums to 0)."""
    N, c = 3, 2.5
    m = O.Mesh(N, N, N, k, bc=O.PERIODIC, theta=I.theta(N ** 3, seed=4), reaction=np.full(N ** 3, c))
    A = O.assemble(m)
    one = np.ones(A.shape[0])
    assert abs(one @ (A @ one) - c) <= 1e-12 * c
    m2 = m.replace(vertices=I.perturbed_vertices(N, 0.1, seed=5))
    A2 = O.assemble(m2)
    assert abs(one @ (A2 @ one) - c) <= 1e-12 * c


@pytest.mark.parametrize("k", [1, 2, 4])
def test_reaction_is_blockwise_kronecker_mass(k):
    """Affine box elements: A(c) - A(0) is block diagonal with blocks
    c_T h_x h_y h_z (M (x) M (x) M), M the 1D mass matrix on [0,1] built from
    independent numpy Gauss / Lobatto tables."""
    nx, ny, nz = 2, 3, 1
    E = nx * ny * nz
    c = np.random.default_rng(7).uniform(0.5, 2.0, E)
    m0 = O.Mesh(nx, ny, nz, k, theta=I.theta(E, seed=3))
    Ac = O.assemble(m0.replace(reaction=c))
    D = (Ac - O.assemble(m0)).toarray()
    nodes = B.gll_nodes01(k + 1)
    xq, wq = B.gauss01(k + 1)
    P, _ = B.lagrange_polys(nodes)
    V = np.array([[np.polynomial.polynomial.polyval(x, P[i]) for i in range(k + 1)] for x in xq])
    M1 = V.T @ np.diag(wq) @ V
    kron = np.kron(M1, np.kron(M1, M1))
    n3 = (k + 1) ** 3
    vol = 1.0 / (nx * ny * nz)
    ref = np.zeros_like(D)
    for e in range(E):
        ref[e * n3:(e + 1) * n3, e * n3:(e + 1) * n3] = c[e] * vol * kron
    # the difference carries the rounding of the O(|A|) diffusion entries it cancels
    assert np.abs(D - ref).max() <= 1e-14 * abs(Ac).max()


@pytest.mark.parametrize("k", [1, 2])
def test_reaction_convergence_rate(k):
    """-div(grad u) + c u = f with u = sin(pi x) sin(pi y) sin(pi z), weak
    Dirichlet: f = (3 pi^2 + c) u, i.e. the load vector of the sine right-hand
    side scaled by (3 pi^2 + c) / (3 pi^2); L2 rate >= k + 1 - 0.2."""
    c = 5.0
    errs = []
    for N in (2, 4, 8):
        m = O.Mesh(N, N, N, k, reaction=np.full(N ** 3, c))
        A = O.assemble(m)
        b = O.rhs(m, "sine") * (3 * np.pi ** 2 + c) / (3 * np.pi ** 2)
        u, it, rr = O.pcg(A, b, rtol=1e-13)
        errs.append(O.l2_error(m, u, "sine"))
    rate = np.log2(errs[-2] / errs[-1])
    assert rate >= k + 1 - 0.2, (errs, rate)
