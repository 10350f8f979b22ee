"""Pins of the CPU oracle against what mathematics fixes (no GPU).

Each test cites the property it checks.  P-numbers refer to the list of pins
in the design notes; the operator is the SWIPDG form of Sec. 4.1.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import brute, oracle as O
from paper_1911_01492_amd import inputs as I

SMALL_MESHES = [(1, 1, 1), (2, 1, 1), (2, 2, 1), (2, 2, 2)]


def _pert_222():
    """2x2x2 mesh with the centre vertex moved (the only interior vertex)."""
    V = I.uniform_vertices(2, 2, 2)
    V[13] += np.array([0.07, -0.05, 0.04])
    return V


# ---------------------------------------------------------------- P1 / P2

@pytest.mark.parametrize("bc", [O.DIRICHLET, O.PERIODIC])
@pytest.mark.parametrize("pert", [False, True])
def test_symmetry(bc, pert):
    """P1: A = A^T (the SWIPDG form is symmetric)."""
    N, k = 3, 2
    V = I.perturbed_vertices(N, 0.1, seed=11) if pert else None
    A = O.assemble(O.Mesh(N, N, N, k, bc=bc, theta=I.theta(N ** 3, seed=3), vertices=V))
    assert abs(A - A.T).max() <= 1e-14 * abs(A).max()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_periodic_constant_nullspace(k):
    """P2: A 1 = 0 on periodic meshes for any K and any periodic perturbation."""
    for theta, V in [(None, None), (I.theta(27, seed=7), I.perturbed_vertices(3, 0.1, seed=8))]:
        A = O.assemble(O.Mesh(3, 3, 3, k, bc=O.PERIODIC, theta=theta, vertices=V))
        r = A @ np.ones(A.shape[0])
        assert np.abs(r).max() <= 1e-13 * abs(A).max()


def test_periodic_q2_4_workload():
    """P2 on the 4^3 periodic Q2 workload, plus its size."""
    A = O.assemble(O.Mesh(4, 4, 4, 2, bc=O.PERIODIC))
    assert A.shape == (1728, 1728)
    assert np.abs(A @ np.ones(1728)).max() <= 1e-13 * abs(A).max()


# ---------------------------------------------------------------- P3

@pytest.mark.parametrize("mesh", SMALL_MESHES)
@pytest.mark.parametrize("k", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", [O.DIRICHLET, O.PERIODIC])
def test_definiteness(mesh, k, bc):
    """P3: Dirichlet lambda_min > 0; periodic exactly one |lambda| < 1e-10 lambda_max,
    lognormal K, chosen penalty."""
    nx, ny, nz = mesh
    th = I.theta(nx * ny * nz, seed=100 + k)
    A = O.assemble(O.Mesh(nx, ny, nz, k, bc=bc, theta=th)).toarray()
    ev = np.linalg.eigvalsh(A)
    if bc == O.DIRICHLET:
        assert ev[0] > 1e-8 * ev[-1]
    else:
        small = np.sum(np.abs(ev) < 1e-10 * ev[-1])
        assert small == 1 and ev[1] > 1e-8 * ev[-1]


@pytest.mark.parametrize("k", [5, 6, 7])
def test_definiteness_high_order(k):
    for mesh in [(1, 1, 1), (2, 1, 1)]:
        A = O.assemble(O.Mesh(*mesh, k, theta=I.theta(np.prod(mesh), seed=k))).toarray()
        ev = np.linalg.eigvalsh(A)
        assert ev[0] > 1e-9 * ev[-1]


def test_definiteness_perturbed():
    A = O.assemble(O.Mesh(2, 2, 2, 3, theta=I.theta(8, seed=9), vertices=_pert_222())).toarray()
    assert np.linalg.eigvalsh(A)[0] > 0


# ---------------------------------------------------------------- P4 / P5

@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("pert", [False, True])
def test_convergence_rate(k, pert):
    """P4: K = 1, u = sin(pi x) sin(pi y) sin(pi z), Dirichlet: the L2 rate of the
    finest pair is >= k + 1 - 0.2 (this pins the sign of the consistency terms)."""
    errs = []
    for N in (2, 4, 8):
        V = I.perturbed_vertices(N, 0.1, seed=21) if pert else None
        m = O.Mesh(N, N, N, k, vertices=V)
        A = O.assemble(m)
        u, _, rr = O.pcg(A, O.rhs(m, "sine"), rtol=1e-13)
        assert rr < 1e-12
        errs.append(O.l2_error(m, u, "sine"))
    rate = np.log2(errs[-2] / errs[-1])
    assert rate >= k + 1 - 0.2, (errs, rate)


@pytest.mark.parametrize("N,k,pert", [(4, 2, False), (2, 3, False), (3, 1, True), (3, 2, True)])
def test_l2_error_closed_forms(N, k, pert):
    """The L2 error helper itself, two-sided: for u_h = 0 it is the L2 norm of the
    exact solution over the unit cube, ||sin(pi x) sin(pi y) sin(pi z)|| = 1/sqrt(8),
    ||x|| = 1/sqrt(3), ||y z|| = 1/3; for u_h = c and u = 0 it is |c| (unit
    volume).  Also on perturbed trilinear meshes, which tile the same cube.  A
    dropped square root, weight or |det J| moves every one of these values."""
    V = I.perturbed_vertices(N, 0.1, seed=5 + k) if pert else None
    m = O.Mesh(N, N, N, k, vertices=V)
    z = np.zeros(m.ndof)
    # the sine is integrated by (k+3)-point Gauss: not exact, error well below 1e-7 here
    assert abs(O.l2_error(m, z, "sine") - 1 / np.sqrt(8)) <= 1e-7
    cx = np.zeros((k + 1,) * 3)
    cx[1, 0, 0] = 1.0
    assert abs(O.l2_error(m, z, "poly", cx) - 1 / np.sqrt(3)) <= 1e-13
    cyz = np.zeros((k + 1,) * 3)
    cyz[0, 1, 1] = 1.0
    assert abs(O.l2_error(m, z, "poly", cyz) - 1 / 3) <= 1e-13
    assert abs(O.l2_error(m, np.full(m.ndof, -2.5), "poly", np.zeros((k + 1,) * 3)) - 2.5) <= 1e-13


@pytest.mark.parametrize("k", [1, 2, 3])
def test_polynomial_reproduction_affine(k):
    """P5: for p in global Q_k with f = -lap p and Dirichlet data g = p, u_h = p."""
    coef = np.random.default_rng(40 + k).uniform(-1, 1, (k + 1, k + 1, k + 1))
    m = O.Mesh(3, 2, 2, k, theta=np.full(12, np.log(2.5)))  # constant K
    A = O.assemble(m)
    u = spla.spsolve(A.tocsc(), O.rhs(m, "poly", coef))
    assert O.l2_error(m, u, "poly", coef) < 1e-11


def test_patch_test_trilinear():
    """P5 on perturbed trilinear meshes: linear p is reproduced exactly."""
    coef = np.zeros((3, 3, 3))
    coef[0, 0, 0], coef[1, 0, 0], coef[0, 1, 0], coef[0, 0, 1] = 0.3, 1.0, -2.0, 0.5
    for k in (1, 2):
        m = O.Mesh(3, 3, 3, k, vertices=I.perturbed_vertices(3, 0.1, seed=5))
        A = O.assemble(m)
        c = coef[: k + 1, : k + 1, : k + 1]
        u = spla.spsolve(A.tocsc(), O.rhs(m, "poly", c))
        assert O.l2_error(m, u, "poly", c) < 1e-11


# ---------------------------------------------------------------- P6 / P7 / P8

@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("bc", [O.DIRICHLET, O.PERIODIC])
def test_kronecker_sum(k, bc):
    """P6: K = 1 on a uniform box mesh, A = M(x)M(x)L + M(x)L(x)M + L(x)M(x)M
    with independently built 1D SWIPDG operators L and masses M."""
    nx, ny, nz = (3, 2, 2) if k <= 3 else (2, 1, 2)
    A = O.assemble(O.Mesh(nx, ny, nz, k, bc=bc)).toarray()
    T = brute.kron_sum_matrix(nx, ny, nz, k, periodic=(bc == O.PERIODIC))
    assert np.max(np.abs(A - T)) <= 1e-13 * np.max(np.abs(A))


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("case", [((2, 1, 1), False), ((2, 2, 1), True), ((1, 2, 2), False),
                                  ((1, 1, 1), True)])
def test_exact_rationals(k, case):
    """P7: exact rational entries for k <= 2 (GLL nodes rational), rational K."""
    (nx, ny, nz), per = case
    E = nx * ny * nz
    Kf = [Fraction(1 + 2 * (e % 3), 1 + (e % 2)) for e in range(E)]
    Ex = brute.exact_matrix(nx, ny, nz, k, periodic=per, K=Kf)
    Exf = np.array([[float(v) for v in r] for r in Ex])
    A = O.assemble(O.Mesh(nx, ny, nz, k, bc=int(per), theta=np.log([float(v) for v in Kf]))).toarray()
    assert np.max(np.abs(A - Exf)) <= 1e-14 * np.max(np.abs(Exf))


@pytest.mark.parametrize("mesh", SMALL_MESHES)
@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("bc", [O.DIRICHLET, O.PERIODIC])
def test_dense_brute_force(mesh, k, bc):
    """P8: independent dense assembly (face loop, omega-weighted average) agrees."""
    th = I.theta(int(np.prod(mesh)), seed=200 + k)
    A = O.assemble(O.Mesh(*mesh, k, bc=bc, theta=th)).toarray()
    D = brute.dense_matrix(*mesh, k, periodic=(bc == O.PERIODIC), theta=th)
    assert np.max(np.abs(A - D)) <= 1e-13 * np.max(np.abs(A))


@pytest.mark.parametrize("k", [1, 2, 3])
def test_dense_brute_force_perturbed(k):
    th = I.theta(8, seed=300 + k)
    V = _pert_222()
    A = O.assemble(O.Mesh(2, 2, 2, k, theta=th, vertices=V)).toarray()
    D = brute.dense_matrix(2, 2, 2, k, theta=th, vertices=V)
    assert np.max(np.abs(A - D)) <= 1e-13 * np.max(np.abs(A))


# ---------------------------------------------------------------- P9 / P11

@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_quadrature_invariance_affine(k):
    """P9: on affine meshes with cellwise-constant K the (k+1)-point rule is exact:
    two more points per direction change nothing."""
    th = I.theta(12, seed=50 + k)
    A = O.assemble(O.Mesh(3, 2, 2, k, theta=th))
    B = O.assemble(O.Mesh(3, 2, 2, k, theta=th, quad_extra=2))
    assert abs(A - B).max() <= 1e-13 * abs(A).max()


def test_translation_invariance():
    """P11: K = 1 on a uniform periodic mesh: every element's block row (its own
    block and the block of each face neighbour, by direction) is the same."""
    N, k = 3, 2
    n3 = (k + 1) ** 3
    A = O.assemble(O.Mesh(N, N, N, k, bc=O.PERIODIC)).tocsr()

    def blocks(e):
        ex, ey, ez = e % N, (e // N) % N, e // (N * N)
        rows = A[e * n3:(e + 1) * n3]
        out = [rows[:, e * n3:(e + 1) * n3].toarray()]
        for d in range(3):
            for s in (-1, 1):
                c = [ex, ey, ez]
                c[d] = (c[d] + s) % N
                nb = c[0] + N * (c[1] + N * c[2])
                out.append(rows[:, nb * n3:(nb + 1) * n3].toarray())
        return np.stack(out)

    ref = blocks(0)
    scale = np.max(np.abs(ref))
    for e in range(1, N ** 3):
        assert np.max(np.abs(blocks(e) - ref)) <= 1e-13 * scale


# ---------------------------------------------------------------- internal consistency

def test_apply_rows_matches_csr():
    N, k = 4, 3
    m = O.Mesh(N, N, N, k, theta=I.theta(N ** 3), vertices=I.perturbed_vertices(N, 0.1, seed=2))
    x = I.uniform_vector(m.ndof, seed=1)
    A = O.assemble(m)
    y = O.spmv(A, x)
    assert np.max(np.abs(y - A @ x)) <= 1e-13 * np.max(np.abs(y))
    el = [0, 5, 21, 63]
    rows = O.apply_rows(m, x, el)
    for i, e in enumerate(el):
        assert np.max(np.abs(rows[i] - y[e * m.n3:(e + 1) * m.n3])) <= 1e-13 * np.max(np.abs(y))


def test_pcg_and_fast_diagonalisation():
    """Alg. PCG (oracle) against a direct solve, and the K = 1 fast-diagonalisation
    solve against a direct solve."""
    N, k = 4, 2
    m = O.Mesh(N, N, N, k, theta=I.theta(N ** 3))
    A = O.assemble(m)
    b = O.rhs(m, "sine")
    x_ref = spla.spsolve(A.tocsc(), b)
    for jac in (True, False):
        x, it, rr = O.pcg(A, b, rtol=1e-12, jacobi=jac)
        assert rr <= 1e-11 and it > 0
        assert np.linalg.norm(x - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
    m1 = O.Mesh(N, 3, 2, k)
    A1 = O.assemble(m1)
    b1 = I.uniform_vector(m1.ndof, seed=4)
    x1 = O.fast_diag_solve(N, 3, 2, k, O.DIRICHLET, b1)
    x1_ref = spla.spsolve(A1.tocsc(), b1)
    assert np.linalg.norm(x1 - x1_ref) <= 1e-11 * np.linalg.norm(x1_ref)


def test_workload_inputs_shapes():
    V = I.perturbed_vertices(4, 0.1)
    assert V.shape == (125, 3)
    U = I.uniform_vertices(4, 4, 4)
    d = np.abs(V - U)
    assert d.max() <= 0.1 / 4 + 1e-15
    bnd = (U == 0.0) | (U == 1.0)
    assert np.all(d[bnd.any(axis=1)] == 0.0)
    b = I.to_bf16_bits(np.array([1.0, -2.5, 1.00390625, 1.005859375, 3.0e38]))
    back = I.bf16_bits_to_f64(b)
    assert back[0] == 1.0 and back[1] == -2.5
    assert back[2] == 1.0          # tie 1 + 2^-8 rounds to even (1.0)
    assert back[3] == 1.0078125    # above the tie rounds up
