"""Pins of the oracle's block-Jacobi PCG (oracle.block_jacobi_pcg), checked
against what is fixed independently of it:
* blocks of size 1 are the point-Jacobi preconditioner: the iterates after 1
  and 10 steps equal those of the C++ Alg. PCG with Jacobi (oracle.pcg);
* on a block-diagonal SPD matrix the preconditioner is the exact inverse, so
  one step gives the solution;
* on the assembled DG operator with lognormal K it converges to the direct
  solution, in fewer iterations than point Jacobi."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import oracle as O
from paper_1911_01492_amd import inputs as I


def _operator(N=3, k=2, seed=1):
    m = O.Mesh(N, N, N, k, theta=I.theta(N ** 3, seed=seed))
    return m, O.assemble(m)


def test_unit_blocks_are_point_jacobi():
    m, A = _operator()
    b = I.uniform_vector(m.ndof, seed=3)
    for steps in (1, 10):
        x_blk, it_blk, _ = O.block_jacobi_pcg(A, b, 1, rtol=1e-30, maxit=steps)
        x_pt, it_pt, _ = O.pcg(A, b, rtol=1e-30, maxit=steps)
        assert it_blk == it_pt == steps
        assert np.linalg.norm(x_blk - x_pt) <= 1e-12 * np.linalg.norm(x_pt)


def test_block_diagonal_matrix_one_step():
    m, A = _operator(N=2, k=2)
    n3 = m.n3
    A = A.tocoo()
    keep = (A.row // n3) == (A.col // n3)
    Ab = sp.csr_matrix((A.data[keep], (A.row[keep], A.col[keep])), shape=A.shape)
    b = I.uniform_vector(m.ndof, seed=4)
    x, it, res = O.block_jacobi_pcg(Ab, b, n3, rtol=1e-14, maxit=5)
    assert it == 1
    assert res <= 1e-13
    assert np.linalg.norm(x - spla.spsolve(Ab.tocsc(), b)) <= 1e-12 * np.linalg.norm(x)


def test_converges_to_direct_solution_faster_than_point_jacobi():
    m, A = _operator(N=4, k=2, seed=2)
    b = I.uniform_vector(m.ndof, seed=5)
    x, it, res = O.block_jacobi_pcg(A, b, m.n3, rtol=1e-11, maxit=2000)
    x_ref = spla.spsolve(A.tocsc(), b)
    _, it_pt, _ = O.pcg(A, b, rtol=1e-11, maxit=2000)
    assert res <= 1e-11
    assert np.linalg.norm(x - x_ref) <= 1e-8 * np.linalg.norm(x_ref)
    assert it < it_pt
