"""Element block-Jacobi PCG (precond "block_jacobi": exact element-block
inverses by fast diagonalisation on axis-parallel box elements) against the
oracle's Alg. PCG with exact element-block inverses taken from its assembled
CSR matrix (oracle.block_jacobi_pcg): iterates after a fixed number of steps
(they depend on every entry of the block inverses at first order), the
converged solution with the true residual measured by the oracle's matrix,
the iteration count against point Jacobi, and the refusals."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1911_01492_amd import inputs as I  # noqa: E402
from paper_1911_01492_amd.dg import DG_ERR_UNSUPPORTED, DGError, DGOperator  # noqa: E402
from tests.gpu_util import banner, dev, host, rel_l2  # noqa: E402


@pytest.mark.parametrize("shape,k,bc,react", [((3, 3, 3), 2, "dirichlet", False), ((4, 3, 2), 3, "dirichlet", True),
                                              ((2, 2, 3), 4, "periodic", False), ((3, 2, 2), 1, "dirichlet", False),
                                              ((2, 2, 2), 5, "dirichlet", True), ((2, 1, 2), 6, "dirichlet", False)])
def test_block_jacobi_iterates_match_oracle(shape, k, bc, react):
    banner(f"block-jacobi iterates {shape} k={k} {bc} reaction={react}")
    E = int(np.prod(shape))
    bcc = {"dirichlet": O.DIRICHLET, "periodic": O.PERIODIC}[bc]
    c = I.reaction(E, seed=12) if react else None
    theta = I.theta(E, seed=11)
    op = DGOperator(*shape, k, bc, theta=dev(theta))
    if react:
        op.set_reaction(dev(c))
    b = I.uniform_vector(op.ndof, seed=13)
    for th in (theta, I.theta(E, seed=14)):  # new coefficients must refresh the factors
        op.set_theta(dev(th))
        m = O.Mesh(*shape, k, bc=bcc, theta=th, reaction=c)
        A = O.assemble(m)
        for steps in (1, 10):
            x, info = op.cg_solve(dev(b), precond="block_jacobi", rtol=1e-30, maxit=steps)
            assert info["iters"] == steps
            x_ref, it, _ = O.block_jacobi_pcg(A, b, m.n3, rtol=1e-30, maxit=steps)
            assert it == steps
            err = rel_l2(host(x), x_ref)
            print(f"{steps} steps: rel diff vs oracle block-Jacobi PCG {err:.2e}")
            assert err <= 1e-12


def test_block_jacobi_solve_and_iterations():
    """8^3 Q3 lognormal K: converges to the oracle's solution with a true
    residual <= 1e-10 (oracle CSR), in fewer iterations than point Jacobi, and
    the transposed solve agrees (the form is symmetric)."""
    N, k = 8, 3
    banner("block-jacobi solve 8^3 Q3")
    theta = I.theta(N ** 3)
    m = O.Mesh(N, N, N, k, theta=theta)
    A = O.assemble(m)
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(theta))
    b = I.uniform_vector(m.ndof, seed=I.S_B)
    u, info = op.cg_solve(dev(b), precond="block_jacobi", rtol=1e-10)
    res = np.linalg.norm(b - A @ host(u)) / np.linalg.norm(b)
    _, info_j = op.cg_solve(dev(b), precond="jacobi", rtol=1e-10)
    x_ref, it_ref, _ = O.block_jacobi_pcg(A, b, m.n3, rtol=1e-10, maxit=5000)
    print(f"block-jacobi {info['iters']} it (oracle {it_ref}), jacobi {info_j['iters']} it; true residual {res:.2e}")
    assert info["status"] == 0 and res <= 1.2e-10
    assert rel_l2(host(u), x_ref) <= 1e-8
    assert abs(info["iters"] - it_ref) <= 2
    assert info["iters"] < info_j["iters"]
    ut, info_t = op.cg_solve(dev(b), precond="block_jacobi", rtol=1e-10, transpose=True)
    assert info_t["status"] == 0 and rel_l2(host(ut), host(u)) <= 1e-8


@pytest.mark.parametrize("prec,mode", [("f32", "restart"), ("f32", "keep"), ("bf16", "restart"), ("bf16", "keep"),
                                       ("bf16_mfma", "keep")])
def test_block_jacobi_defect_correction(prec, mode):
    """FP64 defect correction whose FP32-vector inner PCG uses the block
    preconditioner (FP32 factors): true residual <= 1e-10 with the oracle's
    matrix, the solution of the FP64 block-Jacobi PCG, fewer inner iterations
    than with point Jacobi."""
    N, k = 8, 3
    banner(f"block-jacobi defect correction {prec} {mode}")
    theta = I.theta(N ** 3)
    m = O.Mesh(N, N, N, k, theta=theta)
    A = O.assemble(m)
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(theta))
    b = I.uniform_vector(m.ndof, seed=I.S_B)
    u, info = op.cg_solve(dev(b), prec_inner=prec, dc_mode=mode, precond="block_jacobi", rtol=1e-10)
    res = np.linalg.norm(b - A @ host(u)) / np.linalg.norm(b)
    u64, _ = op.cg_solve(dev(b), precond="block_jacobi", rtol=1e-12)
    _, info_j = op.cg_solve(dev(b), prec_inner=prec, dc_mode=mode, precond="jacobi", rtol=1e-10)
    print(f"{prec} {mode}: block {info['iters']} it / {info['outer_iters']} outer, jacobi {info_j['iters']} it; "
          f"true residual {res:.2e}")
    assert info["status"] == 0 and res <= 1.2e-10
    assert rel_l2(host(u), host(u64)) <= 1e-8
    assert info["iters"] < info_j["iters"]


def test_block_jacobi_refusals():
    banner("block-jacobi refusals")
    op = DGOperator(3, 3, 3, 2, "dirichlet", theta=dev(I.theta(27)))
    b = dev(I.uniform_vector(op.ndof))
    for kw in ({"variant": "single_reduction"},):
        with pytest.raises(DGError) as ei:
            op.cg_solve(b, precond="block_jacobi", **kw)
        assert ei.value.code == DG_ERR_UNSUPPORTED
    tri = DGOperator(3, 3, 3, 2, "dirichlet", vertices=dev(I.perturbed_vertices(3)))
    with pytest.raises(DGError) as ei:
        tri.cg_solve(dev(I.uniform_vector(tri.ndof)), precond="block_jacobi")
    assert ei.value.code == DG_ERR_UNSUPPORTED


def test_block_jacobi_repeatable():
    """Solves that alternate between two right-hand sides give bit-identical
    solutions and iteration counts for the same right-hand side (FP64 PCG and
    the FP32 keep-mode defect correction, 12^3 Q4: an element's 25 threads
    span two wavefronts of the block-apply kernel)."""
    N, k = 12, 4
    banner("block-jacobi repeatability 12^3 Q4")
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(I.theta(N ** 3, seed=40)))
    bs = [dev(I.uniform_vector(op.ndof, seed=s)) for s in (41, 42)]
    for prec, mode in (("f64", "restart"), ("f32", "keep")):
        ref = [op.cg_solve(b, prec_inner=prec, dc_mode=mode, precond="block_jacobi", rtol=1e-10) for b in bs]
        ref = [(u.clone(), info["iters"]) for u, info in ref]
        for r in range(6):
            u, info = op.cg_solve(bs[r % 2], prec_inner=prec, dc_mode=mode, precond="block_jacobi", rtol=1e-10)
            assert info["iters"] == ref[r % 2][1] and torch.equal(u, ref[r % 2][0]), (prec, r)


def test_block_jacobi_many_partials():
    """48^3 Q3 (6912 bricks: more apply partials than the fused form takes,
    so the solve runs the finish kernels): FP64 and FP32 keep-mode
    block-Jacobi solves reach the tolerance, agree with the point-Jacobi FP64
    solution and take fewer iterations."""
    N, k = 48, 3
    banner("block-jacobi 48^3 Q3 (finish-kernel path)")
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(I.theta(N ** 3)))
    b = dev(I.uniform_vector(op.ndof, seed=I.S_B))
    u_pj, info_pj = op.cg_solve(b, rtol=1e-10)
    assert info_pj["status"] == 0
    for prec, mode in (("f64", "restart"), ("f32", "keep")):
        u, info = op.cg_solve(b, prec_inner=prec, dc_mode=mode, precond="block_jacobi", rtol=1e-10)
        print(prec, info, "point Jacobi", info_pj["iters"])
        assert info["status"] == 0 and info["rel_true_residual"] <= 1.2e-10
        assert info["iters"] < info_pj["iters"]
        assert float((u - u_pj).norm() / u_pj.norm()) <= 1e-7
