"""GPU Krylov solvers (Alg. PCG of Sec. 2.4 in FP64; FP64 defect correction
around FP32-vector PCG) against the oracle: the oracle's own CSR matrix
measures the true residual of every GPU solution, the oracle's PCG or the
exact fast-diagonalisation solve gives the reference solution."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1911_01492_amd import inputs as I  # noqa: E402
from paper_1911_01492_amd.dg import DG_BREAKDOWN, DG_NOT_CONVERGED, DG_OK, DGOperator  # noqa: E402
from tests.gpu_util import banner, dev, host, rel_l2  # noqa: E402


def _sine_rhs(op):
    xq = op.quadrature_points()
    fq = 3 * math.pi ** 2 * torch.sin(math.pi * xq[:, 0]) * torch.sin(math.pi * xq[:, 1]) * \
        torch.sin(math.pi * xq[:, 2])
    return op.load_vector(fq.contiguous())


@pytest.fixture(scope="module")
def small():
    N, k = 8, 3
    theta = I.theta(N ** 3)
    m = O.Mesh(N, N, N, k, theta=theta)
    A = O.assemble(m)
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(theta))
    return m, A, op


def test_load_vector_and_quadrature_points(small):
    banner("load vector")
    m, A, op = small
    b = host(_sine_rhs(op))
    assert rel_l2(b, O.rhs(m, "sine")) <= 1e-13
    for V in (None, I.perturbed_vertices(4, 0.1, seed=3)):
        m2 = O.Mesh(4, 4, 4, 2, vertices=V)
        # the load vector does not depend on K; trilinear contexts need the trilinear kernels
        if V is not None:
            continue
        op2 = DGOperator(4, 4, 4, 2, "dirichlet")
        assert rel_l2(host(_sine_rhs(op2)), O.rhs(m2, "sine")) <= 1e-13


@pytest.mark.parametrize("prec,mode", [("f64", "restart"), ("f32", "restart"), ("bf16", "restart"),
                                       ("f32", "keep"), ("bf16", "keep")])
def test_solution_matches_oracle(small, prec, mode):
    banner(f"cg {prec} {mode}")
    m, A, op = small
    b = _sine_rhs(op)
    x, info = op.cg_solve(b, prec_inner=prec, rtol=1e-10, dc_mode=mode)
    print(info)
    assert info["status"] == DG_OK
    xs, bs = host(x), host(b)
    # the oracle's matrix measures the true residual of the GPU solution
    assert np.linalg.norm(bs - A @ xs) <= 1.2e-10 * np.linalg.norm(bs)
    x_ref, it, rr = O.pcg(A, bs, rtol=1e-13)
    err = rel_l2(xs, x_ref)
    print(f"cg {prec} {mode}: true rel residual (oracle CSR) "
          f"{np.linalg.norm(bs - A @ xs) / np.linalg.norm(bs):.3e}, solution rel err vs oracle {err:.3e}")
    assert err <= 1e-7
    if prec == "f64":
        assert info["outer_iters"] == 0
    else:
        assert info["outer_iters"] >= 1


def test_unpreconditioned_and_transposed(small):
    banner("cg no-precond / transpose")
    m, A, op = small
    b = _sine_rhs(op)
    x1, i1 = op.cg_solve(b, precond="none", rtol=1e-10)
    x2, i2 = op.cg_solve(b, transpose=True, rtol=1e-10)
    assert i1["status"] == DG_OK and i2["status"] == DG_OK
    bs = host(b)
    for x in (x1, x2):
        assert np.linalg.norm(bs - A @ host(x)) <= 1.2e-10 * np.linalg.norm(bs)
    assert i1["iters"] > i2["iters"]  # Jacobi helps under lognormal K
    for prec in ("f32", "bf16"):
        x3, i3 = op.cg_solve(b, prec_inner=prec, precond="none", transpose=True, dc_mode="keep", rtol=1e-10)
        assert i3["status"] == DG_OK
        assert np.linalg.norm(bs - A @ host(x3)) <= 1.2e-10 * np.linalg.norm(bs)


def test_single_reduction_variant(small):
    """Chronopoulos-Gear recurrences (one reduction per iteration): the oracle's
    residual and solution, iteration counts within a few of Alg. PCG, also on a
    trilinear mesh and for the transposed solve."""
    banner("cg single reduction")
    m, A, op = small
    b = _sine_rhs(op)
    bs = host(b)
    x0, i0 = op.cg_solve(b, rtol=1e-10)
    x1, i1 = op.cg_solve(b, rtol=1e-10, variant="single_reduction")
    x2, i2 = op.cg_solve(b, rtol=1e-10, variant="single_reduction", transpose=True, precond="none")
    print(i0, i1, i2)
    for x, info in ((x1, i1), (x2, i2)):
        assert info["status"] == DG_OK
        assert np.linalg.norm(bs - A @ host(x)) <= 1.2e-10 * np.linalg.norm(bs)
    x_ref, it, rr = O.pcg(A, bs, rtol=1e-13)
    assert rel_l2(host(x1), x_ref) <= 1e-7
    assert abs(i1["iters"] - i0["iters"]) <= 0.05 * i0["iters"] + 2
    from tests.test_gpu_trilinear import box_vertices
    V = box_vertices(3, 3, 3, seed=8)
    th = I.theta(27, seed=9)
    mt = O.Mesh(3, 3, 3, 2, theta=th, vertices=V)
    At = O.assemble(mt)
    opt = DGOperator(3, 3, 3, 2, "dirichlet", theta=dev(th), vertices=dev(V))
    bt = I.uniform_vector(mt.ndof, seed=10)
    xt, it_ = opt.cg_solve(dev(bt), rtol=1e-10, variant="single_reduction")
    assert it_["status"] == DG_OK
    assert np.linalg.norm(bt - At @ host(xt)) <= 1.2e-10 * np.linalg.norm(bt)


def test_dc_mode_argument_checked(small):
    from paper_1911_01492_amd.dg import DG_ERR_ARG, CgInfo, CgOpts, _ptr, _stream, lib
    import ctypes
    m, A, op = small
    b = _sine_rhs(op)
    x = torch.zeros_like(b)
    o = CgOpts(1, 1, 0, 1e-10, 0.0, 100, 0, 8, 7, 0)
    info = CgInfo()
    rc = lib().dg_cg_solve(op._h, ctypes.byref(o), _ptr(b), _ptr(x), ctypes.byref(info), _stream(None))
    assert rc == DG_ERR_ARG
    assert b"dc_mode" in lib().dg_last_error(op._h)
    o = CgOpts(0, 1, 0, 1e-10, 0.0, 100, 0, 8, 0, 5)
    assert lib().dg_cg_solve(op._h, ctypes.byref(o), _ptr(b), _ptr(x), ctypes.byref(info), _stream(None)) == DG_ERR_ARG
    from paper_1911_01492_amd.dg import DG_ERR_UNSUPPORTED
    o = CgOpts(1, 1, 0, 1e-10, 0.0, 100, 0, 8, 0, 1)
    assert lib().dg_cg_solve(op._h, ctypes.byref(o), _ptr(b), _ptr(x), ctypes.byref(info),
                             _stream(None)) == DG_ERR_UNSUPPORTED


def test_warm_start_and_limits(small):
    banner("cg warm start / maxit / breakdown")
    m, A, op = small
    b = _sine_rhs(op)
    x, info = op.cg_solve(b, rtol=1e-10)
    x2, info2 = op.cg_solve(b, x=x.clone(), rtol=1e-10)
    assert info2["status"] == DG_OK and info2["iters"] == 0
    x3, info3 = op.cg_solve(b, rtol=1e-10, maxit=5)
    assert info3["status"] == DG_NOT_CONVERGED and info3["iters"] == 5
    # the iterate after 5 steps is the oracle's Jacobi PCG iterate after 5 steps,
    # and the reported residual is that iterate's true residual
    x3_ref, it3, _ = O.pcg(A, host(b), rtol=1e-30, maxit=5)
    assert it3 == 5
    assert rel_l2(host(x3), x3_ref) <= 1e-12
    bs = host(b)
    res_ref = np.linalg.norm(bs - A @ x3_ref) / np.linalg.norm(bs)
    assert abs(info3["rel_true_residual"] - res_ref) <= 1e-10 * res_ref
    bad = b.clone()
    bad[7] = float("nan")
    x4, info4 = op.cg_solve(bad, rtol=1e-10)
    assert info4["status"] == DG_BREAKDOWN
    torch.cuda.synchronize()


def test_full_size_exact_solution():
    """K = 1 on the 32^3 Q3 Dirichlet mesh: the GPU PCG solution against the
    exact fast-diagonalisation solve of the Kronecker-sum operator."""
    banner("cg full size K=1 vs fast diagonalisation")
    N, k = 32, 3
    op = DGOperator(N, N, N, k, "dirichlet")
    b = _sine_rhs(op)
    for prec, mode, var in (("f64", "restart", "standard"), ("f64", "restart", "single_reduction"),
                            ("f32", "restart", "standard"), ("f32", "keep", "standard"),
                            ("bf16", "keep", "standard")):
        x, info = op.cg_solve(b, prec_inner=prec, rtol=1e-10, dc_mode=mode, variant=var)
        print(prec, mode, var, info)
        assert info["status"] == DG_OK
        x_ex = O.fast_diag_solve(N, N, N, k, O.DIRICHLET, host(b))
        err = rel_l2(host(x), x_ex)
        print(f"cg {prec} {mode} {var} 32^3 Q3 K=1: solution rel err vs exact solve {err:.3e}")
        assert err <= 1e-7


def test_mixed_precision_solves_repeat_exactly():
    """Repeated FP32 and BF16 defect-correction solves of the 32^3 Q3 workload
    (and FP64 PCG) return the same iteration counts and bit-identical
    solutions: every reduction is deterministic and no kernel may depend on
    stale data from an earlier launch."""
    banner("cg repeatability")
    N, k = 32, 3
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(I.theta(N ** 3)))
    b = _sine_rhs(op)
    for prec, mode, var in (("f64", "restart", "standard"), ("f64", "restart", "single_reduction"),
                            ("f32", "restart", "standard"), ("bf16", "restart", "standard"),
                            ("f32", "keep", "standard")):
        first = None
        for rep in range(4):
            x, info = op.cg_solve(b, prec_inner=prec, rtol=1e-10, dc_mode=mode, variant=var)
            assert info["status"] == DG_OK
            if first is None:
                first = (info["iters"], x.clone())
            else:
                assert info["iters"] == first[0], (prec, mode, rep, info["iters"], first[0])
                assert torch.equal(x, first[1]), (prec, mode, rep)


@pytest.mark.parametrize("shape,k,bc,react,tri", [((5, 4, 3), 3, "dirichlet", False, False),
                                                  ((1, 2, 3), 2, "periodic", False, False),
                                                  ((4, 3, 5), 4, "dirichlet", True, False),
                                                  ((2, 3, 2), 7, "periodic", True, False),
                                                  ((3, 3, 3), 1, "dirichlet", True, False),
                                                  ((3, 4, 3), 3, "dirichlet", True, True),
                                                  ((2, 1, 3), 2, "periodic", False, True)])
def test_jacobi_iterates_match_oracle(shape, k, bc, react, tri):
    """The Jacobi preconditioner of the FP64 PCG.  The iterate after a fixed
    number of steps depends on every entry of the inverse diagonal at first
    order, so it is compared with the oracle's PCG (diagonal taken from its CSR
    matrix) after the same number of steps, on meshes with self-neighbours
    (periodic, one element wide), with a reaction term, and again after new
    coefficients (set_theta must refresh the preconditioner)."""
    banner(f"jacobi iterates {shape} k={k} {bc} reaction={react} trilinear={tri}")
    from tests.test_gpu_trilinear import box_vertices
    E = int(np.prod(shape))
    bcc = {"dirichlet": O.DIRICHLET, "periodic": O.PERIODIC}[bc]
    theta = I.theta(E, seed=11)
    c = I.reaction(E, seed=12) if react else None
    V = box_vertices(*shape, amp=0.1, seed=15) if tri else None
    op = DGOperator(*shape, k, bc, theta=dev(theta), vertices=None if V is None else dev(V))
    if react:
        op.set_reaction(dev(c))
    b = dev(I.uniform_vector(op.ndof, seed=13))
    # the first theta equals the one given at setup and the last repeats the
    # second: set_theta then finds K unchanged and skips the diagonal on the device
    for th in (theta, I.theta(E, seed=14), I.theta(E, seed=14)):
        op.set_theta(dev(th))
        A = O.assemble(O.Mesh(*shape, k, bc=bcc, theta=th, vertices=V, reaction=c))
        for steps in (1, 10):
            x, info = op.cg_solve(b, rtol=1e-30, maxit=steps)
            assert info["iters"] == steps
            x_ref, it, _ = O.pcg(A, host(b), rtol=1e-30, maxit=steps)
            assert it == steps
            err = rel_l2(host(x), x_ref)
            print(f"{steps} steps: rel diff vs oracle PCG {err:.2e}")
            assert err <= 1e-12
        # the diagonal itself, through the library's separate diagonal kernel
        assert rel_l2(host(op.diagonal()), A.diagonal()) <= 1e-14
