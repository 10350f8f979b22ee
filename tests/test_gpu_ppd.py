"""GPU parity of the constant-metric apply on meshes of equal
parallelepipeds (problem B of Sec. 3.3: the grid under one affine map)
against the CPU oracle, which evaluates the same form by brute force with
each element's Jacobian from its own vertices."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1911_01492_amd import inputs as I  # noqa: E402
from paper_1911_01492_amd.dg import DG_OK, DGOperator  # noqa: E402
from tests.gpu_util import banner, bf16_dev, dev, host, rel_l2  # noqa: E402

BCS = {"dirichlet": O.DIRICHLET, "periodic": O.PERIODIC}
# a general affine map: rotation-like mixing of all three axes and shear
A3 = np.array([[1.0, 0.3, -0.2], [0.1, 0.9, 0.25], [-0.15, 0.2, 1.1]])


def affine_vertices(nx, ny, nz):
    return I.uniform_vertices(nx, ny, nz) @ A3.T


def _case(shape, k, bc, V, seed=0, reaction=False):
    E = int(np.prod(shape))
    theta = I.theta(E, seed=seed + 1)
    R = I.reaction(E, seed=seed + 2) if reaction else None
    m = O.Mesh(*shape, k, bc=BCS[bc], theta=theta, vertices=V, reaction=R)
    op = DGOperator(*shape, k, bc, theta=dev(theta), vertices=dev(V))
    if reaction:
        op.set_reaction(dev(R))
    assert op.kernel == "parallelepiped", (shape, k, bc)
    return m, op, I.uniform_vector(m.ndof, seed=seed)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("bc", ["dirichlet", "periodic"])
def test_small_sheared(k, bc):
    for shape in ([(2, 2, 2), (3, 2, 2)] if k <= 4 else [(2, 2, 2)]):
        banner(f"parallelepiped sheared {shape} k={k} {bc}")
        m, op, x = _case(shape, k, bc, I.sheared_vertices(*shape), seed=k)
        assert rel_l2(host(op.apply(dev(x))), O.assemble(m) @ x) <= 1e-12, (shape, k, bc)


@pytest.mark.parametrize("k", [1, 3, 4, 7])
@pytest.mark.parametrize("bc", ["dirichlet", "periodic"])
def test_general_affine_map_with_reaction(k, bc):
    shape = (3, 2, 2) if k <= 4 else (2, 2, 1)
    banner(f"parallelepiped affine map {shape} k={k} {bc} with reaction")
    m, op, x = _case(shape, k, bc, affine_vertices(*shape), seed=10 + k, reaction=True)
    assert rel_l2(host(op.apply(dev(x))), O.assemble(m) @ x) <= 1e-12, (k, bc)


@pytest.mark.parametrize("shape,k", [((7, 5, 3), 3), ((6, 5, 4), 2), ((5, 3, 3), 4), ((6, 4, 2), 5),
                                     ((9, 7, 6), 1)])
def test_ragged_bricks(shape, k):
    """Meshes spanning several bricks with ragged tails in every direction."""
    banner(f"parallelepiped ragged {shape} k={k}")
    m, op, x = _case(shape, k, "dirichlet", I.sheared_vertices(*shape), seed=3)
    assert rel_l2(host(op.apply(dev(x))), O.assemble(m) @ x) <= 1e-12


@pytest.mark.parametrize("shape", [(1, 2, 3), (2, 1, 1), (1, 1, 1)])
@pytest.mark.parametrize("k", [2, 4])
def test_periodic_self_neighbour(shape, k):
    """One element wide along some axes: the element is its own neighbour."""
    banner(f"parallelepiped periodic self-neighbour {shape} k={k}")
    m, op, x = _case(shape, k, "periodic", affine_vertices(*shape), seed=4)
    assert rel_l2(host(op.apply(dev(x))), O.assemble(m) @ x) <= 1e-12


def test_transpose_low_precision_and_diagonal():
    """The transpose is the same operator; FP32 and BF16-in applies within the
    unit-roundoff bars of the other kernels (arithmetic error against the
    oracle applied to the rounded input, total error against the FP64 input)."""
    shape, k = (4, 3, 3), 3
    banner("parallelepiped transpose / fp32 / bf16")
    m, op, x = _case(shape, k, "dirichlet", I.sheared_vertices(*shape), seed=6)
    A = O.assemble(m)
    y = A @ x
    assert rel_l2(host(op.apply(dev(x), transpose=True)), A.T @ x) <= 1e-12
    x32 = I.to_f32(x).astype(np.float64)
    y32 = host(op.apply(dev(I.to_f32(x), torch.float32), prec="f32").double())
    assert rel_l2(y32, A @ x32) <= 2e-5
    bits = I.to_bf16_bits(x)
    xb = I.bf16_bits_to_f64(bits)
    yb = host(op.apply(bf16_dev(bits), prec="bf16").double())
    e_ar, e_tot = rel_l2(yb, A @ xb), rel_l2(yb, y)
    print(f"parallelepiped bf16 arithmetic err {e_ar:.3e}, total err {e_tot:.3e}")
    assert e_ar <= 2e-5 and e_tot <= 2e-2
    assert rel_l2(host(op.diagonal()), A.diagonal()) <= 1e-13


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6])
def test_low_precision_degrees(k):
    """FP32 and BF16-in applies against the oracle at the degrees whose LDS
    layout or row placement differs between precisions (the z-face rows in
    the face-scalar slot at FP32 n = 2, 4, 5 and FP64 n = 2, 3, 4, 7)."""
    shape = (4, 3, 3) if k <= 4 else (3, 2, 2)
    banner(f"parallelepiped fp32 / bf16 {shape} k={k}")
    m, op, x = _case(shape, k, "dirichlet", affine_vertices(*shape), seed=40 + k, reaction=True)
    A = O.assemble(m)
    assert rel_l2(host(op.apply(dev(x))), A @ x) <= 1e-12
    x32 = I.to_f32(x).astype(np.float64)
    y32 = host(op.apply(dev(I.to_f32(x), torch.float32), prec="f32").double())
    assert rel_l2(y32, A @ x32) <= 2e-5
    bits = I.to_bf16_bits(x)
    yb = host(op.apply(bf16_dev(bits), prec="bf16").double())
    assert rel_l2(yb, A @ I.bf16_bits_to_f64(bits)) <= 2e-5


def test_layered_shear_takes_the_general_kernel():
    """Parallelepipeds that differ from layer to layer are not one affine image
    of the grid: setup keeps the trilinear kernel, still exact."""
    shape, k = (3, 4, 2), 3
    banner("layered shear (trilinear kernel)")
    V = I.layered_shear_vertices(*shape)
    theta = I.theta(int(np.prod(shape)), seed=8)
    m = O.Mesh(*shape, k, theta=theta, vertices=V)
    op = DGOperator(*shape, k, "dirichlet", theta=dev(theta), vertices=dev(V))
    assert op.kernel == "trilinear"
    x = I.uniform_vector(m.ndof, seed=8)
    assert rel_l2(host(op.apply(dev(x))), O.assemble(m) @ x) <= 1e-12
    assert DGOperator(2, 2, 2, 1).kernel == "affine"


@pytest.mark.parametrize("prec,mode", [("f64", "restart"), ("f32", "keep"), ("bf16", "keep")])
def test_solvers(prec, mode):
    shape, k = (5, 4, 4), 3
    banner(f"parallelepiped cg {prec} {mode}")
    m, op, _ = _case(shape, k, "dirichlet", I.sheared_vertices(*shape), seed=30)
    A = O.assemble(m)
    b = I.uniform_vector(m.ndof, seed=I.S_B)
    u, info = op.cg_solve(dev(b), prec_inner=prec, dc_mode=mode, rtol=1e-10)
    print(info)
    assert info["status"] == DG_OK
    assert np.linalg.norm(b - A @ host(u)) <= 1.2e-10 * np.linalg.norm(b)


def test_jacobi_iterates_match_oracle():
    """FP64 PCG iterates after 1 and 10 steps equal the oracle's PCG on the same
    matrix (the fused <p, A p> of the parallelepiped kernel feeds the step)."""
    shape, k = (4, 3, 3), 2
    banner("parallelepiped pcg iterates")
    m, op, _ = _case(shape, k, "dirichlet", affine_vertices(*shape), seed=31)
    A = O.assemble(m)
    b = I.uniform_vector(m.ndof, seed=I.S_B)
    for steps in (1, 10):
        u, info = op.cg_solve(dev(b), rtol=1e-30, maxit=steps)
        assert info["iters"] == steps
        ref, it, _ = O.pcg(A, b, rtol=1e-30, maxit=steps)
        assert it == steps
        assert rel_l2(host(u), ref) <= 1e-12, steps


def test_paper_table_size_sampled_rows():
    """40^3 Q3 sheared (4.1M DOF, the size of the operator-throughput table):
    sampled element rows by the oracle, FP64 and FP32."""
    N, k = 40, 3
    banner("parallelepiped 40^3 Q3 sampled rows")
    theta = I.theta(N ** 3)
    V = I.sheared_vertices(N, N, N)
    m = O.Mesh(N, N, N, k, theta=theta, vertices=V)
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(theta), vertices=dev(V))
    assert op.kernel == "parallelepiped"
    x = I.uniform_vector(m.ndof)
    y = host(op.apply(dev(x)))
    el = np.array([0, N - 1, N ** 3 - 1, (N // 2) * (1 + N + N * N), 12345, 40000, 63999], dtype=np.int64)
    ref = O.apply_rows(m, x, el)
    e64 = rel_l2(y.reshape(-1, m.n3)[el], ref)
    print(f"fp64 parallelepiped 40^3 Q3 sampled rows: rel err {e64:.3e}")
    assert e64 <= 1e-12
    y32 = host(op.apply(dev(I.to_f32(x), torch.float32), prec="f32").double())
    e32 = rel_l2(y32.reshape(-1, m.n3)[el], ref)
    print(f"fp32 parallelepiped sampled rows {e32:.3e}")
    assert e32 <= 1e-4
