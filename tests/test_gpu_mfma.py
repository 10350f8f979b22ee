"""BF16-input apply on affine meshes through the matrix-core kernel (precision
bf16_mfma: tangential masses M (x) M on MFMA with exact BF16 plane operands and
a three-term BF16 split of the matrix, FP32 accumulation; degrees 1..4): element by element
against the oracle's assembled matrix.  The arithmetic error (against A x_hat,
x_hat the BF16 input the kernel received) has the FP32 bound of the other
low-precision tests; the total error (against A x) is dominated by the input
rounding 2^-9.  Meshes cover ragged bricks, periodic wrap inside one brick,
elements that are their own neighbours, and the reaction term."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1911_01492_amd import inputs as I  # noqa: E402
from paper_1911_01492_amd.dg import DG_ERR_UNSUPPORTED, DGError, DGOperator  # noqa: E402
from tests.gpu_util import banner, bf16_dev, dev, host, rel_l2  # noqa: E402

MESHES = [(1, 1, 1), (2, 1, 1), (2, 2, 2), (3, 2, 2), (5, 3, 2), (6, 4, 3), (7, 3, 2), (9, 5, 4)]


def _check(shape, k, bc, seed, reaction=False):
    E = int(np.prod(shape))
    theta = I.theta(E, seed=seed)
    c = I.reaction(E) if reaction else None
    m = O.Mesh(*shape, k, bc=O.PERIODIC if bc == "periodic" else O.DIRICHLET, theta=theta, reaction=c)
    op = DGOperator(*shape, k, bc, theta=dev(theta))
    if reaction:
        op.set_reaction(dev(c))
    A = O.assemble(m)
    x = I.uniform_vector(m.ndof, seed=seed + 1)
    bits = I.to_bf16_bits(x)
    xh = I.bf16_bits_to_f64(bits)
    y = host(op.apply(bf16_dev(bits), prec="bf16_mfma"))
    e_arith = rel_l2(y, A @ xh)
    e_total = rel_l2(y, A @ x)
    return e_arith, e_total


@pytest.mark.parametrize("k", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", ["dirichlet", "periodic"])
def test_bf16_mfma_meshes(k, bc):
    worst = 0.0
    for shape in MESHES:
        banner(f"bf16 mfma apply {shape} k={k} {bc}")
        e_arith, e_total = _check(shape, k, bc, seed=10 * k + len(shape))
        worst = max(worst, e_arith)
        assert e_arith <= 2e-5, (shape, k, bc, e_arith)
        assert e_total <= 2e-2, (shape, k, bc, e_total)
    print(f"bf16 mfma k={k} {bc}: worst arithmetic error {worst:.3e}")


@pytest.mark.parametrize("k", [1, 4])
def test_bf16_mfma_reaction(k):
    banner(f"bf16 mfma apply with reaction k={k}")
    e_arith, e_total = _check((5, 3, 2), k, "dirichlet", seed=3, reaction=True)
    assert e_arith <= 2e-5 and e_total <= 2e-2


def test_bf16_mfma_rows_q4_64():
    """The 64^3 Q4 launch: sampled element rows against the oracle, and the
    result bit-identical over repeated launches."""
    N, k = 64, 4
    banner("bf16 mfma apply 64^3 Q4 sampled rows")
    theta = I.theta(N ** 3)
    m = O.Mesh(N, N, N, k, theta=theta)
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(theta))
    x = I.uniform_vector(m.ndof)
    bits = I.to_bf16_bits(x)
    X = bf16_dev(bits)
    xh = I.bf16_bits_to_f64(bits)
    del bits
    el = np.unique(np.r_[0, N - 1, N ** 3 - 1, N ** 3 // 2 + 7,
                         np.random.default_rng(5).choice(N ** 3, 8, replace=False)]).astype(np.int64)
    y = op.apply(X, prec="bf16_mfma")
    got = host(y.view(-1, m.n3)[torch.as_tensor(el, device="cuda")])
    e_arith = rel_l2(got, O.apply_rows(m, xh, el))
    e_total = rel_l2(got, O.apply_rows(m, x, el))
    print(f"bf16 mfma 64^3 Q4 sampled rows: arithmetic {e_arith:.3e} total {e_total:.3e}")
    assert e_arith <= 2e-5 and e_total <= 2e-2
    y1 = y.clone()
    for _ in range(5):
        assert torch.equal(op.apply(X, prec="bf16_mfma"), y1)
    del X, y, y1
    torch.cuda.empty_cache()


def test_bf16_mfma_transpose_and_solver():
    """The transposed apply is the same product (symmetric form); the FP64
    defect correction with bf16_mfma inner solves reaches the FP64 tolerance
    (true residual with the oracle's matrix) and agrees with the VALU BF16 path's
    solution; trilinear meshes and k > 4 are refused."""
    N, k = 6, 3
    banner("bf16 mfma transpose and defect-correction CG")
    theta = I.theta(N ** 3)
    m = O.Mesh(N, N, N, k, theta=theta)
    A = O.assemble(m)
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(theta))
    X = bf16_dev(I.to_bf16_bits(I.uniform_vector(m.ndof, seed=4)))
    assert torch.equal(op.apply(X, prec="bf16_mfma", transpose=True), op.apply(X, prec="bf16_mfma"))
    b = I.uniform_vector(m.ndof, seed=I.S_B)
    for mode in ("restart", "keep"):
        u, info = op.cg_solve(dev(b), prec_inner="bf16_mfma", dc_mode=mode, rtol=1e-10)
        res = np.linalg.norm(b - A @ host(u)) / np.linalg.norm(b)
        u2, _ = op.cg_solve(dev(b), prec_inner="bf16", dc_mode=mode, rtol=1e-10)
        print(f"bf16_mfma DC-CG {mode}: {info}, true residual {res:.2e}")
        assert info["status"] == 0 and res <= 1.2e-10
        assert rel_l2(host(u), host(u2)) <= 1e-8
    tri = DGOperator(3, 3, 3, 2, "dirichlet", vertices=dev(I.perturbed_vertices(3)))
    with pytest.raises(DGError) as ei:
        tri.apply(bf16_dev(I.to_bf16_bits(np.ones(tri.ndof))), prec="bf16_mfma")
    assert ei.value.code == DG_ERR_UNSUPPORTED
    hi = DGOperator(2, 2, 2, 5, "dirichlet")
    with pytest.raises(DGError) as ei:
        hi.apply(bf16_dev(I.to_bf16_bits(np.ones(hi.ndof))), prec="bf16_mfma")
    assert ei.value.code == DG_ERR_UNSUPPORTED
