"""Multi-vector apply Y = A X (dg_apply_multi, the multiple right-hand sides of
Sec. 3.5's block Krylov methods): every vector of Y bit-identical to the
single-vector apply of the same precision (same kernels and arithmetic), the
FP64 result against the oracle's matrix, the transpose, a trilinear mesh
(one apply per vector) and the argument checks of the C ABI."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1911_01492_amd import dg  # noqa: E402
from paper_1911_01492_amd import inputs as I  # noqa: E402
from paper_1911_01492_amd.dg import DG_ERR_ARG, DGOperator  # noqa: E402
from tests.gpu_util import banner, dev, host, rel_l2  # noqa: E402

CONV = {"f64": lambda v: v, "f32": lambda v: v.float(), "bf16": lambda v: v.float().to(torch.bfloat16),
        "bf16_mfma": lambda v: v.float().to(torch.bfloat16)}


@pytest.mark.parametrize("shape,k,bc,nrhs", [((5, 3, 2), 4, "dirichlet", 3), ((4, 4, 3), 3, "periodic", 3),
                                             ((3, 2, 2), 6, "dirichlet", 3), ((7, 5, 3), 1, "dirichlet", 3),
                                             ((6, 5, 3), 2, "periodic", 4), ((3, 3, 2), 5, "dirichlet", 4),
                                             ((2, 2, 3), 7, "periodic", 3)])
def test_multi_matches_single_applies(shape, k, bc, nrhs):
    banner(f"apply_multi {shape} k={k} {bc} nrhs={nrhs}")
    E = int(np.prod(shape))
    theta = I.theta(E, seed=2)
    op = DGOperator(*shape, k, bc, theta=dev(theta))
    A = O.assemble(O.Mesh(*shape, k, bc=O.PERIODIC if bc == "periodic" else O.DIRICHLET, theta=theta))
    X64 = dev(np.stack([I.uniform_vector(op.ndof, seed=40 + j) for j in range(nrhs)]))
    for prec in ("f64", "f32", "bf16", "bf16_mfma"):
        if prec == "bf16_mfma" and k > 4:
            continue
        X = CONV[prec](X64).contiguous()
        for trans in (False, True):
            Y = op.apply_multi(X, prec=prec, transpose=trans)
            for j in range(nrhs):
                assert torch.equal(Y[j], op.apply(X[j].contiguous(), prec=prec, transpose=trans)), (prec, trans, j)
        if prec == "f64":
            Yh = host(op.apply_multi(X))
            for j in range(nrhs):
                assert rel_l2(Yh[j], A @ host(X64[j])) <= 1e-12


def test_multi_reaction_and_repeats():
    """With a reaction term, and repeated with alternating inputs: every vector
    bit-identical to its single apply each time."""
    shape, k = (6, 4, 3), 4
    banner(f"apply_multi reaction {shape} k={k}")
    E = int(np.prod(shape))
    op = DGOperator(*shape, k, "dirichlet", theta=dev(I.theta(E, seed=5)))
    op.set_reaction(dev(I.reaction(E, seed=6)))
    Xs = [dev(np.stack([I.uniform_vector(op.ndof, seed=70 + 4 * r + j) for j in range(4)])) for r in range(2)]
    for prec in ("f64", "f32", "bf16"):
        Xp = [CONV[prec](X).contiguous() for X in Xs]
        ref = [torch.stack([op.apply(X[j].contiguous(), prec=prec) for j in range(4)]) for X in Xp]
        for r in range(10):
            assert torch.equal(op.apply_multi(Xp[r % 2], prec=prec), ref[r % 2]), (prec, r)


def test_multi_trilinear_and_errors():
    banner("apply_multi trilinear and argument checks")
    from tests.test_gpu_trilinear import box_vertices
    V = box_vertices(4, 3, 3, amp=0.1, seed=3)
    op = DGOperator(4, 3, 3, 2, "dirichlet", theta=dev(I.theta(36)), vertices=dev(V))
    X = dev(np.stack([I.uniform_vector(op.ndof, seed=50 + j) for j in range(2)]))
    Y = op.apply_multi(X)
    for j in range(2):
        assert torch.equal(Y[j], op.apply(X[j].contiguous()))
    # meshes of equal parallelepipeds: one launch, the vector as the second grid dimension
    opp = DGOperator(5, 4, 3, 3, "dirichlet", theta=dev(I.theta(60)), vertices=dev(I.sheared_vertices(5, 4, 3)))
    assert opp.kernel == "parallelepiped"
    for prec, conv in (("f64", lambda v: v), ("f32", lambda v: v.float()),
                       ("bf16", lambda v: v.float().to(torch.bfloat16))):
        Xp = conv(dev(np.stack([I.uniform_vector(opp.ndof, seed=60 + j) for j in range(3)]))).contiguous()
        for trans in (False, True):
            Yp = opp.apply_multi(Xp, prec=prec, transpose=trans)
            for j in range(3):
                assert torch.equal(Yp[j], opp.apply(Xp[j].contiguous(), prec=prec, transpose=trans)), (prec, trans, j)
    L = dg.lib()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for nrhs in (0, -1, 70000):
        assert L.dg_apply_multi(op._h, 0, 0, nrhs, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()), s) \
            == DG_ERR_ARG
    assert L.dg_apply_multi(op._h, 0, 0, 2, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(X[1].data_ptr()), s) \
        == DG_ERR_ARG  # overlapping X and Y
    assert L.dg_apply_multi(op._h, 0, 2, 2, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()), s) \
        == DG_ERR_ARG  # transpose flag
    torch.cuda.synchronize()
