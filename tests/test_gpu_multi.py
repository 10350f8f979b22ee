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


@pytest.mark.parametrize("shape,k,bc", [((5, 3, 2), 4, "dirichlet"), ((4, 4, 3), 3, "periodic"),
                                        ((3, 2, 2), 6, "dirichlet"), ((7, 5, 3), 1, "dirichlet")])
def test_multi_matches_single_applies(shape, k, bc):
    banner(f"apply_multi {shape} k={k} {bc}")
    E = int(np.prod(shape))
    theta = I.theta(E, seed=2)
    op = DGOperator(*shape, k, bc, theta=dev(theta))
    A = O.assemble(O.Mesh(*shape, k, bc=O.PERIODIC if bc == "periodic" else O.DIRICHLET, theta=theta))
    nrhs = 3
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
