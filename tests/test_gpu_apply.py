"""GPU parity of the sum-factorised apply (affine elements) against the CPU
oracle: element by element on the same seeded inputs.  FP64 bar: relative
l2 error <= 1e-12 (the stated target); FP32 / BF16 errors against the FP64
oracle are checked against bounds derived from the unit roundoff."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1911_01492_amd import inputs as I  # noqa: E402
from paper_1911_01492_amd.dg import DGError, DGOperator  # noqa: E402
from tests.gpu_util import banner, bf16_dev, dev, host, rel_l2  # noqa: E402

BCS = {"dirichlet": O.DIRICHLET, "periodic": O.PERIODIC}


def _case(nx, ny, nz, k, bc, seed=0, lognormal=True):
    E = nx * ny * nz
    theta = I.theta(E, seed=seed + 1) if lognormal else None
    m = O.Mesh(nx, ny, nz, k, bc=BCS[bc], theta=theta)
    op = DGOperator(nx, ny, nz, k, bc, theta=None if theta is None else dev(theta))
    x = I.uniform_vector(m.ndof, seed=seed)
    return m, op, x


def test_periodic_q2_4_workload():
    """4^3 periodic Q2, K = 1: full-matrix parity and A 1 = 0."""
    banner("apply periodic_q2_4")
    m, op, x = _case(4, 4, 4, 2, "periodic", lognormal=False)
    A = O.assemble(m)
    y = host(op.apply(dev(x)))
    assert rel_l2(y, A @ x) <= 1e-12
    one = host(op.apply(dev(np.ones(m.ndof))))
    assert np.abs(one).max() <= 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("bc", ["dirichlet", "periodic"])
def test_small_meshes_all_degrees(k, bc):
    for mesh in [(1, 1, 1), (2, 1, 1), (2, 2, 1), (2, 2, 2)]:
        if k >= 6 and mesh == (2, 2, 2):
            continue
        banner(f"apply {mesh} k={k} {bc}")
        m, op, x = _case(*mesh, k, bc, seed=k)
        A = O.assemble(m)
        y = host(op.apply(dev(x)))
        err = rel_l2(y, A @ x)
        print(f"fp64 apply {mesh} k={k} {bc}: rel err {err:.3e}")
        assert err <= 1e-12, (mesh, k, bc)


@pytest.mark.parametrize("shape,k", [((7, 5, 3), 3), ((6, 6, 5), 4), ((9, 4, 3), 2), ((5, 3, 4), 1),
                                     ((3, 4, 3), 5), ((3, 2, 3), 6), ((2, 3, 2), 7)])
@pytest.mark.parametrize("bc", ["dirichlet", "periodic"])
def test_ragged_meshes(shape, k, bc):
    """Several element tiles per launch with a ragged last tile."""
    banner(f"apply ragged {shape} k={k} {bc}")
    m, op, x = _case(*shape, k, bc, seed=3)
    A = O.assemble(m)
    y = host(op.apply(dev(x)))
    assert rel_l2(y, A @ x) <= 1e-12


def _sample_elements(N, extra_seed=0):
    E = N ** 3
    corners = [0, N - 1, N * (N - 1), N * N - 1, E - N * N, E - 1, E // 2 + N // 2]
    rnd = np.random.default_rng(100 + extra_seed).choice(E, 9, replace=False)
    return np.unique(np.r_[corners, rnd]).astype(np.int64)


@pytest.mark.parametrize("wl", ["dirichlet_q3_32", "mixed_q4_64"])
def test_full_size_sampled_rows(wl):
    """Full-size workloads (the benchmark's launch configuration): sampled element
    rows computed by the oracle one by one."""
    cfg = I.WORKLOADS[wl]
    N, k = cfg["N"], cfg["k"]
    banner(f"apply full {wl}")
    theta = I.theta(N ** 3)
    m = O.Mesh(N, N, N, k, theta=theta)
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(theta))
    x = I.uniform_vector(m.ndof)
    y = host(op.apply(dev(x)))
    el = _sample_elements(N)
    ref = O.apply_rows(m, x, el)
    got = y.reshape(-1, m.n3)[el]
    err = rel_l2(got, ref)
    print(f"fp64 apply {wl} sampled rows: rel err {err:.3e}")
    assert err <= 1e-12


def test_full_size_low_precision_q4_64():
    """FP32 and BF16 applies of the 64^3 Q4 workload (the benchmark's launch
    configuration, 32.8M DOF) against the oracle on sampled element rows, with
    both errors of each result: the total error against A x (x the FP64
    input) and the arithmetic error against A x_hat (x_hat = the rounded input
    the kernel actually received)."""
    N, k = 64, 4
    banner("apply 64^3 Q4 FP32 / BF16 sampled rows")
    theta = I.theta(N ** 3)
    m = O.Mesh(N, N, N, k, theta=theta)
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(theta))
    x = I.uniform_vector(m.ndof)
    el = _sample_elements(N, extra_seed=4)
    ref = O.apply_rows(m, x, el)
    idx = torch.as_tensor(el, device="cuda")
    x32 = I.to_f32(x)
    X32 = dev(x32, torch.float32)
    got32 = host(op.apply(X32, prec="f32").view(-1, m.n3)[idx])
    del X32
    bits = I.to_bf16_bits(x)
    xh = I.bf16_bits_to_f64(bits)
    X16 = bf16_dev(bits)
    del bits
    got16 = host(op.apply(X16, prec="bf16").view(-1, m.n3)[idx])
    del X16
    e32_total = rel_l2(got32, ref)
    e32_arith = rel_l2(got32, O.apply_rows(m, x32.astype(np.float64), el))
    e16_total = rel_l2(got16, ref)
    e16_arith = rel_l2(got16, O.apply_rows(m, xh, el))
    print(f"64^3 Q4 sampled rows: fp32 total {e32_total:.3e} arithmetic {e32_arith:.3e}; "
          f"bf16 total {e16_total:.3e} arithmetic {e16_arith:.3e}")
    assert e32_arith <= 2e-5 and e32_total <= 2e-5
    assert e16_arith <= 2e-5
    assert e16_total <= 2e-2
    torch.cuda.empty_cache()


def test_full_csr_q3_32():
    """The 32^3 Q3 headline workload against the oracle's full CSR matrix
    (9.1e8 stored entries) and its OpenMP SpMV."""
    N, k = 32, 3
    banner("apply 32^3 Q3 vs full CSR")
    theta = I.theta(N ** 3)
    m = O.Mesh(N, N, N, k, theta=theta)
    A = O.assemble(m)
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(theta))
    x = I.uniform_vector(m.ndof)
    y_ref = O.spmv(A, x)
    del A
    err = rel_l2(host(op.apply(dev(x))), y_ref)
    print(f"fp64 apply dirichlet_q3_32 full CSR: rel err {err:.3e}")
    assert err <= 1e-12


def test_setup_destroy_and_streams():
    """Repeated context creation / destruction, and work enqueued on a
    non-default stream ordered with torch work on that stream."""
    banner("setup/destroy loop and side stream")
    N, k = 6, 2
    theta = I.theta(N ** 3)
    m = O.Mesh(N, N, N, k, theta=theta)
    A = O.assemble(m)
    x = I.uniform_vector(m.ndof)
    for _ in range(20):
        op = DGOperator(N, N, N, k, "dirichlet", theta=dev(theta))
        assert rel_l2(host(op.apply(dev(x))), A @ x) <= 1e-12
        op.close()
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(theta))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        X = dev(x) * 2.0                          # torch work on s
        Y = op.apply(X, stream=s)                 # the library on s, after it
        Z = op.apply(Y * 0.5, stream=s)           # and torch again in between
    s.synchronize()
    assert rel_l2(host(Y), A @ (2.0 * x)) <= 1e-12
    assert rel_l2(host(Z), A @ (A @ x)) <= 1e-12


def test_large_mesh_byte_offsets():
    """168^3 Q3 (303.5M DOF, 2.4 GB per FP64 vector): element data beyond byte
    offset 2^31; sampled element rows (first, last, spread) against the oracle."""
    N, k = 168, 3
    banner("apply 168^3 Q3 (byte offsets > 2^31)")
    theta = I.theta(N ** 3)
    m = O.Mesh(N, N, N, k, theta=theta)
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(theta))
    x = I.uniform_vector(m.ndof)
    X = dev(x)
    el = np.unique(np.r_[0, N - 1, N ** 3 // 2, N ** 3 - N * N, N ** 3 - 1,
                         np.random.default_rng(11).choice(N ** 3, 6, replace=False)]).astype(np.int64)
    ref = O.apply_rows(m, x, el)
    for trans in (False, True):
        y = op.apply(X, transpose=trans)
        got = host(y.view(-1, m.n3)[torch.as_tensor(el, device="cuda")])
        err = rel_l2(got, ref)
        print(f"fp64 apply 168^3 Q3 transpose={trans}: rel err {err:.3e}")
        assert err <= 1e-12, trans
        del y
    del X, op
    torch.cuda.empty_cache()


def test_vector_beyond_4gib():
    """206^3 Q3 (559M DOF, 4.5 GB per FP64 vector): above 4 GiB the apply forms
    64-bit addresses (below it, 32-bit byte offsets); sampled element rows
    against the oracle, including the last elements of the vector."""
    N, k = 206, 3
    banner("apply 206^3 Q3 (vector above 4 GiB)")
    theta = I.theta(N ** 3)
    m = O.Mesh(N, N, N, k, theta=theta)
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(theta))
    assert op.ndof * 8 > 2 ** 32
    el = np.unique(np.r_[0, N ** 3 // 2, N ** 3 - N * N - 1, N ** 3 - 2, N ** 3 - 1,
                         np.random.default_rng(12).choice(N ** 3, 5, replace=False)]).astype(np.int64)
    x = I.uniform_vector(m.ndof)
    X = dev(x)
    y = op.apply(X)
    got = host(y.view(-1, m.n3)[torch.as_tensor(el, device="cuda")])
    err = rel_l2(got, O.apply_rows(m, x, el))
    print(f"fp64 apply 206^3 Q3: rel err {err:.3e}")
    assert err <= 1e-12
    del X, y, op, x
    torch.cuda.empty_cache()


def test_low_precision_errors():
    """FP32 and BF16 (FP32 accumulation) applies against the FP64 oracle.
    FP32: relative error a modest multiple of 2^-24 times the operator's
    cancellation; BF16: arithmetic error against A x_hat (x_hat = rounded input)
    like FP32, total error against A x dominated by the input rounding 2^-9."""
    banner("apply low precision")
    N, k = 6, 4
    theta = I.theta(N ** 3)
    m = O.Mesh(N, N, N, k, theta=theta)
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(theta))
    A = O.assemble(m)
    x = I.uniform_vector(m.ndof)
    y_ref = A @ x
    y32 = host(op.apply(dev(I.to_f32(x), torch.float32), prec="f32"))
    e32 = rel_l2(y32, y_ref)
    bits = I.to_bf16_bits(x)
    xh = I.bf16_bits_to_f64(bits)
    y16 = host(op.apply(bf16_dev(bits), prec="bf16"))
    e16_arith = rel_l2(y16, A @ xh)
    e16_total = rel_l2(y16, y_ref)
    print(f"fp32 err {e32:.3e}  bf16 arithmetic err {e16_arith:.3e}  bf16 total err {e16_total:.3e}")
    assert e32 <= 2e-5
    assert e16_arith <= 2e-5
    assert e16_total <= 2e-2


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_transpose(prec):
    """A^T x equals A x up to rounding (symmetric form), and <y, A x> = <A^T y, x>."""
    banner(f"transpose {prec}")
    N, k = 5, 3
    theta = I.theta(N ** 3)
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(theta))
    nd = op.ndof
    x = I.uniform_vector(nd, seed=1)
    yv = I.uniform_vector(nd, seed=2)
    if prec == "f64":
        X, Y = dev(x), dev(yv)
    elif prec == "f32":
        X, Y = dev(x, torch.float32), dev(yv, torch.float32)
    else:
        X, Y = bf16_dev(I.to_bf16_bits(x)), bf16_dev(I.to_bf16_bits(yv))
    Ax = host(op.apply(X, prec=prec))
    ATx = host(op.apply(X, prec=prec, transpose=True))
    ATy = host(op.apply(Y, prec=prec, transpose=True))
    tol = 1e-14 if prec == "f64" else 1e-6
    assert rel_l2(ATx, Ax) <= tol
    xs, ys = host(X), host(Y)
    lhs, rhs = ys @ Ax, ATy @ xs
    assert abs(lhs - rhs) <= (1e-13 if prec == "f64" else 1e-5) * np.linalg.norm(ys) * np.linalg.norm(Ax)


def test_determinism_and_errors():
    banner("determinism and argument errors")
    N, k = 8, 3
    theta = I.theta(N ** 3)
    op = DGOperator(N, N, N, k, "dirichlet", theta=dev(theta))
    x = dev(I.uniform_vector(op.ndof))
    y1 = op.apply(x).clone()
    y2 = op.apply(x).clone()
    assert torch.equal(y1, y2)
    with pytest.raises(DGError):
        op.apply(x, out=x)                       # aliasing
    with pytest.raises(ValueError):
        op.apply(x[:-1])                          # wrong size
    with pytest.raises(DGError):
        DGOperator(2, 2, 2, 8)                    # unsupported degree
    torch.cuda.synchronize()


def test_diagonal():
    banner("diagonal")
    for (shape, k, bc) in [((3, 2, 2), 3, "dirichlet"), ((1, 2, 3), 2, "periodic"), ((4, 4, 4), 4, "dirichlet")]:
        theta = I.theta(int(np.prod(shape)), seed=9)
        m = O.Mesh(*shape, k, bc=BCS[bc], theta=theta)
        op = DGOperator(*shape, k, bc, theta=dev(theta))
        d = host(op.diagonal())
        assert rel_l2(d, O.assemble(m).diagonal()) <= 1e-13


def test_repeatable_with_changing_inputs():
    """Applies that alternate between two inputs (x1, x2, x1, ...) give
    bit-identical results for the same input in every precision, on affine and
    trilinear meshes: a kernel reading LDS data of another element or of an
    earlier phase before it is rewritten would see the other input's values."""
    banner("repeatability with changing inputs")
    # trilinear k = 2, 4, 5, 6: an element's n^2 threads span two wavefronts,
    # so the face phases depend on workgroup barriers; perturbed meshes take
    # the general trilinear kernel, layered shears its constant-metric
    # variant, sheared meshes (one affine map) the parallelepiped kernel
    # affine k = 2, 4, 5, 6: an element spans two wavefronts (workgroup barriers)
    cases = [(32, 3, None), (12, 1, None), (6, 7, None), (10, 2, None), (12, 4, None), (7, 5, None),
             (6, 6, None), (8, 3, I.perturbed_vertices(8, 0.1, seed=3)),
             (4, 7, I.perturbed_vertices(4, 0.1, seed=4)),
             (9, 2, I.perturbed_vertices(9, 0.1, seed=5)), (7, 4, I.sheared_vertices(7, 7, 7)),
             (6, 5, I.perturbed_vertices(6, 0.1, seed=6)), (5, 6, I.sheared_vertices(5, 5, 5)),
             (5, 4, I.perturbed_vertices(5, 0.1, seed=8)), (6, 2, I.sheared_vertices(6, 6, 6)),
             (9, 3, I.sheared_vertices(9, 9, 9)), (6, 4, I.layered_shear_vertices(6, 6, 6)),
             (5, 5, I.layered_shear_vertices(5, 5, 5)), (7, 2, I.layered_shear_vertices(7, 7, 7)),
             (6, 5, I.sheared_vertices(6, 6, 6)), (4, 7, I.sheared_vertices(4, 4, 4)),
             (9, 1, I.sheared_vertices(9, 9, 9))]
    for N, k, verts in cases:
        op = DGOperator(N, N, N, k, "dirichlet", theta=dev(I.theta(N ** 3)),
                        vertices=None if verts is None else dev(verts))
        print(f"repeatability N={N} k={k} {op.kernel} kernel", flush=True)
        xs = [dev(I.uniform_vector(op.ndof, seed=s)) for s in (21, 22)]
        bf16 = lambda v: v.float().to(torch.bfloat16).contiguous()  # noqa: E731
        precs = [("f64", lambda v: v), ("f32", lambda v: v.float().contiguous()), ("bf16", bf16)]
        if op.kernel == "affine" and k <= 4:
            precs.append(("bf16_mfma", bf16))
        for prec, conv in precs:
            X = [conv(v) for v in xs]
            ref = [op.apply(X[0], prec=prec).clone(), op.apply(X[1], prec=prec).clone()]
            for r in range(40):
                y = op.apply(X[r % 2], prec=prec)
                assert torch.equal(y, ref[r % 2]), (N, k, verts is None, prec, r)
