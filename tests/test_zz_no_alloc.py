"""dg_dA_dtheta_noalloc (scratch in the library's static device array) against
dg_dA_dtheta (scratch in the context's workspace): identical kernels and
arithmetic, so the results must agree bit for bit.  Two calls in a row, the
second on a smaller trilinear mesh (the static array keeps the first call's
contents), then an affine mesh (no scratch) and the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1911_01492_amd import inputs as I  # noqa: E402
from paper_1911_01492_amd.dg import DG_ERR_ARG, DGError, DGOperator  # noqa: E402
from tests.gpu_util import banner, dev, host  # noqa: E402


def _op(N, k, trilinear, seed):
    theta = I.theta(N ** 3, seed=seed)
    verts = dev(I.perturbed_vertices(N)) if trilinear else None
    return DGOperator(N, N, N, k, "dirichlet", theta=dev(theta), vertices=verts)


@pytest.mark.parametrize("trilinear", [True, False])
def test_noalloc_matches_workspace_variant(trilinear):
    for N, k, seed in ((10, 3, 1), (4, 2, 7)):  # second call: smaller mesh
        banner(f"dA_dtheta_noalloc trilinear={trilinear} N={N} k={k}")
        op = _op(N, k, trilinear, seed)
        u = dev(I.uniform_vector(op.ndof, seed=seed + 10))
        v = dev(I.uniform_vector(op.ndof, seed=seed + 11))
        g_ref = host(op.dA_dtheta(u, v))
        out = torch.full((op.E,), float("nan"), dtype=torch.float64, device="cuda")
        g = host(op.dA_dtheta_noalloc(u, v, out))
        assert np.array_equal(g, g_ref), (N, k, np.abs(g - g_ref).max())
        # and against the oracle's closed-form sensitivity on the same inputs
        m = O.Mesh(N, N, N, k, theta=I.theta(N ** 3, seed=seed),
                   vertices=I.perturbed_vertices(N) if trilinear else None)
        g_ora = O.dA_dtheta(m, host(u), host(v))
        assert np.abs(g - g_ora).max() <= 1e-10 * np.abs(g_ora).max()


def test_noalloc_rejects_meshes_beyond_the_static_scratch():
    banner("dA_dtheta_noalloc size limit")
    N = 67  # 300763 elements > 16 MiB / 56 B
    op = _op(N, 1, True, 1)
    u = torch.zeros(op.ndof, dtype=torch.float64, device="cuda")
    out = torch.zeros(op.E, dtype=torch.float64, device="cuda")
    with pytest.raises(DGError) as ei:
        op.dA_dtheta_noalloc(u, u, out)
    assert ei.value.code == DG_ERR_ARG
