"""Sensitivity of the pins: each planted mistake in the oracle (a dropped term,
a wrong sign, a transposed operand, a wrong side or weight) must make at least
one pin fail.  The mistakes are planted in the oracle, on the CPU, through its
``mutation`` switch; expected values are never produced with it set."""
import numpy as np
import pytest

from oracle import brute, oracle as O
from paper_1911_01492_amd import inputs as I


def _pert_222():
    V = I.uniform_vertices(2, 2, 2)
    V[13] += np.array([0.07, -0.05, 0.04])
    return V


def pin_symmetry(mut):
    A = O.assemble(O.Mesh(2, 2, 2, 2, theta=I.theta(8, seed=1), mutation=mut))
    return abs(A - A.T).max() <= 1e-14 * abs(A).max()


def pin_definite(mut):
    A = O.assemble(O.Mesh(2, 2, 1, 2, theta=I.theta(4, seed=2), mutation=mut)).toarray()
    return np.linalg.eigvalsh(0.5 * (A + A.T))[0] > 0


def pin_brute_force(mut):
    th = I.theta(8, seed=3)
    V = _pert_222()
    A = O.assemble(O.Mesh(2, 2, 2, 2, theta=th, vertices=V, mutation=mut)).toarray()
    D = brute.dense_matrix(2, 2, 2, 2, theta=th, vertices=V)
    return np.max(np.abs(A - D)) <= 1e-13 * np.max(np.abs(D))


def pin_convergence(mut):
    errs = []
    for N in (2, 4):
        m = O.Mesh(N, N, N, 2, mutation=mut)
        A = O.assemble(m)
        u = np.linalg.lstsq(A.toarray(), O.rhs(m, "sine"), rcond=None)[0]
        errs.append(O.l2_error(m, u, "sine"))
    return np.log2(errs[0] / errs[1]) >= 2.8


def pin_patch(mut):
    coef = np.zeros((2, 2, 2))
    coef[1, 0, 0], coef[0, 1, 0], coef[0, 0, 1] = 1.0, -2.0, 0.5
    m = O.Mesh(2, 2, 2, 1, vertices=_pert_222(), mutation=mut)
    A = O.assemble(m).toarray()
    u = np.linalg.lstsq(A, O.rhs(m, "poly", coef), rcond=None)[0]
    return O.l2_error(m, u, "poly", coef) < 1e-11


PINS = {"symmetry": pin_symmetry, "definite": pin_definite, "brute_force": pin_brute_force,
        "convergence": pin_convergence, "patch": pin_patch}

# mistake -> the pins expected to catch it
CAUGHT_BY = {
    "plus_consistency": ["convergence", "brute_force"],
    "no_symmetry": ["symmetry", "brute_force"],
    "no_penalty": ["definite", "brute_force"],
    "no_boundary": ["definite", "brute_force", "convergence"],
    "jinv_not_transposed": ["brute_force", "patch"],
    "arith_gamma": ["brute_force"],
    "penalty_no_area": ["brute_force"],
    "plus_side_at_one": ["brute_force", "convergence"],
}


def test_unmutated_oracle_passes_every_pin():
    for name, pin in PINS.items():
        assert pin(0), name


@pytest.mark.parametrize("mistake", sorted(CAUGHT_BY))
def test_planted_mistake_is_caught(mistake):
    mut = O.MUTATIONS[mistake]
    for name in CAUGHT_BY[mistake]:
        assert not PINS[name](mut), f"{mistake} not caught by {name}"
