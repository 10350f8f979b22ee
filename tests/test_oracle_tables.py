"""Pins of the oracle's 1D tables and 1D operators against closed forms.

Gauss-Legendre / Gauss-Lobatto closed forms come from tests/golden (textbook
values); the linear-element 1D SWIPDG matrices are the hand-derived fixture
tests/golden/swipdg_1d_k1.txt (Sec. 4.1 face form, K = 1).
"""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import brute, oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _closed_forms():
    rows = []
    with open(os.path.join(GOLD, "quadrature_closed_forms.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            kind, n, i, x, w = line.split()
            ev = lambda s: eval(s, {"sqrt": np.sqrt})  # noqa: E731  (fixture expressions)
            rows.append((kind, int(n), int(i), float(ev(x)), None if w == "-" else float(ev(w))))
    return rows


def test_gauss_and_lobatto_closed_forms():
    for kind, n, i, x, w in _closed_forms():
        if kind == "gauss":
            _, gx, gw = O.tables(2, n)
            assert abs(gx[i] - 0.5 * (1 + x)) < 1e-15
            assert abs(gw[i] - 0.5 * w) < 1e-15
        else:
            gll, _, _ = O.tables(n, 1)
            assert abs(gll[i] - 0.5 * (1 + x)) < 1e-15


@pytest.mark.parametrize("q", range(1, 13))
def test_gauss_exactness(q):
    """A q-point Gauss rule integrates x^m exactly for m <= 2q-1 and not for m = 2q."""
    _, gx, gw = O.tables(2, q)
    assert abs(gw.sum() - 1.0) < 1e-14
    for m in range(2 * q):
        assert abs(np.dot(gw, gx ** m) - 1.0 / (m + 1)) < 1e-14
    if q <= 8:  # the error (q!)^4 / ((2q+1) ((2q)!)^2) is above rounding up to q = 8
        assert abs(np.dot(gw, gx ** (2 * q)) - 1.0 / (2 * q + 1)) > 1e-12


@pytest.mark.parametrize("n", range(2, 13))
def test_tables_match_library_routines(n):
    gll, gx, gw = O.tables(n, n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.max(np.abs(gx - 0.5 * (xr + 1))) < 2e-15
    assert np.max(np.abs(gw - 0.5 * wr)) < 2e-15
    assert gll[0] == 0.0 and gll[-1] == 1.0
    assert np.max(np.abs(gll + gll[::-1] - 1.0)) < 2e-15
    assert np.max(np.abs(gll - brute.gll_nodes01(n))) < 1e-14


def _parse_matrix(s):
    return np.array([[float(Fraction(t)) for t in r.split()] for r in s.split(";")])


def _fixture():
    out = {}
    with open(os.path.join(GOLD, "swipdg_1d_k1.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, rest = line.split(None, 1)
            out[key] = _parse_matrix(rest)
    return out


@pytest.mark.parametrize("builder", ["oracle", "brute"])
def test_1d_operator_linear_elements(builder):
    """N = 2 periodic, k = 1: L = blockdiag(S, S)/h + F on (e0, e1) + F on (e1, e0)."""
    fx = _fixture()
    N, h = 2, 0.5
    if builder == "oracle":
        L, M = O.swipdg_1d(N, 1, O.PERIODIC)
    else:
        L, M = brute.kron_sum_1d(N, 1, periodic=True)
    S, Mm, F = fx["stiffness_times_h"], fx["mass_over_h"], fx["face_times_h"]
    exp_L = np.zeros((4, 4))
    exp_L[:2, :2] += S / h
    exp_L[2:, 2:] += S / h
    for idx in ([0, 1, 2, 3], [2, 3, 0, 1]):
        exp_L[np.ix_(idx, idx)] += F / h
    exp_M = np.kron(np.eye(2), Mm * h)
    assert np.max(np.abs(L - exp_L)) < 1e-13
    assert np.max(np.abs(M - exp_M)) < 1e-15
