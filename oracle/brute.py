"""Independent checkers for the C++ oracle (TEST INFRASTRUCTURE, NOT PRODUCT CODE).

Nothing here calls ``liboracle.so``: the tables, the geometry, the basis and
the assembly are written again, differently, so that agreement pins the
oracle rather than restating it.

* ``dense_matrix`` -- brute-force dense assembly in numpy.  Unlike the oracle
  (element block rows, every face visited from both sides, gamma/2 form) it
  loops once over every face of the mesh, writes the SWIPDG weighted average in
  its omega form  <K grad u . n>_w = w^- K^- grad u^- . n + w^+ K^+ grad u^+ . n,
  w^- = K^+/(K^- + K^+), w^+ = K^-/(K^- + K^+)  (Sec. 4.1, SWIPDG forms), takes
  Gauss points from ``numpy.polynomial.legendre.leggauss`` and the GLL nodes as
  roots of P_k' from numpy's Legendre class.
* ``exact_matrix`` -- exact rational entries (``fractions.Fraction``) for
  k <= 2 on uniform affine meshes, where the GLL nodes {0, 1} and
  {0, 1/2, 1} are rational: 1D integrals of Lagrange polynomials are done
  symbolically and combined by Fubini's theorem.
* ``kron_sum_1d`` -- the 1D SWIPDG operator and mass matrix in floating point,
  from which the K == 1 operator on a uniform box mesh is the Kronecker sum
  M (x) M (x) L + M (x) L (x) M + L (x) M (x) M.
"""
from __future__ import annotations

from fractions import Fraction
from itertools import product

import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly


# --------------------------------------------------------------------------
# tables (numpy library routines)
# --------------------------------------------------------------------------

def gll_nodes01(n: int) -> np.ndarray:
    k = n - 1
    inner = npleg.Legendre.basis(k).deriv().roots() if k >= 2 else np.array([])
    x = np.sort(np.r_[-1.0, np.real(inner), 1.0])
    return 0.5 * (x + 1.0)


def gauss01(q: int):
    x, w = npleg.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_polys(nodes: np.ndarray):
    """Power-series coefficient arrays of the Lagrange polynomials and their derivatives."""
    n = len(nodes)
    P, dP = [], []
    for i in range(n):
        others = np.delete(nodes, i)
        c = nppoly.polyfromroots(others)
        c = c / nppoly.polyval(nodes[i], c)
        P.append(c)
        dP.append(nppoly.polyder(c))
    return P, dP


# --------------------------------------------------------------------------
# brute-force dense assembly
# --------------------------------------------------------------------------

def _vertices(nx, ny, nz, vertices):
    if vertices is not None:
        return np.asarray(vertices, dtype=np.float64).reshape(nz + 1, ny + 1, nx + 1, 3)
    X = np.zeros((nz + 1, ny + 1, nx + 1, 3))
    X[..., 0] = (np.arange(nx + 1) / nx)[None, None, :]
    X[..., 1] = (np.arange(ny + 1) / ny)[None, :, None]
    X[..., 2] = (np.arange(nz + 1) / nz)[:, None, None]
    return X


class _Elem:
    """Geometry of one trilinear hexahedron from its 8 corner vertices."""

    def __init__(self, Xv, ex, ey, ez):
        self.C = np.array([Xv[ez + c2, ey + c1, ex + c0] for c2 in (0, 1) for c1 in (0, 1)
                           for c0 in (0, 1)])  # corner index c0 + 2 c1 + 4 c2

    def jac(self, xi):
        """xi: (P, 3) -> J: (P, 3, 3), J[p, a, d] = dx_a / dxi_d."""
        xi = np.atleast_2d(xi)
        J = np.zeros((xi.shape[0], 3, 3))
        for c in range(8):
            bits = [(c >> d) & 1 for d in range(3)]
            f = [xi[:, d] if bits[d] else 1.0 - xi[:, d] for d in range(3)]
            df = [1.0 if bits[d] else -1.0 for d in range(3)]
            dN = [df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]]
            for d in range(3):
                J[:, :, d] += np.outer(dN[d], self.C[c])
        return J


def _basis(P, dP, xi):
    """Values (P, n3) and reference gradients (P, n3, 3) of the tensor basis at points xi."""
    n = len(P)
    L = [np.array([nppoly.polyval(xi[:, d], P[i]) for i in range(n)]).T for d in range(3)]
    dL = [np.array([nppoly.polyval(xi[:, d], dP[i]) for i in range(n)]).T for d in range(3)]
    val = np.einsum("pa,pb,pc->pcba", L[0], L[1], L[2]).reshape(xi.shape[0], -1)
    g0 = np.einsum("pa,pb,pc->pcba", dL[0], L[1], L[2]).reshape(xi.shape[0], -1)
    g1 = np.einsum("pa,pb,pc->pcba", L[0], dL[1], L[2]).reshape(xi.shape[0], -1)
    g2 = np.einsum("pa,pb,pc->pcba", L[0], L[1], dL[2]).reshape(xi.shape[0], -1)
    return val, np.stack([g0, g1, g2], axis=-1)


def dense_matrix(nx, ny, nz, k, periodic=False, theta=None, vertices=None, penalty_hat=0.0):
    """Dense A_ij = b_h(phi_j, phi_i) by a single loop over elements and a single
    loop over faces (no face visited twice)."""
    n = k + 1
    n3 = n ** 3
    E = nx * ny * nz
    A = np.zeros((E * n3, E * n3))
    K = np.exp(np.asarray(theta, dtype=np.float64)) if theta is not None else np.ones(E)
    sh = penalty_hat if penalty_hat > 0 else 2.0 * (k + 1) ** 2
    P, dP = lagrange_polys(gll_nodes01(n))
    gx, gw = gauss01(n)
    Xv = _vertices(nx, ny, nz, vertices)
    N = (nx, ny, nz)

    def eid(e):
        return e[0] + nx * (e[1] + ny * e[2])

    elems = {}
    for ez, ey, ex in product(range(nz), range(ny), range(nx)):
        elems[(ex, ey, ez)] = _Elem(Xv, ex, ey, ez)

    # volume terms
    Q = np.array([[gx[a], gx[b], gx[c]] for c in range(n) for b in range(n) for a in range(n)])
    W = np.array([gw[a] * gw[b] * gw[c] for c in range(n) for b in range(n) for a in range(n)])
    val, gref = _basis(P, dP, Q)
    for (ex, ey, ez), el in elems.items():
        J = el.jac(Q)
        Jinv = np.linalg.inv(J)
        g = np.einsum("pda,pid->pia", Jinv, gref)      # J^{-T} ghat
        wdet = W * np.abs(np.linalg.det(J)) * K[eid((ex, ey, ez))]
        s = slice(eid((ex, ey, ez)) * n3, (eid((ex, ey, ez)) + 1) * n3)
        A[s, s] += np.einsum("p,pia,pja->ij", wdet, g, g)

    def face_points(d, side):
        a, b = (d + 1) % 3, (d + 2) % 3
        pts = np.zeros((n * n, 3))
        w = np.zeros(n * n)
        for qb in range(n):
            for qa in range(n):
                p = qa + n * qb
                pts[p, d] = side
                pts[p, a] = gx[qa]
                pts[p, b] = gx[qb]
                w[p] = gw[qa] * gw[qb]
        return pts, w

    def side_data(el, d, side):
        pts, w = face_points(d, side)
        J = el.jac(pts)
        a, b = (d + 1) % 3, (d + 2) % 3
        nvec = np.cross(J[:, :, a], J[:, :, b])        # towards increasing xi_d
        v, gr = _basis(P, dP, pts)
        g = np.einsum("pda,pid->pia", np.linalg.inv(J), gr)
        return w, nvec, v, g

    for d in range(3):
        sig = sh * N[d]
        for ez, ey, ex in product(range(nz), range(ny), range(nx)):
            e = [ex, ey, ez]
            up = list(e)
            up[d] += 1
            if up[d] == N[d]:
                if periodic:
                    up[d] = 0
                else:
                    # boundary at xi_d = 1 of e
                    w, nv, v, g = side_data(elems[tuple(e)], d, 1.0)
                    _add_boundary(A, eid(e) * n3, n3, w, nv, v, g, K[eid(e)], sig)
                    up = None
            if e[d] == 0 and not periodic:
                w, nv, v, g = side_data(elems[tuple(e)], d, 0.0)
                _add_boundary(A, eid(e) * n3, n3, w, -nv, v, g, K[eid(e)], sig)
            if up is None:
                continue
            em, ep = eid(e), eid(up)
            w, nv, vm, gm = side_data(elems[tuple(e)], d, 1.0)
            _, _, vp, gp = side_data(elems[tuple(up)], d, 0.0)
            Km, Kp = K[em], K[ep]
            wm, wp = Kp / (Km + Kp), Km / (Km + Kp)
            gam = 2.0 * Km * Kp / (Km + Kp)
            area = np.linalg.norm(nv, axis=1)
            jump = np.concatenate([vm, -vp], axis=1)                         # (P, 2 n3)
            avg = np.concatenate([wm * Km * np.einsum("pia,pa->pi", gm, nv),
                                  wp * Kp * np.einsum("pia,pa->pi", gp, nv)], axis=1)
            loc = (-np.einsum("p,pj,pi->ij", w, avg, jump)
                   - np.einsum("p,pi,pj->ij", w, avg, jump)
                   + sig * gam * np.einsum("p,pj,pi->ij", w * area, jump, jump))
            idx = np.r_[em * n3:(em + 1) * n3, ep * n3:(ep + 1) * n3]
            np.add.at(A, np.ix_(idx, idx), loc)
    return A


def _add_boundary(A, off, n3, w, nv, v, g, K, sig):
    fl = np.einsum("pia,pa->pi", g, nv)
    area = np.linalg.norm(nv, axis=1)
    loc = K * (-np.einsum("p,pj,pi->ij", w, fl, v) - np.einsum("p,pi,pj->ij", w, fl, v)
               + sig * np.einsum("p,pj,pi->ij", w * area, v, v))
    A[off:off + n3, off:off + n3] += loc


# --------------------------------------------------------------------------
# exact rationals (k <= 2, uniform affine mesh)
# --------------------------------------------------------------------------

def _fr_poly_mul(a, b):
    c = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            c[i + j] += x * y
    return c


def _fr_poly_der(a):
    return [i * a[i] for i in range(1, len(a))] or [Fraction(0)]


def _fr_poly_int01(a):
    return sum(c / (i + 1) for i, c in enumerate(a))


def _fr_poly_val(a, x):
    return sum(c * x ** i for i, c in enumerate(a))


def exact_1d(k: int):
    """Exact 1D objects on [0,1] for k <= 2: mass M, stiffness S, endpoint values e0, e1
    and endpoint derivatives d0, d1 of the GLL Lagrange basis."""
    nodes = {1: [Fraction(0), Fraction(1)], 2: [Fraction(0), Fraction(1, 2), Fraction(1)]}[k]
    n = k + 1
    polys = []
    for i in range(n):
        p = [Fraction(1)]
        for j in range(n):
            if j != i:
                p = _fr_poly_mul(p, [-nodes[j] / (nodes[i] - nodes[j]), 1 / (nodes[i] - nodes[j])])
        polys.append(p)
    der = [_fr_poly_der(p) for p in polys]
    M = [[_fr_poly_int01(_fr_poly_mul(polys[i], polys[j])) for j in range(n)] for i in range(n)]
    S = [[_fr_poly_int01(_fr_poly_mul(der[i], der[j])) for j in range(n)] for i in range(n)]
    e0 = [_fr_poly_val(p, Fraction(0)) for p in polys]
    e1 = [_fr_poly_val(p, Fraction(1)) for p in polys]
    d0 = [_fr_poly_val(p, Fraction(0)) for p in der]
    d1 = [_fr_poly_val(p, Fraction(1)) for p in der]
    return M, S, e0, e1, d0, d1


def exact_matrix(nx, ny, nz, k, periodic=False, K=None, penalty_hat=None):
    """Exact rational matrix for k <= 2 on the uniform nx*ny*nz mesh with
    rational K per element (list of Fractions, default 1)."""
    n = k + 1
    n3 = n ** 3
    N = (nx, ny, nz)
    E = nx * ny * nz
    h = [Fraction(1, N[d]) for d in range(3)]
    K = [Fraction(1)] * E if K is None else [Fraction(x) for x in K]
    sh = Fraction(2 * (k + 1) ** 2) if penalty_hat is None else Fraction(penalty_hat)
    M, S, e0, e1, d0, d1 = exact_1d(k)
    A = [[Fraction(0)] * (E * n3) for _ in range(E * n3)]

    def eid(e):
        return e[0] + nx * (e[1] + ny * e[2])

    def loc(i):
        return (i % n, (i // n) % n, i // (n * n))

    # integral over an element of d_d phi_j d_d phi_i, Fubini per axis
    def vol(i, j):
        ii, jj = loc(i), loc(j)
        s = Fraction(0)
        for d in range(3):
            t = S[ii[d]][jj[d]] / h[d]
            for a in range(3):
                if a != d:
                    t *= M[ii[a]][jj[a]] * h[a]
            s += t
        return s

    def tang(ii, jj, d):
        t = Fraction(1)
        for a in range(3):
            if a != d:
                t *= M[ii[a]][jj[a]] * h[a]
        return t

    for ez, ey, ex in product(range(nz), range(ny), range(nx)):
        e = eid((ex, ey, ez))
        for i in range(n3):
            for j in range(n3):
                A[e * n3 + i][e * n3 + j] += K[e] * vol(i, j)
    for d in range(3):
        sig = sh / h[d]
        for ez, ey, ex in product(range(nz), range(ny), range(nx)):
            ec = [ex, ey, ez]
            e = eid(ec)
            up = list(ec)
            up[d] += 1
            bnd_hi = up[d] == N[d] and not periodic
            if up[d] == N[d]:
                up[d] = 0
            # boundary faces: outward derivative on xi_d = 1 is +d1/h, on xi_d = 0 is -d0/h
            for s_, on in ((1, bnd_hi), (0, ec[d] == 0 and not periodic)):
                if not on:
                    continue
                ev = e1 if s_ else e0
                dv = [x / h[d] for x in (d1 if s_ else d0)]
                sgn = 1 if s_ else -1
                for i in range(n3):
                    for j in range(n3):
                        ii, jj = loc(i), loc(j)
                        t = tang(ii, jj, d)
                        val = (-sgn * dv[jj[d]] * ev[ii[d]] - sgn * dv[ii[d]] * ev[jj[d]]
                               + sig * ev[jj[d]] * ev[ii[d]])
                        A[e * n3 + i][e * n3 + j] += K[e] * t * val
            if bnd_hi:
                continue
            ep = eid(up)
            Km, Kp = K[e], K[ep]
            gam = 2 * Km * Kp / (Km + Kp)
            for sa, ea in ((0, e), (1, ep)):
                for sb, eb in ((0, e), (1, ep)):
                    for i in range(n3):
                        for j in range(n3):
                            ii, jj = loc(i), loc(j)
                            t = tang(ii, jj, d)
                            ja = e1[ii[d]] if sa == 0 else -e0[ii[d]]
                            jb = e1[jj[d]] if sb == 0 else -e0[jj[d]]
                            fa = (d1[ii[d]] if sa == 0 else d0[ii[d]]) / h[d]
                            fb = (d1[jj[d]] if sb == 0 else d0[jj[d]]) / h[d]
                            val = -gam / 2 * fb * ja - gam / 2 * fa * jb + sig * gam * ja * jb
                            A[ea * n3 + i][eb * n3 + j] += t * val
    return A


# --------------------------------------------------------------------------
# Kronecker sum (K == 1, uniform box mesh)
# --------------------------------------------------------------------------

def kron_sum_1d(N: int, k: int, periodic: bool, penalty_hat: float = 0.0):
    """1D SWIPDG operator L and mass M on N elements (h = 1/N), numpy tables."""
    n = k + 1
    h = 1.0 / N
    sh = penalty_hat if penalty_hat > 0 else 2.0 * (k + 1) ** 2
    P, dP = lagrange_polys(gll_nodes01(n))
    gx, gw = gauss01(n)
    B = np.array([[nppoly.polyval(x, P[i]) for i in range(n)] for x in gx])
    D = np.array([[nppoly.polyval(x, dP[i]) for i in range(n)] for x in gx])
    e0 = np.array([nppoly.polyval(0.0, P[i]) for i in range(n)])
    e1 = np.array([nppoly.polyval(1.0, P[i]) for i in range(n)])
    d0 = np.array([nppoly.polyval(0.0, dP[i]) for i in range(n)]) / h
    d1 = np.array([nppoly.polyval(1.0, dP[i]) for i in range(n)]) / h
    Ml = h * (B.T * gw) @ B
    Sl = (D.T * gw) @ D / h
    L = np.kron(np.eye(N), Sl)
    M = np.kron(np.eye(N), Ml)
    sig = sh / h
    faces = range(N) if periodic else range(N - 1)
    for f in faces:
        a, b = f, (f + 1) % N
        jump = np.zeros(N * n)
        flux = np.zeros(N * n)
        jump[a * n:(a + 1) * n] += e1
        jump[b * n:(b + 1) * n] -= e0
        flux[a * n:(a + 1) * n] += d1
        flux[b * n:(b + 1) * n] += d0
        L += -0.5 * np.outer(jump, flux) - 0.5 * np.outer(flux, jump) + sig * np.outer(jump, jump)
    if not periodic:
        v = np.zeros(N * n)
        dv = np.zeros(N * n)
        v[:n] = e0
        dv[:n] = -d0                       # outward derivative at x = 0
        L += -np.outer(v, dv) - np.outer(dv, v) + sig * np.outer(v, v)
        v = np.zeros(N * n)
        dv = np.zeros(N * n)
        v[-n:] = e1
        dv[-n:] = d1
        L += -np.outer(v, dv) - np.outer(dv, v) + sig * np.outer(v, v)
    return L, M


def kron_sum_matrix(nx, ny, nz, k, periodic, penalty_hat=0.0):
    """K == 1 operator in the element-blocked ordering, from the Kronecker sum."""
    n = k + 1
    Lx, Mx = kron_sum_1d(nx, k, periodic, penalty_hat)
    Ly, My = kron_sum_1d(ny, k, periodic, penalty_hat)
    Lz, Mz = kron_sum_1d(nz, k, periodic, penalty_hat)
    T = (np.kron(Mz, np.kron(My, Lx)) + np.kron(Mz, np.kron(Ly, Mx)) + np.kron(Lz, np.kron(My, Mx)))
    # permutation: tensor index (gz, gy, gx) -> blocked (ez, ey, ex, i3, i2, i1)
    idx = np.arange(T.shape[0]).reshape(nz, n, ny, n, nx, n).transpose(0, 2, 4, 1, 3, 5).reshape(-1)
    return T[np.ix_(idx, idx)]
