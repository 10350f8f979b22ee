// dg_trilinear.hip -- SWIPDG apply on trilinear hexahedra (curved meshes,
// "problem C" with multilinear geometries of Sec. 3.3), Jacobians computed
// on the fly at every volume and face quadrature point.
//
// Volume (sum factorisation through the Gauss points):
//   v    = (B (x) B (x) B) u                      interpolation GLL -> Gauss
//   gr_d = Dg along axis d applied to v            reference gradient
//   g    = G_q gr,  G_q = w_q K |det J| J^{-1} J^{-T} = w_q K adj(J) adj(J)^T / |det J|
//   y    = (B^T (x) B^T (x) B^T) (sum_d Dg_d^T g_d + c w_q |det J| v)
// (the last term is the optional reaction, c = 0 without it)
// Faces (Sec. 4.1 face form b_h^e, with its readings as in the affine path):
// at the n^2 face Gauss points, traces and reference gradients of both sides
// (normal derivative from each side's lines, tangential interpolation and
// derivatives by 2D sum factorisation through LDS), physical gradients with
// each side's own Jacobian, area-weighted normal n dS = dF/dxi_a x dF/dxi_b
// of T^-; the test-function side is projected back with the transposed
// tangential operators.  Each interior face is evaluated once, by its lower
// element T^-, in the first of two passes: T^- adds its own rows and leaves
// the two line scalars per face node of the T^+ side in a face buffer of the
// workspace, which the second pass adds to T^+ (no atomics).  Dirichlet faces
// are evaluated by their only element in the first pass.
//
// The discrete form is symmetric, so the transposed apply evaluates the same
// kernel.
#include "dg_internal.hpp"
#include "dg_kernels.hpp"
#include "dg_lines.hpp"
#include "dg_geom.hpp"

namespace dg {

// Synchronisation of the n^2 threads of one element: every exchange through
// LDS in these kernels stays inside one element (its tiles, face buffers and
// corner slots).  When n^2 divides 64 an element lies inside one wavefront,
// whose lanes execute together and whose LDS operations complete in order, so
// only the compiler has to be kept from moving LDS accesses across this
// point; otherwise the element may span two wavefronts and the workgroup
// barrier is used.
template <int N>
__device__ __forceinline__ void elem_sync() {
  if constexpr (64 % (N * N) == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// coordinate a of corner c (bit 0: +x, bit 1: +y, bit 2: +z) of the element
// at grid position (cx, cy, cz) (the callers know it: no index division)
template <typename TC>
__device__ __forceinline__ void corner_at(const MeshArgs<TC>& m, int cx, int cy, int cz, int c, int a, TC& out) {
  const int vx = cx + (c & 1), vy = cy + ((c >> 1) & 1), vz = cz + ((c >> 2) & 1);
  const int64_t v = vx + (int64_t)(m.nx + 1) * (vy + (int64_t)(m.ny + 1) * vz);
  out = m.vert[3 * v + a];
}

// Face contributions of the face normal to axis D on side s of the thread's
// element, added into the element's accumulator tile Y.  UNIT: with the face
// coefficient set to 1 (gamma_e on interior faces, K_T on boundary faces),
// for the sensitivity dA/dtheta.  AFF: the element is a parallelepiped and
// Gc holds its constant J, adj J and det J.  PAIR (upper faces, s = 1): the
// face is evaluated once for both elements; the neighbour's side (T^+, whose
// lower face it is) is projected as well and its two line scalars per face
// node go to m.fb for the second pass.  All threads of the block call this
// (it synchronises); act marks threads owning an element.
template <int N, int D, typename TC, typename TIN, bool UNIT = false, bool AFF = false, bool PAIR = false, int LV = 0>
__device__ void face_term(const MeshArgs<TC>& m, const Tables<TC>& T, const TIN* __restrict__ x, int64_t e,
                          int ex, int ey, int ez, const TC (&X)[8][3], TC (&Xn)[8][3], TC K, int t1, int t2,
                          TC* Y, TC (*F)[N * N], bool act, int s, const TC* Gc = nullptr) {
  constexpr int NN = N * N;
  const int t = t1 + N * t2;
  const int ax = (D == 0) ? 1 : 0;  // reference axis of t1
  const int bx = (D == 2) ? 1 : 2;  // reference axis of t2
  const TC* dS = s ? T.d1 : T.d0;   // own derivative at the own face end
  const TC* dN = s ? T.d0 : T.d1;   // neighbour's derivative at its face end
  int64_t nb = -1;
  TC Uo = TC(0), Go = TC(0), Un = TC(0), Gn = TC(0);
  if (act) {
    nb = neighbour<D>(m, ex, ey, ez, s);
    // the neighbour's corners, staged once per element (read after the barriers below)
    if (nb >= 0) {
      int g[3] = {ex, ey, ez};
      g[D] = nb_coord(g[D], s, D == 0 ? m.nx : (D == 1 ? m.ny : m.nz), m.periodic);
      for (int q = t; q < 24; q += NN) corner_at(m, g[0], g[1], g[2], q / 3, q % 3, Xn[q / 3][q % 3]);
    }
    TC own[N];
    glb_get<N, D, TC, TIN>(x, e, t1, t2, own);
    Uo = own[s ? N - 1 : 0];
#pragma unroll
    for (int i = 0; i < N; ++i) Go += dS[i] * own[i];
    if (nb >= 0) {
      TC nl[N];
      glb_get<N, D, TC, TIN>(x, nb, t1, t2, nl);
      Un = nl[s ? 0 : N - 1];
#pragma unroll
      for (int i = 0; i < N; ++i) Gn += dN[i] * nl[i];
    }
  }
  elem_sync<N>();  // face buffers free
  if (act) {
    F[0][t] = Uo;
    F[1][t] = Go;
    F[2][t] = Un;
    F[3][t] = Gn;
  }
  elem_sync<N>();
  if (act) {  // interpolation / derivative along t1 (axis ax)
    TC bu = 0, du = 0, bg = 0, bun = 0, dun = 0, bgn = 0;
#pragma unroll
    for (int a = 0; a < N; ++a) {
      const TC B = T.B[t1 * kMaxN + a], Dd = T.D[t1 * kMaxN + a];
      bu += B * F[0][t2 * N + a];
      du += Dd * F[0][t2 * N + a];
      bg += B * F[1][t2 * N + a];
      bun += B * F[2][t2 * N + a];
      dun += Dd * F[2][t2 * N + a];
      bgn += B * F[3][t2 * N + a];
    }
    F[4][t] = bu;
    F[5][t] = du;
    F[6][t] = bg;
    F[7][t] = bun;
    F[8][t] = dun;
    F[9][t] = bgn;
  }
  elem_sync<N>();
  TC P = 0, Ra = 0, Rb = 0, Rd = 0;
  TC Pn = 0, Ran = 0, Rbn = 0, Rdn = 0;  // PAIR: the neighbour's side (T^+)
  if (act) {  // along t2 (axis bx): values at face Gauss point (qa, qb) = (t1, t2)
    TC uo = 0, gao = 0, gbo = 0, gdo = 0, un = 0, gan = 0, gbn = 0, gdn = 0;
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const TC B = T.B[t2 * kMaxN + b], Dd = T.D[t2 * kMaxN + b];
      uo += B * F[4][b * N + t1];
      gao += B * F[5][b * N + t1];
      gbo += Dd * F[4][b * N + t1];
      gdo += B * F[6][b * N + t1];
      un += B * F[7][b * N + t1];
      gan += B * F[8][b * N + t1];
      gbn += Dd * F[7][b * N + t1];
      gdn += B * F[9][b * N + t1];
    }
    TC xi[3];
    xi[D] = TC(s);
    xi[ax] = T.gx[t1];
    xi[bx] = T.gx[t2];
    TC Jo[3][3], Ao[3][3], deto;
    if (AFF) {  // parallelepiped: the element's constant J, adj J, det J (Gc = 9 + 9 + 1 values)
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          Jo[r][cc] = Gc[3 * r + cc];
          Ao[r][cc] = Gc[9 + 3 * r + cc];
        }
      deto = Gc[18];
    } else {
      face_jacobian<D>(X, s, xi[ax], xi[bx], Jo);
      adj3(Jo, Ao);
      deto = det3(Jo);
    }
    TC gro[3];
    gro[D] = gdo;
    gro[ax] = gao;
    gro[bx] = gbo;
    const TC ideto = TC(1) / deto;
    TC go[3];  // physical gradient, own side: adj^T gr / det
#pragma unroll
    for (int c = 0; c < 3; ++c) go[c] = (Ao[0][c] * gro[0] + Ao[1][c] * gro[1] + Ao[2][c] * gro[2]) * ideto;
    const TC w = T.gw[t1] * T.gw[t2];
    const TC h = D == 0 ? m.hx : (D == 1 ? m.hy : m.hz);
    const TC sig = m.sig_hat / h;
    TC Nv[3];
    const int c1 = (D + 1) % 3, c2 = (D + 2) % 3;
    if (nb >= 0) {
      TC xin[3];
      xin[D] = TC(1 - s);
      xin[ax] = xi[ax];
      xin[bx] = xi[bx];
      TC Jn[3][3], An[3][3];
      if (AFF) {  // the neighbour is a parallelepiped too: J is its three edge vectors
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) Jn[r][cc] = Xn[1 << cc][r] - Xn[0][r];
      } else {
        face_jacobian<D>(Xn, 1 - s, xi[ax], xi[bx], Jn);
      }
      adj3(Jn, An);
      const TC idetn = TC(1) / det3(Jn);
      TC grn[3];
      grn[D] = gdn;
      grn[ax] = gan;
      grn[bx] = gbn;
      TC gn[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) gn[c] = (An[0][c] * grn[0] + An[1][c] * grn[1] + An[2][c] * grn[2]) * idetn;
      // n dS from T^-: the own element on the upper face, the neighbour on the lower face
      const TC (&Jm)[3][3] = s ? Jo : Jn;
      Nv[0] = Jm[1][c1] * Jm[2][c2] - Jm[2][c1] * Jm[1][c2];
      Nv[1] = Jm[2][c1] * Jm[0][c2] - Jm[0][c1] * Jm[2][c2];
      Nv[2] = Jm[0][c1] * Jm[1][c2] - Jm[1][c1] * Jm[0][c2];
      const TC area = sqrt(Nv[0] * Nv[0] + Nv[1] * Nv[1] + Nv[2] * Nv[2]);
      const TC Kn = m.K[nb];
      const TC gam = UNIT ? TC(1) : TC(2) * K * Kn / (K + Kn);
      const TC Jq = s ? uo - un : un - uo;
      const TC Fq = TC(0.5) * gam * w * ((go[0] + gn[0]) * Nv[0] + (go[1] + gn[1]) * Nv[1] + (go[2] + gn[2]) * Nv[2]);
      const TC pen = sig * gam * area * w * Jq;
      P = s ? (pen - Fq) : (Fq - pen);
      const TC cr = -TC(0.5) * gam * w * Jq * ideto;
      TC R[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) R[c] = cr * (Ao[c][0] * Nv[0] + Ao[c][1] * Nv[1] + Ao[c][2] * Nv[2]);
      Ra = R[ax];
      Rb = R[bx];
      Rd = R[D];
      if (PAIR) {  // T^+ side of the same face: the opposite flux-minus-penalty term, and
                   // its symmetry term with its own adj J and det J
        Pn = -P;
        const TC crn = -TC(0.5) * gam * w * Jq * idetn;
#pragma unroll
        for (int c = 0; c < 3; ++c) R[c] = crn * (An[c][0] * Nv[0] + An[c][1] * Nv[1] + An[c][2] * Nv[2]);
        Ran = R[ax];
        Rbn = R[bx];
        Rdn = R[D];
      }
    } else {
      // weak Dirichlet: -K grad u.n v - K grad v.n u + sigma K u v, outward n
      const TC sg = s ? TC(1) : TC(-1);
      Nv[0] = sg * (Jo[1][c1] * Jo[2][c2] - Jo[2][c1] * Jo[1][c2]);
      Nv[1] = sg * (Jo[2][c1] * Jo[0][c2] - Jo[0][c1] * Jo[2][c2]);
      Nv[2] = sg * (Jo[0][c1] * Jo[1][c2] - Jo[1][c1] * Jo[0][c2]);
      const TC area = sqrt(Nv[0] * Nv[0] + Nv[1] * Nv[1] + Nv[2] * Nv[2]);
      const TC Kb = UNIT ? TC(1) : K;
      P = -Kb * w * (go[0] * Nv[0] + go[1] * Nv[1] + go[2] * Nv[2]) + sig * Kb * area * w * uo;
      const TC cr = -Kb * w * uo * ideto;
      TC R[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) R[c] = cr * (Ao[c][0] * Nv[0] + Ao[c][1] * Nv[1] + Ao[c][2] * Nv[2]);
      Ra = R[ax];
      Rb = R[bx];
      Rd = R[D];
    }
    F[0][t] = P;  // F[0..3] were last read before the previous barrier
    F[1][t] = Ra;
    F[2][t] = Rb;
    F[3][t] = Rd;
  }
  if (PAIR) {
    // F[4..9] are read above by every thread of the element, which may span
    // two wavefronts (n^2 not dividing 64): the T^+ rows wait for all of them
    elem_sync<N>();
    if (act) {
      F[4][t] = Pn;
      F[5][t] = Ran;
      F[6][t] = Rbn;
      F[7][t] = Rdn;
    }
  }
  elem_sync<N>();
  // transposed tangential operators, contraction over qb: thread (qa, b) = (t1, t2);
  // rows: own side F[4..6] (PAIR: F[0..2]), neighbour side F[3..5]
  constexpr int O = PAIR ? 0 : 4;
  {
    TC xs = 0, ys = 0, zs = 0, xn = 0, yn = 0, zn = 0;
    if (act) {
#pragma unroll
      for (int qb = 0; qb < N; ++qb) {
        const TC B = T.B[qb * kMaxN + t2], Dd = T.D[qb * kMaxN + t2];
        xs += B * F[0][qb * N + t1] + Dd * F[2][qb * N + t1];
        ys += B * F[1][qb * N + t1];
        zs += B * F[3][qb * N + t1];
        if (PAIR) {
          xn += B * F[4][qb * N + t1] + Dd * F[6][qb * N + t1];
          yn += B * F[5][qb * N + t1];
          zn += B * F[7][qb * N + t1];
        }
      }
    }
    if (PAIR) elem_sync<N>();  // the inputs are overwritten below
    if (act) {
      F[O + 0][t2 * N + t1] = xs;
      F[O + 1][t2 * N + t1] = ys;
      F[O + 2][t2 * N + t1] = zs;
      if (PAIR) {
        F[3][t2 * N + t1] = xn;
        F[4][t2 * N + t1] = yn;
        F[5][t2 * N + t1] = zn;
      }
    }
  }
  elem_sync<N>();
  if (act) {  // contraction over qa: thread (a, b) = (t1, t2) owns face node (a, b) of its line
    TC out = 0, z = 0, outn = 0, zn = 0;
#pragma unroll
    for (int qa = 0; qa < N; ++qa) {
      const TC B = T.B[qa * kMaxN + t1], Dd = T.D[qa * kMaxN + t1];
      out += B * F[O + 0][t2 * N + qa] + Dd * F[O + 1][t2 * N + qa];
      z += B * F[O + 2][t2 * N + qa];
      if (PAIR) {
        outn += B * F[3][t2 * N + qa] + Dd * F[4][t2 * N + qa];
        zn += B * F[5][t2 * N + qa];
      }
    }
    TC yl[N];
    lds_get<N, D, TC, LV>(Y, t1, t2, yl);
#pragma unroll
    for (int i = 0; i < N; ++i) yl[i] += dS[i] * z;
    yl[s ? N - 1 : 0] += out;
    lds_put<N, D, TC, LV>(Y, t1, t2, yl);
    if (PAIR && nb >= 0) {  // the neighbour's line (t1, t2) along D, added by its second pass
      TC* fbn = m.fb + ((int64_t)nb * 3 + D) * 2 * NN;
      // read once, by the second pass: stored nontemporal
      __builtin_nontemporal_store(outn, &fbn[t]);
      __builtin_nontemporal_store(zn, &fbn[NN + t]);
    }
  }
}

// Volume part of the trilinear apply for the thread's element: the element
// tile C receives (B^T (x) B^T (x) B^T)(sum_d Dg_d^T g_d + c w |det J| v) of
// the input x (see the file header), with coefficient K (and the reaction
// coefficients of m, if any); (ex, ey, ez): the element's grid position.
// Xs: the element's corner slot in LDS (filled here).  All threads of the
// block call this (it synchronises).
template <int N, typename TC, typename TIN, bool AFF = false, int LV = 0>
__device__ void tri_volume(const MeshArgs<TC>& m, const Tables<TC>& T, const TIN* __restrict__ x, int64_t e,
                           int ex, int ey, int ez, bool act, int t, int t1, int t2, TC K, TC (&Xs)[8][3], TC* A,
                           TC* B, TC* C) {
  constexpr int NN = N * N;
  if (act) {
    TC uz[N];
    for (int q = t; q < 24; q += NN) corner_at(m, ex, ey, ez, q / 3, q % 3, Xs[q / 3][q % 3]);
    glb_get<N, 2, TC, TIN>(x, e, t1, t2, uz);
    TC a[N];
    contract_eo<N, TC, 1>(T.eB, uz, a);  // phase Z: interpolate along z
    lds_put<N, 2, TC, LV>(A, t1, t2, a);
  }
  elem_sync<N>();
  const TC (&X)[8][3] = Xs;
  if (act) {  // phase Y
    TC a[N], b[N];
    lds_get<N, 1, TC, LV>(A, t1, t2, a);
    contract_eo<N, TC, 1>(T.eB, a, b);
    lds_put<N, 1, TC, LV>(B, t1, t2, b);
  }
  elem_sync<N>();
  if (act) {  // phase X: v and d/dxi_0
    TC a[N], v[N], d1[N];
    lds_get<N, 0, TC, LV>(B, t1, t2, a);
    contract_eo<N, TC, 1>(T.eB, a, v);
    contract_eo<N, TC, -1>(T.eDg, v, d1);
    lds_put<N, 0, TC, LV>(A, t1, t2, v);
    lds_put<N, 0, TC, LV>(C, t1, t2, d1);
  }
  elem_sync<N>();
  if (act) {  // phase Y': d/dxi_1
    TC v[N], d2[N];
    lds_get<N, 1, TC, LV>(A, t1, t2, v);
    contract_eo<N, TC, -1>(T.eDg, v, d2);
    lds_put<N, 1, TC, LV>(B, t1, t2, d2);
  }
  elem_sync<N>();
  if (act) {  // phase Z': d/dxi_2, geometry, g = G gr, Dg_z^T g_2
    TC d1[N], d2[N], d3[N], wz[N], v[N];
    lds_get<N, 2, TC, LV>(A, t1, t2, v);
    contract_eo<N, TC, -1>(T.eDg, v, d3);
    lds_get<N, 2, TC, LV>(C, t1, t2, d1);
    lds_get<N, 2, TC, LV>(B, t1, t2, d2);
    const TC wq12 = T.gw[t1] * T.gw[t2] * K;
    const TC cw12 = m.R ? m.R[e] * T.gw[t1] * T.gw[t2] : TC(0);  // reaction weight
    TC G0[3][3], dJ0 = TC(1);
    if (AFF) {  // parallelepiped: adj adj^T / |det J| and |det J| are the same at every point
      const TC xi[3] = {TC(0.5), TC(0.5), TC(0.5)};
      TC J[3][3], Aj[3][3];
      trilinear_jacobian(X, xi, J);
      adj3(J, Aj);
      dJ0 = fabs(det3(J));
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int cc = r; cc < 3; ++cc) {
          G0[r][cc] = (Aj[r][0] * Aj[cc][0] + Aj[r][1] * Aj[cc][1] + Aj[r][2] * Aj[cc][2]) / dJ0;
          G0[cc][r] = G0[r][cc];
        }
    }
    const JacZLine<TC> jz(X, T.gx[t1], T.gx[t2]);  // unused (and dropped) for AFF
#pragma unroll
    for (int q = 0; q < N; ++q) {
      TC Gm[3][3];
      if (AFF) {
        const TC c = wq12 * T.gw[q];
        v[q] *= cw12 * T.gw[q] * dJ0;  // reaction c w |det J| u at the point
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) Gm[r][cc] = c * G0[r][cc];
      } else {
        TC J[3][3], Aj[3][3];
        jz.at(T.gx[q], J);
        adj3(J, Aj);
        const TC dJ = fabs(det3(J));
        const TC c = wq12 * T.gw[q] / dJ;
        v[q] *= cw12 * T.gw[q] * dJ;  // reaction c w |det J| u at the point
        // G = c adj adj^T (symmetric)
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int cc = r; cc < 3; ++cc) {
            const TC sgm = Aj[r][0] * Aj[cc][0] + Aj[r][1] * Aj[cc][1] + Aj[r][2] * Aj[cc][2];
            Gm[r][cc] = c * sgm;
            Gm[cc][r] = c * sgm;
          }
      }
      const TC a1 = d1[q], a2 = d2[q], a3 = d3[q];  // G gr in place of gr
      d1[q] = Gm[0][0] * a1 + Gm[0][1] * a2 + Gm[0][2] * a3;
      d2[q] = Gm[1][0] * a1 + Gm[1][1] * a2 + Gm[1][2] * a3;
      d3[q] = Gm[2][0] * a1 + Gm[2][1] * a2 + Gm[2][2] * a3;
    }
    contract_eo<N, TC, -1>(T.eDgt, d3, wz);
#pragma unroll
    for (int q = 0; q < N; ++q) wz[q] += v[q];
    lds_put<N, 2, TC, LV>(A, t1, t2, wz);
    lds_put<N, 2, TC, LV>(C, t1, t2, d1);
    lds_put<N, 2, TC, LV>(B, t1, t2, d2);
  }
  elem_sync<N>();
  if (act) {  // phase Y'': += Dg_y^T g_1
    TC g2[N], w[N], r[N];
    lds_get<N, 1, TC, LV>(B, t1, t2, g2);
    lds_get<N, 1, TC, LV>(A, t1, t2, w);
    contract_eo<N, TC, -1>(T.eDgt, g2, r);
#pragma unroll
    for (int i = 0; i < N; ++i) w[i] += r[i];
    lds_put<N, 1, TC, LV>(A, t1, t2, w);
  }
  elem_sync<N>();
  if (act) {  // phase X'': += Dg_x^T g_0, then B_x^T
    TC g1[N], w[N], r[N], o[N];
    lds_get<N, 0, TC, LV>(C, t1, t2, g1);
    lds_get<N, 0, TC, LV>(A, t1, t2, w);
    contract_eo<N, TC, -1>(T.eDgt, g1, r);
#pragma unroll
    for (int i = 0; i < N; ++i) w[i] += r[i];
    contract_eo<N, TC, 1>(T.eBt, w, o);
    lds_put<N, 0, TC, LV>(A, t1, t2, o);
  }
  elem_sync<N>();
  if (act) {  // phase Y''': B_y^T
    TC w[N], o[N];
    lds_get<N, 1, TC, LV>(A, t1, t2, w);
    contract_eo<N, TC, 1>(T.eBt, w, o);
    lds_put<N, 1, TC, LV>(A, t1, t2, o);
  }
  elem_sync<N>();
  if (act) {  // phase Z''': B_z^T -> accumulator C
    TC w[N], o[N];
    lds_get<N, 2, TC, LV>(A, t1, t2, w);
    contract_eo<N, TC, 1>(T.eBt, w, o);
    lds_put<N, 2, TC, LV>(C, t1, t2, o);
  }
}

// The T^+ side of the lower face (D, 0) of element e on the thread's line
// along D at (t1, t2), added to the element tile C: z l'(0) on the line, the
// trace term on node 0 (the two scalars left in m.fb by the first pass).
template <int N, int D, typename TC>
__device__ __forceinline__ void lower_line(const MeshArgs<TC>& m, const Tables<TC>& T, int64_t e, int t1, int t2,
                                           TC* C) {
  constexpr int NN = N * N;
  const TC* fb = m.fb + ((int64_t)e * 3 + D) * 2 * NN;
  const int t = t1 + N * t2;
  const TC out = fb[t], z = fb[NN + t];
  TC yl[N];
  lds_get<N, D>(C, t1, t2, yl);
#pragma unroll
  for (int i = 0; i < N; ++i) yl[i] += T.d0[i] * z;
  yl[0] += out;
  lds_put<N, D>(C, t1, t2, yl);
}

// First pass of the trilinear apply: y_T = volume part + the element's three
// upper faces (evaluated once for both of their elements; the T^+ side goes
// to m.fb) + its lower faces on a Dirichlet boundary.  The second pass
// (k_tri_lower) adds the lower interior faces from m.fb.
// Waves per SIMD the first pass asks the register allocator for: three in
// FP64 at n = 5, 6, where the face rows sharing the volume scratch tiles
// leave LDS for three workgroups per CU (n = 6: 8% faster than with two;
// at n = 7, 8 the registers would spill and the pass ran slower); five in
// FP32 from n = 6 on (at most 96 VGPRs instead of 97-104; LDS leaves room
// for five workgroups; 48^3 Q7 1-2% faster, 26^3 Q5 up to 4%)
__host__ __device__ constexpr int tri_min_waves(int n, int bytes) {
  return bytes == 8 && (n == 5 || n == 6) ? 3 : (bytes == 4 && n >= 6 ? 5 : 1);
}

template <int N, typename TIN, typename TOUT, typename TC, bool AFF>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(tri_min_waves(N, sizeof(TC))))) void k_apply_trilinear(MeshArgs<TC> m, const TIN* __restrict__ x,
                                                            TOUT* __restrict__ y, const int* skip) {
  // FP64 at n = 4: tiles of stride 80 (no more modelled bank conflicts) hold
  // the face rows, which then need no LDS area of their own (55.8 -> 36.9 KB
  // per workgroup: three workgroups per CU instead of two)
  constexpr int LV = (N == 4 && sizeof(TC) == 8) ? 2 : 0;
  constexpr int NN = N * N, N3 = NN * N, EPB = elems_per_block(N), PE = Lay<N, TC, LV>::PE;
  // the face rows (10 n^2 per element) live in the volume scratch tiles A, B
  // once the volume term is done, when they fit there (n >= 5)
  constexpr bool F_IN_AB = 10 * NN <= 2 * PE;
  __shared__ TC sAB[2 * EPB * PE], sC[EPB * PE];
  __shared__ TC sX[EPB][8][3], sXn[EPB][8][3];
  __shared__ TC sFx[F_IN_AB ? 1 : EPB * 10 * NN];
  if (skip != nullptr && *skip) return;
  const Tables<TC>& T = *m.tab;
  const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
  const int tid = threadIdx.x, el = tid / NN, t = tid % NN, t1 = t % N, t2 = t / N;
  const int64_t e = blk * EPB + el;
  const bool act = (el < EPB) && (e < m.E);
  const int le = act ? el : 0;
  TC* A = sAB + le * PE;
  TC* B = sAB + (EPB + le) * PE;
  TC* C = sC + le * PE;
  TC(*F)[NN] = (TC(*)[NN])((F_IN_AB ? sAB : sFx) + le * 10 * NN);
  int ex = 0, ey = 0, ez = 0;
  TC K = TC(1);
  if (act) {
    ex = (int)(e % m.nx);
    ey = (int)((e / m.nx) % m.ny);
    ez = (int)(e / ((int64_t)m.nx * m.ny));
    K = m.K[e];
  }
  tri_volume<N, TC, TIN, AFF, LV>(m, T, x, e, ex, ey, ez, act, t, t1, t2, K, sX[le], A, B, C);
  // F_IN_AB: the face rows of an element overlap other elements' scratch tiles
  if (F_IN_AB) __syncthreads();
  const TC (&X)[8][3] = sX[le];
  TC Gc[19];  // AFF: constant J, adj J, det J of the element
  if (AFF) {
    const TC xi[3] = {TC(0.5), TC(0.5), TC(0.5)};
    TC J[3][3], Aj[3][3];
    trilinear_jacobian(X, xi, J);
    adj3(J, Aj);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        Gc[3 * r + cc] = J[r][cc];
        Gc[9 + 3 * r + cc] = Aj[r][cc];
      }
    Gc[18] = det3(J);
  }
  // upper faces for both sides; lower faces only where there is no element below
  // (each call synchronises before touching shared buffers)
  const bool bx0 = act && neighbour<0>(m, ex, ey, ez, 0) < 0;
  const bool by0 = act && neighbour<1>(m, ex, ey, ez, 0) < 0;
  const bool bz0 = act && neighbour<2>(m, ex, ey, ez, 0) < 0;
  face_term<N, 0, TC, TIN, false, AFF, true, LV>(m, T, x, e, ex, ey, ez, X, sXn[le], K, t1, t2, C, F, act, 1, Gc);
  face_term<N, 0, TC, TIN, false, AFF, false, LV>(m, T, x, e, ex, ey, ez, X, sXn[le], K, t1, t2, C, F, bx0, 0, Gc);
  elem_sync<N>();
  face_term<N, 1, TC, TIN, false, AFF, true, LV>(m, T, x, e, ex, ey, ez, X, sXn[le], K, t1, t2, C, F, act, 1, Gc);
  face_term<N, 1, TC, TIN, false, AFF, false, LV>(m, T, x, e, ex, ey, ez, X, sXn[le], K, t1, t2, C, F, by0, 0, Gc);
  elem_sync<N>();
  face_term<N, 2, TC, TIN, false, AFF, true, LV>(m, T, x, e, ex, ey, ez, X, sXn[le], K, t1, t2, C, F, act, 1, Gc);
  face_term<N, 2, TC, TIN, false, AFF, false, LV>(m, T, x, e, ex, ey, ez, X, sXn[le], K, t1, t2, C, F, bz0, 0, Gc);
  elem_sync<N>();
  if (act) {
    TC o[N];
    lds_get<N, 2, TC, LV>(C, t1, t2, o);
    TOUT* py = y + e * N3;
#pragma unroll
    // y and the face buffer are not read again in this pass: nontemporal
    // stores leave L2 to the x lines the face phases re-read
    for (int i = 0; i < N; ++i) __builtin_nontemporal_store((TOUT)o[i], &py[lidx<N, 2>(t1, t2, i)]);
  }
}

// Second pass: y_T += the T^+ side of each interior lower face of T, from the
// line scalars the first pass left in m.fb (its line along d at (t1, t2):
// l_i'(0) z added to every node, the trace term to node 0).  DOT: block
// partials of <x, y> for the CG.
template <int N, typename TIN, typename TOUT, typename TC, bool DOT>
__global__ __launch_bounds__(kBlock) void k_tri_lower(MeshArgs<TC> m, const TIN* __restrict__ x,
                                                      TOUT* __restrict__ y, double* partials, const int* skip) {
  constexpr int NN = N * N, N3 = NN * N, EPB = elems_per_block(N), PE = Lay<N, TC>::PE;
  __shared__ TC sC[EPB * PE];
  __shared__ double red[kBlock / 64];
  if (skip != nullptr && *skip) return;
  const Tables<TC>& T = *m.tab;
  const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
  const int tid = threadIdx.x, el = tid / NN, t = tid % NN, t1 = t % N, t2 = t / N;
  const int64_t e = blk * EPB + el;
  const bool act = (el < EPB) && (e < m.E);
  const int le = act ? el : 0;
  TC* C = sC + le * PE;
  int ex = 0, ey = 0, ez = 0;
  TOUT* py = y + e * N3;
  if (act) {
    ex = (int)(e % m.nx);
    ey = (int)((e / m.nx) % m.ny);
    ez = (int)(e / ((int64_t)m.nx * m.ny));
    TC o[N];
#pragma unroll
    for (int i = 0; i < N; ++i) o[i] = (TC)py[lidx<N, 2>(t1, t2, i)];
    lds_put<N, 2>(C, t1, t2, o);
  }
  elem_sync<N>();
  if (act && neighbour<0>(m, ex, ey, ez, 0) >= 0) lower_line<N, 0>(m, T, e, t1, t2, C);
  elem_sync<N>();
  if (act && neighbour<1>(m, ex, ey, ez, 0) >= 0) lower_line<N, 1>(m, T, e, t1, t2, C);
  elem_sync<N>();
  if (act && neighbour<2>(m, ex, ey, ez, 0) >= 0) lower_line<N, 2>(m, T, e, t1, t2, C);
  elem_sync<N>();
  double part = 0.0;
  if (act) {
    TC o[N], uz[N];
    lds_get<N, 2>(C, t1, t2, o);
    if (DOT) glb_get<N, 2, TC, TIN>(x, e, t1, t2, uz);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const TOUT v = (TOUT)o[i];
      __builtin_nontemporal_store(v, &py[lidx<N, 2>(t1, t2, i)]);
      if (DOT) part += (double)uz[i] * (double)v;
    }
  }
  if (DOT) {
    const double mine[1] = {block_sum<kBlock>(part, red)};
    store_partials<1>(mine, partials, blockIdx.x);
  }
}

// ---------------------------------------------------------------- dA / dtheta
// Per element T, with u and v: parts[7 T] = u_T . (volume form of T with
// K = 1) v_T and parts[7 T + 1 + 2 d + s] = u_T . (rows of T of the face form
// of face (d, s) with unit coefficient) v.  The reaction term does not depend
// on theta and is left out.
template <int N>
__global__ __launch_bounds__(kBlock) void k_dA_parts_trilinear(MeshArgs<double> m, const double* __restrict__ u,
                                                               const double* __restrict__ v,
                                                               double* __restrict__ parts) {
  constexpr int NN = N * N, EPB = elems_per_block(N), PE = Lay<N, double>::PE;
  __shared__ double sA[EPB * PE], sB[EPB * PE], sC[EPB * PE];
  __shared__ double sX[EPB][8][3], sXn[EPB][8][3];
  __shared__ double sF[EPB][10][NN];
  __shared__ double sRed[kBlock];
  const Tables<double>& T = *m.tab;
  const int tid = threadIdx.x, el = tid / NN, t = tid % NN, t1 = t % N, t2 = t / N;
  const int64_t e = (int64_t)blockIdx.x * EPB + el;
  const bool act = (el < EPB) && (e < m.E);
  const int le = act ? el : 0;
  double* A = sA + le * PE;
  double* B = sB + le * PE;
  double* C = sC + le * PE;
  int ex = 0, ey = 0, ez = 0;
  if (act) {
    ex = (int)(e % m.nx);
    ey = (int)((e / m.nx) % m.ny);
    ez = (int)(e / ((int64_t)m.nx * m.ny));
  }
  MeshArgs<double> m1 = m;
  m1.R = nullptr;
  tri_volume<N, double, double>(m1, T, v, e, ex, ey, ez, act, t, t1, t2, 1.0, sX[le], A, B, C);
  const double (&X)[8][3] = sX[le];
  double uz[N];
  if (act) glb_get<N, 2, double, double>(u, e, t1, t2, uz);
  // u_T . C for the thread's element, then C = 0 (deterministic: per-thread
  // partial sums, added in thread order by the element's first thread)
  auto take = [&](int slot) {
    elem_sync<N>();
    double p = 0.0;
    if (act) {
      double c[N], z[N];
      lds_get<N, 2>(C, t1, t2, c);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        p += uz[i] * c[i];
        z[i] = 0.0;
      }
      lds_put<N, 2>(C, t1, t2, z);
    }
    sRed[tid] = p;
    elem_sync<N>();
    if (act && t == 0) {
      double s = 0.0;
      for (int j = 0; j < NN; ++j) s += sRed[el * NN + j];
      parts[7 * e + slot] = s;
    }
  };
  take(0);
  face_term<N, 0, double, double, true>(m1, T, v, e, ex, ey, ez, X, sXn[le], 1.0, t1, t2, C, sF[le], act, 0);
  take(1);
  face_term<N, 0, double, double, true>(m1, T, v, e, ex, ey, ez, X, sXn[le], 1.0, t1, t2, C, sF[le], act, 1);
  take(2);
  face_term<N, 1, double, double, true>(m1, T, v, e, ex, ey, ez, X, sXn[le], 1.0, t1, t2, C, sF[le], act, 0);
  take(3);
  face_term<N, 1, double, double, true>(m1, T, v, e, ex, ey, ez, X, sXn[le], 1.0, t1, t2, C, sF[le], act, 1);
  take(4);
  face_term<N, 2, double, double, true>(m1, T, v, e, ex, ey, ez, X, sXn[le], 1.0, t1, t2, C, sF[le], act, 0);
  take(5);
  face_term<N, 2, double, double, true>(m1, T, v, e, ex, ey, ez, X, sXn[le], 1.0, t1, t2, C, sF[le], act, 1);
  take(6);
}

// g_T = K_T parts[T][0] + sum over faces (d, s) of dgamma/dtheta_T times the
// whole unit-coefficient face form: the rows of T (parts of T) plus the rows
// of the neighbour N (parts of N for its face (d, 1 - s)).
// dgamma/dtheta_T = gamma K_N / (K_T + K_N) on interior faces, K_T on boundary faces.
__global__ __launch_bounds__(256) void k_dA_combine_trilinear(MeshArgs<double> m, const double* __restrict__ parts,
                                                              double* __restrict__ g) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.E) return;
  const int ex = (int)(e % m.nx), ey = (int)((e / m.nx) % m.ny), ez = (int)(e / ((int64_t)m.nx * m.ny));
  const double K = m.K[e];
  double acc = K * parts[7 * e];
  for (int d = 0; d < 3; ++d)
    for (int s = 0; s < 2; ++s) {
      int64_t nb;
      if (d == 0) nb = neighbour<0>(m, ex, ey, ez, s);
      else if (d == 1) nb = neighbour<1>(m, ex, ey, ez, s);
      else nb = neighbour<2>(m, ex, ey, ez, s);
      const double own = parts[7 * e + 1 + 2 * d + s];
      if (nb < 0) {
        acc += K * own;
      } else {
        const double Kn = m.K[nb];
        const double gam = 2.0 * K * Kn / (K + Kn);
        acc += gam * Kn / (K + Kn) * (own + parts[7 * nb + 1 + 2 * d + (1 - s)]);
      }
    }
  g[e] = acc;
}

// ---------------------------------------------------------------- diagonal
// one block per element: G_q of every volume point into LDS, then one thread
// per DOF sums gr_i^T G_q gr_i over the points, plus the face terms of the
// face-layer DOFs (a_e(phi_i, phi_i) with phi_i on its own side).
template <int N>
__global__ __launch_bounds__(512) void k_diag_trilinear(MeshArgs<double> m, double* __restrict__ d,
                                                        const int* run) {
  constexpr int NN = N * N, N3 = NN * N;
  __shared__ double G[N3][7];
  if (run != nullptr && *run == 0) return;
  const int64_t e = blockIdx.x;
  const int t = threadIdx.x;
  const Tables<double>& T = *m.tab;
  double X[8][3];
  element_corners(m, e, X);
  const double K = m.K[e];
  if (t < N3) {
    const int q1 = t % N, q2 = (t / N) % N, q3 = t / NN;
    const double xi[3] = {T.gx[q1], T.gx[q2], T.gx[q3]};
    double J[3][3], Aj[3][3];
    trilinear_jacobian(X, xi, J);
    adj3(J, Aj);
    const double c = T.gw[q1] * T.gw[q2] * T.gw[q3] * K / fabs(det3(J));
    int k = 0;
    for (int r = 0; r < 3; ++r)
      for (int cc = r; cc < 3; ++cc)
        G[t][k++] = c * (Aj[r][0] * Aj[cc][0] + Aj[r][1] * Aj[cc][1] + Aj[r][2] * Aj[cc][2]);
    G[t][6] = m.R ? m.R[e] * T.gw[q1] * T.gw[q2] * T.gw[q3] * fabs(det3(J)) : 0.0;  // reaction
  }
  __syncthreads();  // G is shared by the whole block
  if (t >= N3) return;
  const int i1 = t % N, i2 = (t / N) % N, i3 = t / NN;
  const int ii[3] = {i1, i2, i3};
  double acc = 0.0;
  for (int q3 = 0; q3 < N; ++q3)
    for (int q2 = 0; q2 < N; ++q2)
      for (int q1 = 0; q1 < N; ++q1) {
        const double b1 = T.B[q1 * kMaxN + i1], b2 = T.B[q2 * kMaxN + i2], b3 = T.B[q3 * kMaxN + i3];
        const double g0 = T.D[q1 * kMaxN + i1] * b2 * b3;
        const double g1 = b1 * T.D[q2 * kMaxN + i2] * b3;
        const double g2 = b1 * b2 * T.D[q3 * kMaxN + i3];
        const double* Gq = G[q1 + N * (q2 + N * q3)];
        acc += Gq[0] * g0 * g0 + Gq[3] * g1 * g1 + Gq[5] * g2 * g2 +
               2.0 * (Gq[1] * g0 * g1 + Gq[2] * g0 * g2 + Gq[4] * g1 * g2) + Gq[6] * (b1 * b2 * b3) * (b1 * b2 * b3);
      }
  const int ex = (int)(e % m.nx), ey = (int)((e / m.nx) % m.ny), ez = (int)(e / ((int64_t)m.nx * m.ny));
  for (int D = 0; D < 3; ++D) {
    const int ax = (D == 0) ? 1 : 0, bx = (D == 2) ? 1 : 2;
    const int c1 = (D + 1) % 3, c2 = (D + 2) % 3;
    const double h = D == 0 ? m.hx : (D == 1 ? m.hy : m.hz);
    const double sig = m.sig_hat / h;
    for (int s = 0; s < 2; ++s) {
      int64_t nb;
      if (D == 0) nb = neighbour<0>(m, ex, ey, ez, s);
      else if (D == 1) nb = neighbour<1>(m, ex, ey, ez, s);
      else nb = neighbour<2>(m, ex, ey, ez, s);
      const bool self = (nb == e);
      if (self && s == 0) continue;  // the element's own periodic face: once
      const int end = s ? N - 1 : 0;
      if (!self && ii[D] != end) continue;
      double gam = K;
      if (nb >= 0) {
        const double Kn = m.K[nb];
        gam = 2.0 * K * Kn / (K + Kn);
      }
      for (int qb = 0; qb < N; ++qb)
        for (int qa = 0; qa < N; ++qa) {
          const double w = T.gw[qa] * T.gw[qb];
          // value and physical gradient of phi_i on this element at xi_D = side
          auto eval = [&](int side, double& val, double (&g)[3], double (&Jc)[3][3]) {
            double xi[3];
            xi[D] = side;
            xi[ax] = T.gx[qa];
            xi[bx] = T.gx[qb];
            double Aj[3][3];
            trilinear_jacobian(X, xi, Jc);
            adj3(Jc, Aj);
            const double det = det3(Jc);
            const double* dE = side ? T.d1 : T.d0;
            const double la = T.B[qa * kMaxN + ii[ax]], lb = T.B[qb * kMaxN + ii[bx]];
            const double le = (ii[D] == (side ? N - 1 : 0)) ? 1.0 : 0.0;
            val = le * la * lb;
            double gr[3];
            gr[D] = dE[ii[D]] * la * lb;
            gr[ax] = le * T.D[qa * kMaxN + ii[ax]] * lb;
            gr[bx] = le * la * T.D[qb * kMaxN + ii[bx]];
            for (int c = 0; c < 3; ++c) g[c] = (Aj[0][c] * gr[0] + Aj[1][c] * gr[1] + Aj[2][c] * gr[2]) / det;
          };
          double v1, gA[3], J1[3][3];
          eval(s, v1, gA, J1);
          double Nv[3];
          Nv[0] = J1[1][c1] * J1[2][c2] - J1[2][c1] * J1[1][c2];
          Nv[1] = J1[2][c1] * J1[0][c2] - J1[0][c1] * J1[2][c2];
          Nv[2] = J1[0][c1] * J1[1][c2] - J1[1][c1] * J1[0][c2];
          const double area = sqrt(Nv[0] * Nv[0] + Nv[1] * Nv[1] + Nv[2] * Nv[2]);
          if (self) {  // phi_i on both sides of the face: [phi] = phi(1) - phi(0)
            double v0, gB[3], J0[3][3];
            eval(0, v0, gB, J0);
            const double jump = v1 - v0;
            const double avg = 0.5 * gam * ((gA[0] + gB[0]) * Nv[0] + (gA[1] + gB[1]) * Nv[1] + (gA[2] + gB[2]) * Nv[2]);
            acc += w * (-2.0 * avg * jump + sig * gam * area * jump * jump);
          } else if (nb >= 0) {
            const double fl = gA[0] * Nv[0] + gA[1] * Nv[1] + gA[2] * Nv[2];
            const double sg = s ? -1.0 : 1.0;  // [phi] = +phi on the upper face, -phi on the lower
            acc += w * (sg * gam * fl * v1 + sig * gam * area * v1 * v1);
          } else {
            const double sg = s ? 1.0 : -1.0;  // outward normal
            const double fl = sg * (gA[0] * Nv[0] + gA[1] * Nv[1] + gA[2] * Nv[2]);
            acc += w * (-2.0 * K * fl * v1 + sig * K * area * v1 * v1);
          }
        }
    }
  }
  d[e * N3 + t] = acc;
}

// ---------------------------------------------------------------- launchers
template <int N, typename TIN, typename TOUT, typename TC, bool DOT>
static hipError_t run_tri(const MeshArgs<TC>& m, const void* x, void* y, double* partials, CgState* st, int par,
                          const int* skip, hipStream_t s) {
  const int64_t nb = element_blocks(N, m.E);
  if (m.affg)
    hipLaunchKernelGGL((k_apply_trilinear<N, TIN, TOUT, TC, true>), dim3((unsigned)nb), dim3(kBlock), 0, s, m,
                       (const TIN*)x, (TOUT*)y, skip);
  else
    hipLaunchKernelGGL((k_apply_trilinear<N, TIN, TOUT, TC, false>), dim3((unsigned)nb), dim3(kBlock), 0, s, m,
                       (const TIN*)x, (TOUT*)y, skip);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_tri_lower<N, TIN, TOUT, TC, DOT>), dim3((unsigned)nb), dim3(kBlock), 0, s, m, (const TIN*)x,
                     (TOUT*)y, partials, skip);
  e = hipGetLastError();
  if (e != hipSuccess || !DOT || st == nullptr) return e;  // st == nullptr: partials only
  return launch_finish_dot(partials, nb, st, par, s);
}

template <int N, bool DOT>
static hipError_t run_tri_prec(int prec, const MeshArgs<double>& m64, const MeshArgs<float>& m32, const void* x,
                               void* y, double* partials, CgState* st, int par, const int* skip, hipStream_t s) {
  switch (prec) {
    case 0: return run_tri<N, double, double, double, DOT>(m64, x, y, partials, st, par, skip, s);
    case 1: return run_tri<N, float, float, float, DOT>(m32, x, y, partials, st, par, skip, s);
    case 2: return run_tri<N, uint16_t, float, float, DOT>(m32, x, y, partials, st, par, skip, s);
  }
  return hipErrorInvalidValue;
}

template <int N>
static hipError_t run_tri_n(int prec, int dot, const MeshArgs<double>& m64, const MeshArgs<float>& m32,
                            const void* x, void* y, double* partials, CgState* st, int par, const int* skip,
                            hipStream_t s) {
  if (dot) return run_tri_prec<N, true>(prec, m64, m32, x, y, partials, st, par, skip, s);
  return run_tri_prec<N, false>(prec, m64, m32, x, y, partials, st, par, skip, s);
}

hipError_t launch_apply_trilinear(int n, int prec, int trans, int dot, const MeshArgs<double>& m64,
                                  const MeshArgs<float>& m32, const void* x, void* y, double* partials,
                                  CgState* st, int par, const int* skip, hipStream_t s) {
  (void)trans;  // symmetric form: A^T x is evaluated by the same kernel
  switch (n) {
    case 2: return run_tri_n<2>(prec, dot, m64, m32, x, y, partials, st, par, skip, s);
    case 3: return run_tri_n<3>(prec, dot, m64, m32, x, y, partials, st, par, skip, s);
    case 4: return run_tri_n<4>(prec, dot, m64, m32, x, y, partials, st, par, skip, s);
    case 5: return run_tri_n<5>(prec, dot, m64, m32, x, y, partials, st, par, skip, s);
    case 6: return run_tri_n<6>(prec, dot, m64, m32, x, y, partials, st, par, skip, s);
    case 7: return run_tri_n<7>(prec, dot, m64, m32, x, y, partials, st, par, skip, s);
    case 8: return run_tri_n<8>(prec, dot, m64, m32, x, y, partials, st, par, skip, s);
  }
  return hipErrorInvalidValue;
}

template <int N>
static hipError_t run_tri_diag(const MeshArgs<double>& m, double* d, const int* run, hipStream_t s) {
  const int th = ((N * N * N + 63) / 64) * 64;
  hipLaunchKernelGGL((k_diag_trilinear<N>), dim3((unsigned)m.E), dim3(th), 0, s, m, d, run);
  return hipGetLastError();
}
template <int N>
static hipError_t run_dA_tri(const MeshArgs<double>& m, const double* u, const double* v, double* parts, double* g,
                             hipStream_t s) {
  const int64_t nb = element_blocks(N, m.E);
  hipLaunchKernelGGL((k_dA_parts_trilinear<N>), dim3((unsigned)nb), dim3(kBlock), 0, s, m, u, v, parts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dA_combine_trilinear, dim3((unsigned)((m.E + 255) / 256)), dim3(256), 0, s, m, parts, g);
  return hipGetLastError();
}

hipError_t launch_dA_trilinear(int n, const MeshArgs<double>& m, const double* u, const double* v, double* parts,
                               double* g, hipStream_t s) {
  switch (n) {
    case 2: return run_dA_tri<2>(m, u, v, parts, g, s);
    case 3: return run_dA_tri<3>(m, u, v, parts, g, s);
    case 4: return run_dA_tri<4>(m, u, v, parts, g, s);
    case 5: return run_dA_tri<5>(m, u, v, parts, g, s);
    case 6: return run_dA_tri<6>(m, u, v, parts, g, s);
    case 7: return run_dA_tri<7>(m, u, v, parts, g, s);
    case 8: return run_dA_tri<8>(m, u, v, parts, g, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_diag_trilinear(int n, const MeshArgs<double>& m, double* d, const int* run, hipStream_t s) {
  switch (n) {
    case 2: return run_tri_diag<2>(m, d, run, s);
    case 3: return run_tri_diag<3>(m, d, run, s);
    case 4: return run_tri_diag<4>(m, d, run, s);
    case 5: return run_tri_diag<5>(m, d, run, s);
    case 6: return run_tri_diag<6>(m, d, run, s);
    case 7: return run_tri_diag<7>(m, d, run, s);
    case 8: return run_tri_diag<8>(m, d, run, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace dg
