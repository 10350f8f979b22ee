// dg_affine.hip -- sum-factorised SWIPDG apply on affine (axis-parallel box)
// elements: y = A x, its transpose, the Jacobi diagonal and the coefficient
// sensitivity u^T (dA/dtheta_T) v.
//
// Operator (Sec. 4.1, SWIPDG forms b_h and b_h^e) on a box element with
// constant K: it is a sum over the three axes of tensor products
//
//     A = sum_d  M_t1 (x) M_t2 (x) L_d ,
//
// where M is the 1D mass matrix along the two tangential axes and L_d the 1D
// DG operator along axis d: K h_t1 h_t2 / h_d S plus the face terms of the two
// faces normal to d (consistency, symmetry and penalty terms, harmonic
// gamma_e).  The face terms of a line only need the two neighbouring lines
// along d (trace u at the shared end and normal derivative l'(end) . line), so
// every thread owns one line of an element in each of the three orientations
// and the tangential masses are applied afterwards in the same sum
// factorisation as the volume term (Sec. 3.3: matrix-free, sum-factorised,
// no gather/scatter: the kernels index the global element-blocked vectors).
//
// Layout: block = elems_per_block(n) consecutive elements (after the XCD
// remap), n^2 threads per element; per element three n^3 LDS tiles.
//
//   phase Z : own z-lines from HBM, z-neighbour lines   -> bz = L_z u
//   phase Y : own y-lines from LDS, y-neighbour lines   -> by = L_y u
//   phase X : own x-lines from LDS, x-neighbour lines   -> bx = L_x u,
//             c = M_x by, e = M_x bz
//   phase Y2: f = M_y bx + c, g = M_y e
//   phase Z2: y = M_z f + g -> HBM
//
// so that y = M_z (M_y bx + M_x by) + M_y M_x bz.
#include "dg_internal.hpp"
#include "dg_kernels.hpp"
#include "dg_lines.hpp"

namespace dg {

// 1D SWIPDG operator on one line:  b = L u  (TRANS: b = L^T u), with
//   volume   K (At / h) S u                      (At = h_t1 h_t2, h = h_d)
//   upper face (this element is T^-):  J = u[n-1] - uH[0],
//       F = cF (G^- + G^+),  G^- = d1.u / h,  G^+ = d0.uH / h
//       b[n-1] += At (-F + aP J),   b[i] -= At cC d1[i] J
//   lower face (this element is T^+):  J = uL[n-1] - u[0],
//       F = cF (G^- + G^+),  G^- = d1.uL / h,  G^+ = d0.u / h
//       b[0]   += At (F - aP J),    b[i] -= At cC d0[i] J
// interior faces: gamma = 2 K K' / (K + K'), cF = gamma/2, aP = sigma gamma,
// cC = gamma / (2h); Dirichlet faces: neighbour terms 0, cF = K, aP = sigma K,
// cC = K / h.  The transpose swaps the roles of cF / h and cC.
template <int N, typename TC, bool TRANS>
__device__ __forceinline__ void line_op(const Tables<TC>& T, const TC (&u)[N], const TC (&uL)[N],
                                        const TC (&uH)[N], bool hasL, bool hasH, TC K, TC KL, TC KH,
                                        TC h, TC At, TC sig_hat, bool faces, TC (&b)[N]) {
  const TC vs = K * At / h;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    TC s = TC(0);
#pragma unroll
    for (int j = 0; j < N; ++j) s += (TRANS ? T.S[j * kMaxN + i] : T.S[i * kMaxN + j]) * u[j];
    b[i] = vs * s;
  }
  if (!faces) return;
  const TC ih = TC(1) / h;
  const TC sig = sig_hat * ih;
  {  // upper face
    TC Gm = TC(0), Gp = TC(0);
#pragma unroll
    for (int j = 0; j < N; ++j) Gm += T.d1[j] * u[j];
    TC Up = TC(0), aF, aP, aC;
    if (hasH) {
#pragma unroll
      for (int j = 0; j < N; ++j) Gp += T.d0[j] * uH[j];
      Up = uH[0];
      const TC g = TC(2) * K * KH / (K + KH);
      aF = TC(0.5) * g;
      aP = sig * g;
      aC = TC(0.5) * g * ih;
    } else {
      aF = K;
      aP = sig * K;
      aC = K * ih;
    }
    const TC cF = TRANS ? aC * h : aF, cC = TRANS ? aF * ih : aC;
    const TC J = u[N - 1] - Up;
    const TC F = cF * ih * (Gm + Gp);
    b[N - 1] += At * (aP * J - F);
    const TC cj = At * cC * J;
#pragma unroll
    for (int i = 0; i < N; ++i) b[i] -= cj * T.d1[i];
  }
  {  // lower face
    TC Gm = TC(0), Gp = TC(0);
#pragma unroll
    for (int j = 0; j < N; ++j) Gp += T.d0[j] * u[j];
    TC Um = TC(0), aF, aP, aC;
    if (hasL) {
#pragma unroll
      for (int j = 0; j < N; ++j) Gm += T.d1[j] * uL[j];
      Um = uL[N - 1];
      const TC g = TC(2) * K * KL / (K + KL);
      aF = TC(0.5) * g;
      aP = sig * g;
      aC = TC(0.5) * g * ih;
    } else {
      aF = K;
      aP = sig * K;
      aC = K * ih;
    }
    const TC cF = TRANS ? aC * h : aF, cC = TRANS ? aF * ih : aC;
    const TC J = Um - u[0];
    const TC F = cF * ih * (Gm + Gp);
    b[0] += At * (F - aP * J);
    const TC cj = At * cC * J;
#pragma unroll
    for (int i = 0; i < N; ++i) b[i] -= cj * T.d0[i];
  }
}

// out = A1 a (+ add), A1 = M (TRANS: M^T) along the line
template <int N, typename TC, bool TRANS>
__device__ __forceinline__ void mass_line(const Tables<TC>& T, const TC (&a)[N], TC (&out)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    TC s = TC(0);
#pragma unroll
    for (int j = 0; j < N; ++j) s += (TRANS ? T.M[j * kMaxN + i] : T.M[i * kMaxN + j]) * a[j];
    out[i] = s;
  }
}

// line operator of axis D for the thread's line, neighbour lines from HBM
template <int N, int D, typename TC, typename TIN, bool TRANS>
__device__ __forceinline__ void axis_op(const MeshArgs<TC>& m, const Tables<TC>& T,
                                        const TIN* __restrict__ x, int ex, int ey, int ez, TC K,
                                        int t1, int t2, const TC (&u)[N], TC (&b)[N]) {
  const int64_t nL = neighbour<D>(m, ex, ey, ez, 0), nH = neighbour<D>(m, ex, ey, ez, 1);
  TC uL[N], uH[N];
  TC KL = TC(1), KH = TC(1);
  if (nL >= 0) {
    glb_get<N, D, TC, TIN>(x, nL, t1, t2, uL);
    KL = m.K[nL];
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) uL[i] = TC(0);
  }
  if (nH >= 0) {
    glb_get<N, D, TC, TIN>(x, nH, t1, t2, uH);
    KH = m.K[nH];
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) uH[i] = TC(0);
  }
  const TC h = D == 0 ? m.hx : (D == 1 ? m.hy : m.hz);
  const TC At = D == 0 ? m.hy * m.hz : (D == 1 ? m.hx * m.hz : m.hx * m.hy);
  line_op<N, TC, TRANS>(T, u, uL, uH, nL >= 0, nH >= 0, K, KL, KH, h, At, m.sig_hat, true, b);
}

template <typename TOUT>
__device__ __forceinline__ TOUT store_cast(double v) { return (TOUT)v; }

// y = A x (TRANS: A^T x).  DOT: also <x, y> (y as stored) into *dot_out by a
// deterministic grid reduction.  skip != nullptr && *skip: do nothing (used
// by the solver once it has converged).
template <int N, typename TIN, typename TOUT, typename TC, bool TRANS, bool DOT>
__global__ __launch_bounds__(kBlock) void k_apply_affine(MeshArgs<TC> m, const TIN* __restrict__ x,
                                                         TOUT* __restrict__ y, double* partials,
                                                         unsigned* counter, double* dot_out,
                                                         const int* skip) {
  constexpr int NN = N * N, N3 = NN * N, EPB = elems_per_block(N);
  __shared__ TC sU[EPB * N3], sA[EPB * N3], sB[EPB * N3];
  __shared__ double red[kBlock / 64];
  if (skip != nullptr && *skip) return;
  const Tables<TC>& T = *m.tab;
  const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
  const int tid = threadIdx.x, el = tid / NN, t = tid % NN, t1 = t % N, t2 = t / N;
  const int64_t e = blk * EPB + el;
  const bool act = (el < EPB) && (e < m.E);
  TC* U = sU + (act ? el : 0) * N3;
  TC* A = sA + (act ? el : 0) * N3;
  TC* B = sB + (act ? el : 0) * N3;
  int ex = 0, ey = 0, ez = 0;
  TC K = TC(1);
  TC uz[N];
  if (act) {
    ex = (int)(e % m.nx);
    ey = (int)((e / m.nx) % m.ny);
    ez = (int)(e / ((int64_t)m.nx * m.ny));
    K = m.K[e];
    // phase Z
    TC b[N];
    glb_get<N, 2, TC, TIN>(x, e, t1, t2, uz);
    axis_op<N, 2, TC, TIN, TRANS>(m, T, x, ex, ey, ez, K, t1, t2, uz, b);
    lds_put<N, 2>(U, t1, t2, uz);
    lds_put<N, 2>(B, t1, t2, b);
  }
  __syncthreads();
  if (act) {  // phase Y
    TC u[N], b[N];
    lds_get<N, 1>(U, t1, t2, u);
    axis_op<N, 1, TC, TIN, TRANS>(m, T, x, ex, ey, ez, K, t1, t2, u, b);
    lds_put<N, 1>(A, t1, t2, b);
  }
  __syncthreads();
  if (act) {  // phase X
    TC u[N], bx[N], by[N], bz[N], c[N], ee[N];
    lds_get<N, 0>(U, t1, t2, u);
    axis_op<N, 0, TC, TIN, TRANS>(m, T, x, ex, ey, ez, K, t1, t2, u, bx);
    lds_get<N, 0>(A, t1, t2, by);
    lds_get<N, 0>(B, t1, t2, bz);
    mass_line<N, TC, TRANS>(T, by, c);
    mass_line<N, TC, TRANS>(T, bz, ee);
    lds_put<N, 0>(U, t1, t2, bx);
    lds_put<N, 0>(A, t1, t2, c);
    lds_put<N, 0>(B, t1, t2, ee);
  }
  __syncthreads();
  if (act) {  // phase Y2
    TC bx[N], c[N], ee[N], f[N], g[N];
    lds_get<N, 1>(U, t1, t2, bx);
    lds_get<N, 1>(A, t1, t2, c);
    lds_get<N, 1>(B, t1, t2, ee);
    mass_line<N, TC, TRANS>(T, bx, f);
    mass_line<N, TC, TRANS>(T, ee, g);
#pragma unroll
    for (int i = 0; i < N; ++i) f[i] += c[i];
    lds_put<N, 1>(U, t1, t2, f);
    lds_put<N, 1>(A, t1, t2, g);
  }
  __syncthreads();
  double part = 0.0;
  if (act) {  // phase Z2
    TC f[N], g[N], r[N];
    lds_get<N, 2>(U, t1, t2, f);
    lds_get<N, 2>(A, t1, t2, g);
    mass_line<N, TC, TRANS>(T, f, r);
    TOUT* py = y + e * N3;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const TOUT v = (TOUT)(r[i] + g[i]);
      py[lidx<N, 2>(t1, t2, i)] = v;
      if (DOT) part += (double)uz[i] * (double)v;
    }
  }
  if (DOT) {
    double s = block_sum<kBlock>(part, red);
    double mine[1] = {s};
    grid_finish<1, kBlock>(mine, partials, counter, gridDim.x, blockIdx.x,
                           [&](const double* tot) { *dot_out = tot[0]; });
  }
}

// diag(A): one thread per DOF; (L_d)_{ii} from the line operator applied to
// the unit line (the neighbour line is the unit line too when the element is
// its own neighbour, i.e. one element along d with periodic wrap).
template <int N>
__global__ __launch_bounds__(256) void k_diag_affine(MeshArgs<double> m, double* __restrict__ d) {
  constexpr int NN = N * N, N3 = NN * N;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= m.E * N3) return;
  const Tables<double>& T = *m.tab;
  const int64_t e = gid / N3;
  const int li = (int)(gid % N3);
  const int i1 = li % N, i2 = (li / N) % N, i3 = li / NN;
  const int ex = (int)(e % m.nx), ey = (int)((e / m.nx) % m.ny), ez = (int)(e / ((int64_t)m.nx * m.ny));
  const double K = m.K[e];
  double acc = 0.0;
#pragma unroll
  for (int D = 0; D < 3; ++D) {
    const int id = D == 0 ? i1 : (D == 1 ? i2 : i3);
    const int ta = D == 0 ? i2 : i1, tb = D == 0 ? i3 : (D == 1 ? i3 : i2);
    int64_t nL, nH;
    if (D == 0) { nL = neighbour<0>(m, ex, ey, ez, 0); nH = neighbour<0>(m, ex, ey, ez, 1); }
    else if (D == 1) { nL = neighbour<1>(m, ex, ey, ez, 0); nH = neighbour<1>(m, ex, ey, ez, 1); }
    else { nL = neighbour<2>(m, ex, ey, ez, 0); nH = neighbour<2>(m, ex, ey, ez, 1); }
    double u[N], uL[N], uH[N], b[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      u[i] = i == id ? 1.0 : 0.0;
      uL[i] = (nL == e && i == id) ? 1.0 : 0.0;
      uH[i] = (nH == e && i == id) ? 1.0 : 0.0;
    }
    const double KL = nL >= 0 ? m.K[nL] : 1.0, KH = nH >= 0 ? m.K[nH] : 1.0;
    const double h = D == 0 ? m.hx : (D == 1 ? m.hy : m.hz);
    const double At = D == 0 ? m.hy * m.hz : (D == 1 ? m.hx * m.hz : m.hx * m.hy);
    line_op<N, double, false>(T, u, uL, uH, nL >= 0, nH >= 0, K, KL, KH, h, At, m.sig_hat, true, b);
    double bi = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (i == id) bi = b[i];
    acc += T.M[ta * kMaxN + ta] * T.M[tb * kMaxN + tb] * bi;
  }
  d[gid] = acc;
}

// g_T = u^T (dA/dtheta_T) v on affine meshes (FP64).  Per element:
//  volume  K_T u_T^T A_vol v_T with A_vol = sum_d M (x) M (x) (At/h) S_d
//          (dK/dtheta = K), composed like the apply:
//          A_vol v = M_z (M_y wx + M_x wy) + M_y M_x wz, w_d = (At/h) S_d v
//  faces   dgamma/dtheta_T * a_e(u, v) with gamma = 1, where on the face
//          a_e = At sum_p [ -Jv (MM Fu) - Fv (MM Ju) + sigma Jv (MM Ju) ],
//          J = trace jump, F = average normal derivative (interior) or the
//          own normal derivative (boundary), MM = M (x) M on the n^2 face
//          nodes; dgamma/dtheta_T = gamma K_other / (K^- + K^+) or K_T.
template <int N>
__global__ __launch_bounds__(kBlock) void k_dA_dtheta_affine(MeshArgs<double> m,
                                                             const double* __restrict__ u,
                                                             const double* __restrict__ v,
                                                             double* __restrict__ g) {
  constexpr int NN = N * N, N3 = NN * N, EPB = elems_per_block(N);
  __shared__ double sU[EPB * N3], sV[EPB * N3], sW[EPB * N3], sX[EPB * N3];
  __shared__ double sF[EPB][2][NN];
  __shared__ double sPart[kBlock];
  const Tables<double>& T = *m.tab;
  const int tid = threadIdx.x, el = tid / NN, t = tid % NN, t1 = t % N, t2 = t / N;
  const int64_t e = (int64_t)blockIdx.x * EPB + el;
  const bool act = (el < EPB) && (e < m.E);
  const int le = act ? el : 0;
  double* U = sU + le * N3;
  double* V = sV + le * N3;
  double* W = sW + le * N3;
  double* X = sX + le * N3;
  int ex = 0, ey = 0, ez = 0;
  double K = 1.0;
  double part = 0.0;
  if (act) {
    ex = (int)(e % m.nx);
    ey = (int)((e / m.nx) % m.ny);
    ez = (int)(e / ((int64_t)m.nx * m.ny));
    K = m.K[e];
    double a[N], b[N];
    glb_get<N, 2, double, double>(u, e, t1, t2, a);
    glb_get<N, 2, double, double>(v, e, t1, t2, b);
    lds_put<N, 2>(U, t1, t2, a);
    lds_put<N, 2>(V, t1, t2, b);
  }
  __syncthreads();
#pragma unroll
  for (int D = 0; D < 3; ++D) {
    const double h = D == 0 ? m.hx : (D == 1 ? m.hy : m.hz);
    const double At = D == 0 ? m.hy * m.hz : (D == 1 ? m.hx * m.hz : m.hx * m.hy);
    const double ih = 1.0 / h, sig = m.sig_hat * ih;
    double fu[2][2], fv[2][2], dg[2];  // [side][J, F]
    if (act) {
      double lu[N], lv[N], nu[N], nv[N];
      if (D == 0) { lds_get<N, 0>(U, t1, t2, lu); lds_get<N, 0>(V, t1, t2, lv); }
      else if (D == 1) { lds_get<N, 1>(U, t1, t2, lu); lds_get<N, 1>(V, t1, t2, lv); }
      else { lds_get<N, 2>(U, t1, t2, lu); lds_get<N, 2>(V, t1, t2, lv); }
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        int64_t nb;
        if (D == 0) nb = neighbour<0>(m, ex, ey, ez, s);
        else if (D == 1) nb = neighbour<1>(m, ex, ey, ez, s);
        else nb = neighbour<2>(m, ex, ey, ez, s);
        const double* dn = s ? T.d1 : T.d0;  // own derivative at this face
        double Gu = 0.0, Gv = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j) { Gu += dn[j] * lu[j]; Gv += dn[j] * lv[j]; }
        Gu *= ih;
        Gv *= ih;
        const double Uu = s ? lu[N - 1] : lu[0], Uv = s ? lv[N - 1] : lv[0];
        if (nb >= 0) {
          if (D == 0) { glb_get<N, 0, double, double>(u, nb, t1, t2, nu); glb_get<N, 0, double, double>(v, nb, t1, t2, nv); }
          else if (D == 1) { glb_get<N, 1, double, double>(u, nb, t1, t2, nu); glb_get<N, 1, double, double>(v, nb, t1, t2, nv); }
          else { glb_get<N, 2, double, double>(u, nb, t1, t2, nu); glb_get<N, 2, double, double>(v, nb, t1, t2, nv); }
          const double* dm = s ? T.d0 : T.d1;  // neighbour's derivative at the shared face
          double Hu = 0.0, Hv = 0.0;
#pragma unroll
          for (int j = 0; j < N; ++j) { Hu += dm[j] * nu[j]; Hv += dm[j] * nv[j]; }
          Hu *= ih;
          Hv *= ih;
          const double Vu = s ? nu[0] : nu[N - 1], Vv = s ? nv[0] : nv[N - 1];
          // [w] = w^- - w^+ ; on the upper face this element is '-', on the lower '+'
          fu[s][0] = s ? Uu - Vu : Vu - Uu;
          fv[s][0] = s ? Uv - Vv : Vv - Uv;
          fu[s][1] = 0.5 * (Gu + Hu);
          fv[s][1] = 0.5 * (Gv + Hv);
          const double Kn = m.K[nb];
          const double gam = 2.0 * K * Kn / (K + Kn);
          dg[s] = gam * Kn / (K + Kn);
        } else {
          fu[s][0] = s ? Uu : -Uu;
          fv[s][0] = s ? Uv : -Uv;
          fu[s][1] = Gu;
          fv[s][1] = Gv;
          dg[s] = K;
        }
      }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      __syncthreads();
      if (act) {
        sF[le][0][t] = fu[s][0];
        sF[le][1][t] = fu[s][1];
      }
      __syncthreads();
      if (act) {
        double MJu = 0.0, MFu = 0.0;
#pragma unroll
        for (int b2 = 0; b2 < N; ++b2)
#pragma unroll
          for (int b1 = 0; b1 < N; ++b1) {
            const double w = T.M[t1 * kMaxN + b1] * T.M[t2 * kMaxN + b2];
            MJu += w * sF[le][0][b2 * N + b1];
            MFu += w * sF[le][1][b2 * N + b1];
          }
        const double Jv = fv[s][0], Fv = fv[s][1];
        part += dg[s] * At * (-Jv * MFu - Fv * MJu + sig * Jv * MJu);
      }
    }
  }
  // volume term
  double z0[N];
#pragma unroll
  for (int i = 0; i < N; ++i) z0[i] = 0.0;
  if (act) {  // Z
    double lv[N], w[N];
    lds_get<N, 2>(V, t1, t2, lv);
    line_op<N, double, false>(T, lv, z0, z0, false, false, 1.0, 1.0, 1.0, m.hz, m.hx * m.hy, m.sig_hat, false, w);
    lds_put<N, 2>(W, t1, t2, w);
  }
  __syncthreads();
  if (act) {  // Y
    double lv[N], w[N];
    lds_get<N, 1>(V, t1, t2, lv);
    line_op<N, double, false>(T, lv, z0, z0, false, false, 1.0, 1.0, 1.0, m.hy, m.hx * m.hz, m.sig_hat, false, w);
    lds_put<N, 1>(X, t1, t2, w);
  }
  __syncthreads();
  if (act) {  // X
    double lv[N], wx[N], wy[N], wz[N], c[N], ee[N];
    lds_get<N, 0>(V, t1, t2, lv);
    line_op<N, double, false>(T, lv, z0, z0, false, false, 1.0, 1.0, 1.0, m.hx, m.hy * m.hz, m.sig_hat, false, wx);
    lds_get<N, 0>(X, t1, t2, wy);
    lds_get<N, 0>(W, t1, t2, wz);
    mass_line<N, double, false>(T, wy, c);
    mass_line<N, double, false>(T, wz, ee);
    lds_put<N, 0>(V, t1, t2, wx);
    lds_put<N, 0>(X, t1, t2, c);
    lds_put<N, 0>(W, t1, t2, ee);
  }
  __syncthreads();
  if (act) {  // Y2
    double wx[N], c[N], ee[N], f[N], gg[N];
    lds_get<N, 1>(V, t1, t2, wx);
    lds_get<N, 1>(X, t1, t2, c);
    lds_get<N, 1>(W, t1, t2, ee);
    mass_line<N, double, false>(T, wx, f);
    mass_line<N, double, false>(T, ee, gg);
#pragma unroll
    for (int i = 0; i < N; ++i) f[i] += c[i];
    lds_put<N, 1>(V, t1, t2, f);
    lds_put<N, 1>(W, t1, t2, gg);
  }
  __syncthreads();
  if (act) {  // Z2 and <u, A_vol v>
    double f[N], gg[N], r[N], lu[N];
    lds_get<N, 2>(V, t1, t2, f);
    lds_get<N, 2>(W, t1, t2, gg);
    lds_get<N, 2>(U, t1, t2, lu);
    mass_line<N, double, false>(T, f, r);
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) s += lu[i] * (r[i] + gg[i]);
    part += K * s;
  }
  sPart[tid] = part;
  __syncthreads();
  if (act && t == 0) {
    double s = 0.0;
    for (int i = 0; i < NN; ++i) s += sPart[el * NN + i];
    g[e] = s;
  }
}

// ---------------------------------------------------------------- launchers

int64_t element_blocks(int n, int64_t E) {
  const int epb = elems_per_block(n);
  return (E + epb - 1) / epb;
}

template <int N, typename TIN, typename TOUT, typename TC, bool TRANS, bool DOT>
static hipError_t run_apply(const MeshArgs<TC>& m, const void* x, void* y, double* partials,
                            unsigned* counter, double* dot_out, const int* skip, hipStream_t s) {
  const int64_t nb = element_blocks(N, m.E);
  hipLaunchKernelGGL((k_apply_affine<N, TIN, TOUT, TC, TRANS, DOT>), dim3((unsigned)nb), dim3(kBlock), 0, s, m,
                     (const TIN*)x, (TOUT*)y, partials, counter, dot_out, skip);
  return hipGetLastError();
}

template <int N, bool TRANS, bool DOT>
static hipError_t run_apply_prec(int prec, const MeshArgs<double>& m64, const MeshArgs<float>& m32,
                                 const void* x, void* y, double* partials, unsigned* counter,
                                 double* dot_out, const int* skip, hipStream_t s) {
  switch (prec) {
    case 0: return run_apply<N, double, double, double, TRANS, DOT>(m64, x, y, partials, counter, dot_out, skip, s);
    case 1: return run_apply<N, float, float, float, TRANS, DOT>(m32, x, y, partials, counter, dot_out, skip, s);
    case 2: return run_apply<N, uint16_t, float, float, TRANS, DOT>(m32, x, y, partials, counter, dot_out, skip, s);
  }
  return hipErrorInvalidValue;
}

template <int N>
static hipError_t run_apply_n(int prec, int trans, int dot, const MeshArgs<double>& m64,
                              const MeshArgs<float>& m32, const void* x, void* y, double* partials,
                              unsigned* counter, double* dot_out, const int* skip, hipStream_t s) {
  if (trans) {
    if (dot) return run_apply_prec<N, true, true>(prec, m64, m32, x, y, partials, counter, dot_out, skip, s);
    return run_apply_prec<N, true, false>(prec, m64, m32, x, y, partials, counter, dot_out, skip, s);
  }
  if (dot) return run_apply_prec<N, false, true>(prec, m64, m32, x, y, partials, counter, dot_out, skip, s);
  return run_apply_prec<N, false, false>(prec, m64, m32, x, y, partials, counter, dot_out, skip, s);
}

hipError_t launch_apply_affine(int n, int prec, int trans, int dot, const MeshArgs<double>& m64,
                               const MeshArgs<float>& m32, const void* x, void* y, double* partials,
                               unsigned* counter, double* dot_out, const int* skip, hipStream_t s) {
  switch (n) {
    case 2: return run_apply_n<2>(prec, trans, dot, m64, m32, x, y, partials, counter, dot_out, skip, s);
    case 3: return run_apply_n<3>(prec, trans, dot, m64, m32, x, y, partials, counter, dot_out, skip, s);
    case 4: return run_apply_n<4>(prec, trans, dot, m64, m32, x, y, partials, counter, dot_out, skip, s);
    case 5: return run_apply_n<5>(prec, trans, dot, m64, m32, x, y, partials, counter, dot_out, skip, s);
    case 6: return run_apply_n<6>(prec, trans, dot, m64, m32, x, y, partials, counter, dot_out, skip, s);
    case 7: return run_apply_n<7>(prec, trans, dot, m64, m32, x, y, partials, counter, dot_out, skip, s);
    case 8: return run_apply_n<8>(prec, trans, dot, m64, m32, x, y, partials, counter, dot_out, skip, s);
  }
  return hipErrorInvalidValue;
}

template <int N>
static hipError_t run_diag(const MeshArgs<double>& m, double* d, hipStream_t s) {
  const int64_t tot = m.E * N * N * N;
  hipLaunchKernelGGL((k_diag_affine<N>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, m, d);
  return hipGetLastError();
}
hipError_t launch_diag_affine(int n, const MeshArgs<double>& m, double* d, hipStream_t s) {
  switch (n) {
    case 2: return run_diag<2>(m, d, s);
    case 3: return run_diag<3>(m, d, s);
    case 4: return run_diag<4>(m, d, s);
    case 5: return run_diag<5>(m, d, s);
    case 6: return run_diag<6>(m, d, s);
    case 7: return run_diag<7>(m, d, s);
    case 8: return run_diag<8>(m, d, s);
  }
  return hipErrorInvalidValue;
}

template <int N>
static hipError_t run_dA(const MeshArgs<double>& m, const double* u, const double* v, double* g,
                         hipStream_t s) {
  const int64_t nb = element_blocks(N, m.E);
  hipLaunchKernelGGL((k_dA_dtheta_affine<N>), dim3((unsigned)nb), dim3(kBlock), 0, s, m, u, v, g);
  return hipGetLastError();
}
hipError_t launch_dA_affine(int n, const MeshArgs<double>& m, const double* u, const double* v, double* g,
                            hipStream_t s) {
  switch (n) {
    case 2: return run_dA<2>(m, u, v, g, s);
    case 3: return run_dA<3>(m, u, v, g, s);
    case 4: return run_dA<4>(m, u, v, g, s);
    case 5: return run_dA<5>(m, u, v, g, s);
    case 6: return run_dA<6>(m, u, v, g, s);
    case 7: return run_dA<7>(m, u, v, g, s);
    case 8: return run_dA<8>(m, u, v, g, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace dg
