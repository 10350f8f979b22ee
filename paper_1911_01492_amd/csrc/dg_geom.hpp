// dg_geom.hpp -- trilinear element maps on the device.
//
// Element e = ex + nx (ey + ny ez) has the 8 corner vertices
// (ex + c0, ey + c1, ez + c2), corner index c = c0 + 2 c1 + 4 c2, of the
// (nx+1)(ny+1)(nz+1) vertex grid (x-index fastest); without a vertex array
// the grid is uniform, vertex (i, j, l) at (i/nx, j/ny, l/nz).
#pragma once

#include "dg_internal.hpp"

namespace dg {

template <typename T>
__device__ __forceinline__ void element_corners(const MeshArgs<T>& m, int64_t e, T (&X)[8][3]) {
  const int ex = (int)(e % m.nx), ey = (int)((e / m.nx) % m.ny), ez = (int)(e / ((int64_t)m.nx * m.ny));
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int vx = ex + (c & 1), vy = ey + ((c >> 1) & 1), vz = ez + ((c >> 2) & 1);
    if (m.vert) {
      const int64_t v = vx + (int64_t)(m.nx + 1) * (vy + (int64_t)(m.ny + 1) * vz);
      X[c][0] = m.vert[3 * v];
      X[c][1] = m.vert[3 * v + 1];
      X[c][2] = m.vert[3 * v + 2];
    } else {
      X[c][0] = (T)vx * m.hx;
      X[c][1] = (T)vy * m.hy;
      X[c][2] = (T)vz * m.hz;
    }
  }
}

// x = F(xi) = sum_c X_c prod_d (c_d ? xi_d : 1 - xi_d)
template <typename T>
__device__ __forceinline__ void trilinear_map(const T (&X)[8][3], const T (&xi)[3], T (&x)[3]) {
  x[0] = x[1] = x[2] = T(0);
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const T w = ((c & 1) ? xi[0] : T(1) - xi[0]) * ((c & 2) ? xi[1] : T(1) - xi[1]) *
                ((c & 4) ? xi[2] : T(1) - xi[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] += w * X[c][a];
  }
}

// J[a][d] = d x_a / d xi_d, written with the edge vectors of the corner cube:
// dF/dxi_0 = (1-xi_1)(1-xi_2)(X1-X0) + xi_1(1-xi_2)(X3-X2) + (1-xi_1)xi_2(X5-X4) + xi_1 xi_2 (X7-X6)
// and cyclically for the other two directions.
template <typename T>
__device__ __forceinline__ void trilinear_jacobian(const T (&X)[8][3], const T (&xi)[3], T (&J)[3][3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int b = 1 << d;
    const int o1 = (d == 0) ? 1 : 0, o2 = (d == 2) ? 1 : 2;  // the other two axes
    const T s1 = xi[o1], s2 = xi[o2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      T acc = T(0);
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        if (c & b) continue;  // edge from corner c to c + b
        const T w = (((c >> o1) & 1) ? s1 : T(1) - s1) * (((c >> o2) & 1) ? s2 : T(1) - s2);
        acc += w * (X[c + b][a] - X[c][a]);
      }
      J[a][d] = acc;
    }
  }
}

// J at the points of one line along xi_2 (xi_0, xi_1 fixed).  In the sum of
// trilinear_jacobian the column along xi_2 depends on xi_0, xi_1 only and the
// other two columns are affine in xi_2, so after this set-up (the edge
// vectors of the corner cube combined once per line) each point costs six
// multiply-adds: J[.][0] = p0 + xi_2 d0, J[.][1] = p1 + xi_2 d1, J[.][2] = c2.
template <typename T>
struct JacZLine {
  T p0[3], d0[3], p1[3], d1[3], c2[3];
  __device__ __forceinline__ JacZLine(const T (&X)[8][3], T x0, T x1) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      // edges along xi_0 from corners 0, 2, 4, 6 (weights in xi_1, xi_2)
      const T lo0 = (T(1) - x1) * (X[1][a] - X[0][a]) + x1 * (X[3][a] - X[2][a]);
      const T hi0 = (T(1) - x1) * (X[5][a] - X[4][a]) + x1 * (X[7][a] - X[6][a]);
      p0[a] = lo0;
      d0[a] = hi0 - lo0;
      // edges along xi_1 from corners 0, 1, 4, 5 (weights in xi_0, xi_2)
      const T lo1 = (T(1) - x0) * (X[2][a] - X[0][a]) + x0 * (X[3][a] - X[1][a]);
      const T hi1 = (T(1) - x0) * (X[6][a] - X[4][a]) + x0 * (X[7][a] - X[5][a]);
      p1[a] = lo1;
      d1[a] = hi1 - lo1;
      // edges along xi_2 from corners 0..3 (weights in xi_0, xi_1)
      c2[a] = (T(1) - x1) * ((T(1) - x0) * (X[4][a] - X[0][a]) + x0 * (X[5][a] - X[1][a])) +
              x1 * ((T(1) - x0) * (X[6][a] - X[2][a]) + x0 * (X[7][a] - X[3][a]));
    }
  }
  __device__ __forceinline__ void at(T x2, T (&J)[3][3]) const {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      J[a][0] = p0[a] + x2 * d0[a];
      J[a][1] = p1[a] + x2 * d1[a];
      J[a][2] = c2[a];
    }
  }
};

// J at the point (xi_A, xi_B) = (ta, tb) of the face xi_D = s (s = 0 or 1),
// A < B the tangential axes.  On the face the weights of trilinear_jacobian
// that carry the factor xi_D or 1 - xi_D are 0 or 1: the tangential columns
// keep the two edges of the face itself, the normal column all four edges
// along D.
template <int D, typename T>
__device__ __forceinline__ void face_jacobian(const T (&X)[8][3], int s, T ta, T tb, T (&J)[3][3]) {
  constexpr int A = D == 0 ? 1 : 0, B = D == 2 ? 1 : 2;
  constexpr int BD = 1 << D, BA = 1 << A, BB = 1 << B;
  const int c0 = s ? BD : 0;  // the face's first corner
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    J[r][D] = (T(1) - tb) * ((T(1) - ta) * (X[BD][r] - X[0][r]) + ta * (X[BA + BD][r] - X[BA][r])) +
              tb * ((T(1) - ta) * (X[BB + BD][r] - X[BB][r]) + ta * (X[BA + BB + BD][r] - X[BA + BB][r]));
    J[r][A] = (T(1) - tb) * (X[c0 + BA][r] - X[c0][r]) + tb * (X[c0 + BB + BA][r] - X[c0 + BB][r]);
    J[r][B] = (T(1) - ta) * (X[c0 + BB][r] - X[c0][r]) + ta * (X[c0 + BA + BB][r] - X[c0 + BA][r]);
  }
}

template <typename T>
__device__ __forceinline__ T det3(const T (&J)[3][3]) {
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// adjugate: adj(J) = det(J) J^{-1}
template <typename T>
__device__ __forceinline__ void adj3(const T (&J)[3][3], T (&A)[3][3]) {
  A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
}

}  // namespace dg
