// dg_lines.hpp -- per-line access helpers shared by the element kernels.
//
// Every element kernel gives each element n^2 threads; in orientation D a
// thread (t1, t2) owns the line of n values along axis D at tangential
// position (t1, t2): D = 0 (x-lines): (i2, i3) = (t1, t2); D = 1 (y-lines):
// (i1, i3) = (t1, t2); D = 2 (z-lines): (i1, i2) = (t1, t2).
#pragma once

#include "dg_internal.hpp"

namespace dg {

// offset of value i of the line along axis D at tangential position (t1, t2)
// inside an element block (i1 + n (i2 + n i3))
template <int N, int D>
__device__ __forceinline__ int lidx(int t1, int t2, int i) {
  if constexpr (D == 0) return t2 * N * N + t1 * N + i;  // x-line: i2 = t1, i3 = t2
  else if constexpr (D == 1) return t2 * N * N + i * N + t1;  // y-line: i1 = t1, i3 = t2
  else return i * N * N + t2 * N + t1;  // z-line: i1 = t1, i2 = t2
}

// neighbour element across the lower (s = 0) or upper (s = 1) face normal to
// axis D; -1 on a Dirichlet boundary, periodic wrap otherwise
template <int D, typename T>
__device__ __forceinline__ int64_t neighbour(const MeshArgs<T>& m, int ex, int ey, int ez, int s) {
  int c0 = ex, c1 = ey, c2 = ez;
  int& c = D == 0 ? c0 : (D == 1 ? c1 : c2);
  const int Nd = D == 0 ? m.nx : (D == 1 ? m.ny : m.nz);
  int v = c + (s ? 1 : -1);
  if (v < 0 || v >= Nd) {
    if (!m.periodic) return -1;
    v = v < 0 ? Nd - 1 : 0;
  }
  c = v;
  return c0 + (int64_t)m.nx * (c1 + (int64_t)m.ny * c2);
}

// LDS layout of one element tile, chosen so that the three line orientations
// read and write with at most 2-way bank conflicts: a thread group served in
// one LDS pass (16 lanes for 8-byte words, 32 lanes for 4-byte words) should
// hit distinct banks.  Offsets are affine, i1 + P2 i2 + P3 i3 (element stride
// PE), so that every access is a per-thread base plus an immediate; the
// paddings come from an exhaustive search over small values.
template <int N, typename TC>
struct Lay {
  static constexpr bool f64 = sizeof(TC) == 8;
  static constexpr int P2 = N == 6 ? (f64 ? 6 : 7) : N == 8 ? 9 : N;
  static constexpr int P3 = N == 2 ? 5 : N == 4 ? 19 : N == 6 ? (f64 ? 39 : 42) : N == 7 ? (f64 ? 52 : 56) :
                            N == 8 ? 72 : N * N;
  static constexpr int PE = N == 2 ? 12 : N == 4 ? 76 : N == 6 ? (f64 ? 244 : 252) :
                            N == 7 ? (f64 ? 369 : 401) : N == 8 ? 576 : N * N * N;
  __device__ static __forceinline__ int off(int i1, int i2, int i3) { return i1 + P2 * i2 + P3 * i3; }
};

// LDS offset of value i of the line along axis D at tangential (t1, t2)
template <int N, int D, typename TC>
__device__ __forceinline__ int lds_idx(int t1, int t2, int i) {
  if constexpr (D == 0) return Lay<N, TC>::off(i, t1, t2);
  else if constexpr (D == 1) return Lay<N, TC>::off(t1, i, t2);
  else return Lay<N, TC>::off(t1, t2, i);
}

template <int N, int D, typename TC>
__device__ __forceinline__ void lds_get(const TC* tile, int t1, int t2, TC (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = tile[lds_idx<N, D, TC>(t1, t2, i)];
}
template <int N, int D, typename TC>
__device__ __forceinline__ void lds_put(TC* tile, int t1, int t2, const TC (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) tile[lds_idx<N, D, TC>(t1, t2, i)] = v[i];
}
// global line load; the element offset is a 32-bit index (the library limits
// N_dof below 2^31), so the address is a scalar base plus a 32-bit offset
template <int N, int D, typename TC, typename TIN>
__device__ __forceinline__ void glb_get(const TIN* __restrict__ x, int64_t e, int t1, int t2,
                                        TC (&v)[N]) {
  const uint32_t base = (uint32_t)e * (uint32_t)(N * N * N) + (uint32_t)lidx<N, D>(t1, t2, 0);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = load_as<TC, TIN>(x + (base + (uint32_t)(lidx<N, D>(0, 0, i))));
}

// out = A a for A given by its even-odd halves (SIGN: A[n-1-i][n-1-j] = SIGN A[i][j]):
// with a_e = a_j + a_{n-1-j}, a_o = a_j - a_{n-1-j} (j < n/2),
//   P_i = E a_e (+ C_i a_m), Q_i = O a_o,  out_i = P_i + Q_i,  out_{n-1-i} = SIGN (P_i - Q_i),
// and for odd n the middle row R a_e + mm a_m (SIGN = +1) or R a_o (SIGN = -1).
template <int N, typename TC, int SIGN>
__device__ __forceinline__ void contract_eo(const EvenOdd<TC>& A, const TC (&a)[N], TC (&out)[N]) {
  constexpr int H = N / 2;
  TC ae[H], ao[H];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    ae[j] = a[j] + a[N - 1 - j];
    ao[j] = a[j] - a[N - 1 - j];
  }
#pragma unroll
  for (int i = 0; i < H; ++i) {
    TC P = (N & 1) ? A.C[i] * a[H] : TC(0), Q = TC(0);
#pragma unroll
    for (int j = 0; j < H; ++j) {
      P += A.E[i * kMaxH + j] * ae[j];
      Q += A.O[i * kMaxH + j] * ao[j];
    }
    out[i] = P + Q;
    out[N - 1 - i] = SIGN > 0 ? P - Q : Q - P;
  }
  if (N & 1) {
    TC s = SIGN > 0 ? A.mm * a[H] : TC(0);
#pragma unroll
    for (int j = 0; j < H; ++j) s += A.R[j] * (SIGN > 0 ? ae[j] : ao[j]);
    out[H] = s;
  }
}

}  // namespace dg
