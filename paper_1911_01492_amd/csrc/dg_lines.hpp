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
// paddings come from an exhaustive search over small values.  V = 1 is a
// variant for kernels whose occupancy the LDS limits (the affine apply in
// FP64 at n = 6, the parallelepiped apply in FP64): n = 4 with element stride 74 (the same modelled
// conflicts), n = 6 and 7 unpadded (slab strides 36 and 49, element strides
// 216 and 343; 2% and 6% more), and n = 3 with element stride 36, so that
// the face-scalar slot (4 n^2) fits in a tile and needs no area of its own
// (34% more).  V = 2, n = 4 in FP64: element stride 80 (no more modelled
// conflicts), so that two tiles hold an element's 10 n^2 face rows (the
// trilinear apply).
template <int N, typename TC, int V = 0>
struct Lay {
  static constexpr bool f64 = sizeof(TC) == 8;
  static constexpr bool dense = V == 1 && f64 && (N == 3 || N == 4 || N == 6 || N == 7);
  static constexpr int P2 = N == 6 ? (f64 ? 6 : 7) : N == 8 ? 9 : N;
  static constexpr int P3 = N == 2 ? 5 : N == 4 ? 19 : N == 6 ? (dense ? 36 : f64 ? 39 : 42) :
                            N == 7 ? (dense ? 49 : f64 ? 52 : 56) : N == 8 ? 72 : N * N;
  static constexpr bool roomy = V == 2 && f64 && N == 4;
  static constexpr int PE = N == 2 ? 12 : N == 3 ? (dense ? 36 : 27) : N == 4 ? (dense ? 74 : roomy ? 80 : 76) : N == 6 ? (dense ? 216 : f64 ? 244 : 252) :
                            N == 7 ? (dense ? 343 : f64 ? 369 : 401) : N == 8 ? 576 : N * N * N;
  __device__ static __forceinline__ int off(int i1, int i2, int i3) { return i1 + P2 * i2 + P3 * i3; }
};

// LDS offset of value i of the line along axis D at tangential (t1, t2)
template <int N, int D, typename TC, int V = 0>
__device__ __forceinline__ int lds_idx(int t1, int t2, int i) {
  if constexpr (D == 0) return Lay<N, TC, V>::off(i, t1, t2);
  else if constexpr (D == 1) return Lay<N, TC, V>::off(t1, i, t2);
  else return Lay<N, TC, V>::off(t1, t2, i);
}

template <int N, int D, typename TC, int V = 0>
__device__ __forceinline__ void lds_get(const TC* tile, int t1, int t2, TC (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = tile[lds_idx<N, D, TC, V>(t1, t2, i)];
}
template <int N, int D, typename TC, int V = 0>
__device__ __forceinline__ void lds_put(TC* tile, int t1, int t2, const TC (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) tile[lds_idx<N, D, TC, V>(t1, t2, i)] = v[i];
}
// global line load; the element offset is a 32-bit index (the library limits
// N_dof below 2^31), so the address is a scalar base plus a 32-bit offset.
// OFF32 (the vector has fewer than 2^32 bytes): the byte offset itself is
// formed in 32 bits, which lets the load take the scalar-base form with a
// 32-bit vector offset instead of a 64-bit address computed per load.
template <int N, int D, typename TC, typename TIN, bool OFF32 = false>
__device__ __forceinline__ void glb_get_at(const TIN* __restrict__ x, uint32_t eo, int t1, int t2, TC (&v)[N]) {
  // eo: the element's first entry (element index times n^3)
  if constexpr (OFF32) {
    const uint32_t b = (eo + (uint32_t)lidx<N, D>(t1, t2, 0)) * (uint32_t)sizeof(TIN);
#pragma unroll
    for (int i = 0; i < N; ++i)
      v[i] = load_as<TC, TIN>((const TIN*)((const char*)x + (b + (uint32_t)(lidx<N, D>(0, 0, i) * sizeof(TIN)))));
  } else {
    const uint32_t base = eo + (uint32_t)lidx<N, D>(t1, t2, 0);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = load_as<TC, TIN>(x + (base + (uint32_t)(lidx<N, D>(0, 0, i))));
  }
}
template <int N, int D, typename TC, typename TIN, bool OFF32 = false>
__device__ __forceinline__ void glb_get(const TIN* __restrict__ x, int64_t e, int t1, int t2,
                                        TC (&v)[N]) {
  glb_get_at<N, D, TC, TIN, OFF32>(x, (uint32_t)e * (uint32_t)(N * N * N), t1, t2, v);
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

// out = A a along the line for the symmetric, centro-symmetric 1D matrix A
// (M or S, so A^T a = A a) given in full (Af) and by its even-odd halves
// (Ae): the halves from n = 5 on, where they save operations (n^2/2 + 2n
// against n^2 at even n), the full matrix below.
template <int N, typename TC>
__device__ __forceinline__ void sym_line(const TC* Af, const EvenOdd<TC>& Ae, const TC (&a)[N], TC (&out)[N]) {
  if constexpr (N >= 5) {
    contract_eo<N, TC, 1>(Ae, a, out);
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      TC s = TC(0);
#pragma unroll
      for (int j = 0; j < N; ++j) s += Af[i * kMaxN + j] * a[j];
      out[i] = s;
    }
  }
}

// out = M a along the line (M is symmetric: also M^T a)
template <int N, typename TC, bool TRANS>
__device__ __forceinline__ void mass_line(const Tables<TC>& T, const TC (&a)[N], TC (&out)[N]) {
  sym_line<N, TC>(T.M, T.eM, a, out);
}

// Line operator with the neighbour data reduced to the two scalars the face
// terms need: the neighbour's trace at the shared end (U) and its raw normal
// derivative at that end (Gr = l'(end) . line, without 1/h), both zero on a
// side without neighbour (Dirichlet face).  Own face scalars: u[0],
// g0 = d0.u, u[n-1], g1 = d1.u.  Same algebra as line_op.
template <int N, typename TC, bool TRANS>
__device__ __forceinline__ void line_op_s(const Tables<TC>& T, const TC (&u)[N], TC g0, TC g1, TC UL, TC GLr,
                                          TC UH, TC GHr, bool hasL, bool hasH, TC GL, TC GH, TC vs, TC ih,
                                          TC sig, TC At, TC (&b)[N]) {
  {  // volume: vs S u (S is symmetric: also the transpose)
    TC su[N];
    sym_line<N, TC>(T.S, T.eS, u, su);
#pragma unroll
    for (int i = 0; i < N; ++i) b[i] = vs * su[i];
  }
  {  // upper face: this element is T^-
    const TC g = g1 + GHr;
    const TC J = u[N - 1] - UH;
    const TC aP = sig * GH * (hasH ? TC(2) : TC(1));
    const TC GAi = At * GH * ih;
    b[N - 1] += At * aP * J - GAi * g;
    const TC cj = GAi * J;
#pragma unroll
    for (int i = 0; i < N; ++i) b[i] -= cj * T.d1[i];
  }
  {  // lower face: this element is T^+
    const TC g = g0 + GLr;
    const TC J = UL - u[0];
    const TC aP = sig * GL * (hasL ? TC(2) : TC(1));
    const TC GAi = At * GL * ih;
    b[0] += GAi * g - At * aP * J;
    const TC cj = GAi * J;
#pragma unroll
    for (int i = 0; i < N; ++i) b[i] -= cj * T.d0[i];
  }
}

// d0 . u (END = 0) or d1 . u (END = 1)
template <int N, typename TC, int END>
__device__ __forceinline__ TC dot_end(const Tables<TC>& T, const TC (&u)[N]) {
  TC s = TC(0);
#pragma unroll
  for (int j = 0; j < N; ++j) s += (END ? T.d1[j] : T.d0[j]) * u[j];
  return s;
}

// Brick of elements per workgroup for n nodes per direction (BX x BY x BZ,
// at most kBlock / n^2 elements); x is the fastest element index inside the
// brick so that a wave's elements share their y and z position.
__host__ __device__ constexpr int tile_x(int n) { return n == 2 ? 4 : n == 3 ? 4 : n == 4 ? 4 : n == 5 ? 5 : n == 6 ? 7 : n == 7 ? 5 : 4; }
__host__ __device__ constexpr int tile_y(int n) { return n == 2 ? 4 : n == 3 ? 3 : n == 4 ? 2 : n == 5 ? 2 : 1; }
__host__ __device__ constexpr int tile_z(int n) { return n == 2 ? 4 : n == 3 ? 2 : n == 4 ? 2 : 1; }
// threads per workgroup of the affine apply: the brick's lines, rounded up to whole waves
__host__ __device__ constexpr int apply_block(int n) {
  return ((tile_x(n) * tile_y(n) * tile_z(n) * n * n + 63) / 64) * 64;
}

// Origin of logical brick tb.  The brick grid (ntx x nty x ntz) is cut into
// slabs of CY brick rows along y; a slab is walked x fastest, then y, then z.
// Consecutive logical bricks run on the same XCD (xcd_remap), so the bricks
// that read an element's lines as neighbours run close in time to the brick
// that owns it: x-neighbours 1 brick apart, y-neighbours ntx, z-neighbours
// ntx CY (about 96 bricks), and the lines are still in that XCD's L2.  (With
// plain x-y-z order the z-neighbours were ntx nty bricks apart and each x
// line was fetched from HBM three times.)  Only the y-faces between slabs
// (one in CY brick rows) read lines of bricks that run much later.
template <int BX, int BY, int BZ>
__device__ __forceinline__ void brick_origin(int tb, int nx, int ny, int nz, int (&o)[3]) {
  const int ntx = (nx + BX - 1) / BX, nty = (ny + BY - 1) / BY, ntz = (nz + BZ - 1) / BZ;
  const int CY = max(1, min(nty, 96 / ntx));
  const int slab = ntx * CY * ntz;
  const int g = tb / slab, r = tb - g * slab;
  const int cy = min(CY, nty - g * CY);  // brick rows of this slab (the last one may be thinner)
  const int bx = r % ntx, q = r / ntx;
  o[0] = bx * BX;
  o[1] = (g * CY + q % cy) * BY;
  o[2] = (q / cy) * BZ;
}

// neighbour coordinate along one axis (periodic wrap), -1 on a Dirichlet boundary
__device__ __forceinline__ int nb_coord(int c, int s, int Nd, int periodic) {
  int v = c + (s ? 1 : -1);
  if (v < 0 || v >= Nd) {
    if (!periodic) return -1;
    v = v < 0 ? Nd - 1 : 0;
  }
  return v;
}

}  // namespace dg
