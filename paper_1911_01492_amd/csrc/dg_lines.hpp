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

template <int N, int D, typename TC>
__device__ __forceinline__ void lds_get(const TC* tile, int t1, int t2, TC (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = tile[lidx<N, D>(t1, t2, i)];
}
template <int N, int D, typename TC>
__device__ __forceinline__ void lds_put(TC* tile, int t1, int t2, const TC (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) tile[lidx<N, D>(t1, t2, i)] = v[i];
}
template <int N, int D, typename TC, typename TIN>
__device__ __forceinline__ void glb_get(const TIN* __restrict__ x, int64_t e, int t1, int t2,
                                        TC (&v)[N]) {
  const TIN* p = x + e * (N * N * N);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = load_as<TC, TIN>(p + lidx<N, D>(t1, t2, i));
}

}  // namespace dg
