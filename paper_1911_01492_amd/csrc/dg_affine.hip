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
// Layout: a workgroup owns a brick of BX x BY x BZ elements (tile_x/y/z(n)),
// n^2 threads per element, two n^3 LDS tiles per element (S1, S2).
// Neighbour lines inside the brick come from LDS, the others from HBM
// (issued up front).  The phases of the apply kernel:
//
//   X : own x-lines, x-neighbour scalars -> b_x = L_x u            -> S1
//   Y : own y-lines, y-neighbour scalars -> b_y = L_y u -> S2, M_y S1 -> S1
//   X2: S1 + M_x S2                                                -> S1
//   Z : own z-lines, z-neighbour scalars -> b_z = L_z u -> S2, r = M_z S1
//   X3, Y3: M_y M_x S2                                             -> S2
//   Z2: y = r + S2 -> HBM
//
// so that y = M_z (M_y b_x + M_x b_y) + M_y M_x b_z.
#include "dg_internal.hpp"
#include "dg_kernels.hpp"
#include "dg_lines.hpp"
#include "dg_faces.hpp"

namespace dg {

// 1D SWIPDG operator on one line:  b = L u  (TRANS: b = L^T u), with
//   volume   vs S u                         (vs = K At / h, At = h_t1 h_t2, h = h_d)
//   upper face (this element is T^-):  J = u[n-1] - uH[0],
//       F = GH (G^- + G^+),  G^- = d1.u / h,  G^+ = d0.uH / h
//       b[n-1] += At (aP J - F),   b[i] -= At (GH / h) d1[i] J
//   lower face (this element is T^+):  J = uL[n-1] - u[0],
//       F = GL (G^- + G^+),  G^- = d1.uL / h,  G^+ = d0.u / h
//       b[0]   += At (F - aP J),   b[i] -= At (GL / h) d0[i] J
// with the face coefficient G = gamma/2 = K K'/(K + K') and aP = sigma gamma
// = 2 sigma G on interior faces, G = K and aP = sigma K on Dirichlet faces
// (neighbour terms 0).  The per-face algebra is symmetric (the coefficients
// of the flux-times-jump and jump-times-flux terms coincide), so the
// transpose only transposes S.
template <int N, typename TC, bool TRANS>
__device__ __forceinline__ void line_op(const Tables<TC>& T, const TC (&u)[N], const TC (&uL)[N],
                                        const TC (&uH)[N], bool hasL, bool hasH, TC GL, TC GH, TC vs,
                                        TC ih, TC sig, TC At, bool faces, TC (&b)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    TC s = TC(0);
#pragma unroll
    for (int j = 0; j < N; ++j) s += (TRANS ? T.S[j * kMaxN + i] : T.S[i * kMaxN + j]) * u[j];
    b[i] = vs * s;
  }
  if (!faces) return;
  {  // upper face
    TC g = TC(0);
#pragma unroll
    for (int j = 0; j < N; ++j) g += T.d1[j] * u[j];
    TC Up = TC(0);
    if (hasH) {
#pragma unroll
      for (int j = 0; j < N; ++j) g += T.d0[j] * uH[j];
      Up = uH[0];
    }
    const TC J = u[N - 1] - Up;
    const TC aP = sig * GH * (hasH ? TC(2) : TC(1));
    const TC GAi = At * GH * ih;
    b[N - 1] += At * aP * J - GAi * g;
    const TC cj = GAi * J;
#pragma unroll
    for (int i = 0; i < N; ++i) b[i] -= cj * T.d1[i];
  }
  {  // lower face
    TC g = TC(0);
#pragma unroll
    for (int j = 0; j < N; ++j) g += T.d0[j] * u[j];
    TC Um = TC(0);
    if (hasL) {
#pragma unroll
      for (int j = 0; j < N; ++j) g += T.d1[j] * uL[j];
      Um = uL[N - 1];
    }
    const TC J = Um - u[0];
    const TC aP = sig * GL * (hasL ? TC(2) : TC(1));
    const TC GAi = At * GL * ih;
    b[0] += GAi * g - At * aP * J;
    const TC cj = GAi * J;
#pragma unroll
    for (int i = 0; i < N; ++i) b[i] -= cj * T.d0[i];
  }
}


// y = A x (TRANS: A^T x) on affine meshes.  DOT: also the block partials of
// <x, y> (y as stored) for the CG scalar <p, A p>.  skip != nullptr &&
// *skip: do nothing (the solver has converged).  With a reaction term,
// c_T |T| M_z u joins b_z, so that the last two masses complete c_T |T| M (x) M (x) M u.
//
// With b_d = L_d u (the 1D DG operator along d, face terms included) the
// element result is y = M_z (M_y b_x + M_x b_y) + M_y M_x b_z.  The phases
// keep two element tiles in LDS (S1, S2; the face-scalar exchange area
// aliases S2), so that a block of the Q3 brick needs under 20 KB:
//   X : b_x                      -> S1
//   Y : b_y -> S2, M_y b_x       -> S1
//   X2: M_y b_x + M_x b_y        -> S1
//   Z : b_z -> S2, r = M_z S1       (registers)
//   X3, Y3: S2 <- M_y M_x S2
//   Z2: y = r + S2
template <int N, typename TIN, typename TOUT, typename TC, bool TRANS, bool DOT, bool OFF32>
__global__ __launch_bounds__(apply_block(N), (N == 5 && sizeof(TC) == 8) ? 8 : 1) void k_apply_affine(MeshArgs<TC> m, const TIN* __restrict__ x,
                                                         TOUT* __restrict__ y, double* partials,
                                                         const int* skip) {
  constexpr int NN = N * N, N3 = NN * N;
  constexpr int BX = tile_x(N), BY = tile_y(N), BZ = tile_z(N), TE = BX * BY * BZ;
  // in FP64 at n = 6 the LDS tiles bound the occupancy (five workgroups per
  // CU): the denser layout (2% more modelled bank conflicts) fits a sixth
  constexpr int LV = N == 6 ? 1 : 0;
  constexpr int PE = Lay<N, TC, LV>::PE;
  constexpr bool F_IN_S2 = 4 * NN <= PE;
  constexpr int FS = F_IN_S2 ? PE : 4 * NN;  // element stride of the face-scalar slots
  constexpr int BLOCK = apply_block(N);
  static_assert(TE * NN <= BLOCK && BLOCK <= kBlock, "brick too large");
  // an element's threads lie in one wavefront (ELEM), and so does each x-row
  // of the brick (XROW, which implies ELEM): those exchanges need only
  // wavefront-level synchronisation
  constexpr bool ELEM = 64 % NN == 0, XROW = 64 % (BX * NN) == 0;
  // padding threads (if the block has any) repeat the work of the brick's last
  // element lane for lane: they write the same values to the same LDS words in
  // the same instructions as their twins, which share their wavefront (the
  // brick's last element and the padding lie in the block's last wavefront),
  // so no slot of their own is needed
  constexpr int SLOTS = TE;
  static_assert(TE * NN == BLOCK || BLOCK - (TE - 1) * NN <= 64, "padding lanes and their twins share a wavefront");
  __shared__ TC sS1[SLOTS * PE], sS2[SLOTS * PE];
  __shared__ TC sFx[F_IN_S2 ? 1 : SLOTS * 4 * NN];
  __shared__ double red[BLOCK / 64];
  if (skip != nullptr && *skip) return;
  // vector blockIdx.y of a multi-vector apply (the vectors follow each other)
  x += (size_t)blockIdx.y * (size_t)m.E * N3;
  y += (size_t)blockIdx.y * (size_t)m.E * N3;
  TC* F = F_IN_S2 ? sS2 : sFx;
  // The 1D tables are read through the scalar cache.  At n = 8 in FP64 they
  // do not fit in scalar registers for the whole kernel (the compiler spills
  // them into vector-register lanes): there each use re-derives their address
  // through a constant-address pointer, so each phase loads what it uses.
  auto tabs = [&]() -> const Tables<TC>& {
    if constexpr (N >= 8 && sizeof(TC) == 8) {
      uint64_t a = (uint64_t)m.tab;
      asm volatile("" : "+s"(a));
      typedef const __attribute__((address_space(4))) Tables<TC>* ConstTab;
      return *(const Tables<TC>*)(ConstTab)a;
    } else {
      return *m.tab;
    }
  };
  // brick coordinates: uniform per workgroup (scalar arithmetic)
  const int tb = (int)xcd_remap(blockIdx.x, gridDim.x);
  int o[3];
  brick_origin<BX, BY, BZ>(tb, m.nx, m.ny, m.nz, o);
  const int Nd[3] = {m.nx, m.ny, m.nz};
  const int tid = threadIdx.x, el0 = tid / NN, t = tid - el0 * NN, t1 = t % N, t2 = t / N;
  const int el = min(el0, TE - 1);
  const int lx = el % BX, ly = (el / BX) % BY, lz = el / (BX * BY);
  const int cu[3] = {o[0] + lx, o[1] + ly, o[2] + lz};
  // own: the lane's element (for a padding lane its twin's) lies in the mesh;
  // the lanes of a brick's elements overhanging the mesh compute on the
  // nearest mesh element, see no neighbours and write only their own LDS slot.
  // act: own, and not a padding lane; only these store results.
  const bool own = cu[0] < m.nx && cu[1] < m.ny && cu[2] < m.nz;
  const bool act = el0 < TE && own;
  const int c[3] = {min(cu[0], m.nx - 1), min(cu[1], m.ny - 1), min(cu[2], m.nz - 1)};
  const int le = el;
  TC* S1 = sS1 + le * PE;
  TC* S2 = sS2 + le * PE;
  // the face-scalar slot of an element lies inside its own S2 tile (slot
  // stride PE): F traffic never touches another element's tile, so the
  // element-local hand-offs below need no workgroup barrier
  TC* Fe = F + le * FS;
  const int64_t e = c[0] + (int64_t)m.nx * (c[1] + (int64_t)m.ny * c[2]);
  const uint32_t eo = (uint32_t)e * (uint32_t)N3;  // the element's first entry (N_dof < 2^31)
  const TC K = m.K[e];
  // face coefficients of the element's faces 2D and 2D+1, loaded in the phase
  // that uses them (keeps the register count at 64 for n = 5 in FP64)
  auto gco = [&](int f) { return OFF32 ? m.G[(uint32_t)(6 * e + f)] : m.G[6 * e + f]; };
  TC b[N], v[N], w[N];
  // ---------------- X: b_x -> S1
  face_phase<N, 0, BX, BY, BZ, FS, TC, TIN, TRANS, OFF32>(m, tabs(), x, own, eo, c, o, Nd, t, t1, t2, Fe, K, gco(0), gco(1), TC(0), b);
  lds_put<N, 0, TC, LV>(S1, t1, t2, b);
  lds_sync<XROW>();  // F (read by the x-neighbours) is rewritten by the next phase
  // ---------------- Y: b_y -> S2, M_y b_x -> S1
  face_phase<N, 1, BX, BY, BZ, FS, TC, TIN, TRANS, OFF32>(m, tabs(), x, own, eo, c, o, Nd, t, t1, t2, Fe, K, gco(2), gco(3), TC(0), b);
  {
    lds_get<N, 1, TC, LV>(S1, t1, t2, v);
    mass_line<N, TC, TRANS>(tabs(), v, w);
  }
  if (F_IN_S2) __syncthreads();  // the face scalars in S2 have been read
  {
    lds_put<N, 1, TC, LV>(S2, t1, t2, b);
    lds_put<N, 1, TC, LV>(S1, t1, t2, w);
  }
  lds_sync<ELEM>();
  // ---------------- X2: M_y b_x + M_x b_y -> S1
  {
    lds_get<N, 0, TC, LV>(S2, t1, t2, v);
    lds_get<N, 0, TC, LV>(S1, t1, t2, w);
    mass_line<N, TC, TRANS>(tabs(), v, b);
#pragma unroll
    for (int i = 0; i < N; ++i) w[i] += b[i];
    lds_put<N, 0, TC, LV>(S1, t1, t2, w);
  }
  lds_sync<ELEM>();
  // ---------------- Z: b_z -> S2, r = M_z S1
  TC r[N], xz[N];  // xz: the thread's z-line of x, for the fused <x, y>
  const TC cr = m.R ? m.R[e] * m.vol : TC(0);
  face_phase<N, 2, BX, BY, BZ, FS, TC, TIN, TRANS, OFF32>(m, tabs(), x, own, eo, c, o, Nd, t, t1, t2, Fe, K, gco(4), gco(5), cr, b,
                                               DOT ? xz : nullptr);
  {
    lds_get<N, 2, TC, LV>(S1, t1, t2, v);
    mass_line<N, TC, TRANS>(tabs(), v, r);
  }
  if (F_IN_S2) __syncthreads();
  lds_put<N, 2, TC, LV>(S2, t1, t2, b);
  lds_sync<ELEM>();
  // ---------------- X3, Y3: S2 <- M_y M_x S2
  {
    lds_get<N, 0, TC, LV>(S2, t1, t2, v);
    mass_line<N, TC, TRANS>(tabs(), v, w);
    lds_put<N, 0, TC, LV>(S2, t1, t2, w);
  }
  lds_sync<ELEM>();
  {
    lds_get<N, 1, TC, LV>(S2, t1, t2, v);
    mass_line<N, TC, TRANS>(tabs(), v, w);
    lds_put<N, 1, TC, LV>(S2, t1, t2, w);
  }
  lds_sync<ELEM>();
  // ---------------- Z2: y = r + S2
  double part = 0.0;
  lds_get<N, 2, TC, LV>(S2, t1, t2, v);
  if (act) {
    // y is written once and not read back here: nontemporal stores keep it
    // from displacing in L2 the x lines that neighbouring bricks still read
    const uint32_t yb = (eo + (uint32_t)lidx<N, 2>(t1, t2, 0)) * (uint32_t)sizeof(TOUT);
    TOUT* py = y + e * N3;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const TOUT yv = (TOUT)(r[i] + v[i]);
      TOUT* dst = OFF32 ? (TOUT*)((char*)y + (yb + (uint32_t)(lidx<N, 2>(0, 0, i) * sizeof(TOUT))))
                        : &py[lidx<N, 2>(t1, t2, i)];
      __builtin_nontemporal_store(yv, dst);
      if (DOT) part += (double)xz[i] * (double)yv;
    }
  }
  if (DOT) {
    const double mine[1] = {block_sum<BLOCK>(part, red)};
    store_partials<1>(mine, partials, blockIdx.x);
  }
}

// diag(A): one thread per DOF; (L_d)_{ii} from the line operator applied to
// the unit line (the neighbour line is the unit line too when the element is
// its own neighbour, i.e. one element along d with periodic wrap).
template <int N>
__global__ __launch_bounds__(256) void k_diag_affine(MeshArgs<double> m, double* __restrict__ d, const int* run) {
  constexpr int NN = N * N, N3 = NN * N;
  if (run != nullptr && *run == 0) return;
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
    line_op<N, double, false>(T, u, uL, uH, nL >= 0, nH >= 0, m.G[6 * e + 2 * D], m.G[6 * e + 2 * D + 1],
                              K * m.vs[D], m.ih[D], m.sg[D], m.At[D], true, b);
    double bi = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (i == id) bi = b[i];
    acc += T.M[ta * kMaxN + ta] * T.M[tb * kMaxN + tb] * bi;
  }
  if (m.R) acc += m.R[e] * m.vol * T.M[i1 * kMaxN + i1] * T.M[i2 * kMaxN + i2] * T.M[i3 * kMaxN + i3];
  d[gid] = acc;
}

// ------------------------------------------------------------ element block-Jacobi
// Sec. 3.4 builds preconditioners from the element blocks of the DG matrix.
// On an axis-parallel box element with constant coefficients the diagonal
// block is a Kronecker sum of per-element 1D operators,
//     A_TT = M (x) M (x) L_x + M (x) L_y (x) M + L_z (x) M (x) M
// (L_d: the 1D DG operator along d restricted to the element's own values --
// stiffness, penalty and consistency terms of its two faces, the neighbour
// coupling only when the element is its own neighbour -- plus the reaction
// c |T| M on one axis), so its inverse follows from the generalized
// eigenproblems L_d q = lambda M q (fast diagonalisation):
//     A_TT^-1 = (Q_z (x) Q_y (x) Q_x) diag(1 / (l_z + l_y + l_x)) (Q_z (x) Q_y (x) Q_x)^T,
// with Q_d^T M Q_d = I and Q_d^T L_d Q_d = diag(l_d).  Setup: one thread per
// (element, axis) forms L_d column by column with the line operator, takes
// the symmetric C L_d C (C = M^-1/2), diagonalises it by cyclic Jacobi
// rotations and stores Q_d = C V (N x N, row = node, column = mode) and l_d.
template <int N>
__global__ __launch_bounds__(256) void k_bj_setup(MeshArgs<double> m, double* __restrict__ Q, double* __restrict__ lam,
                                                  float* __restrict__ Q32, float* __restrict__ lam32) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= 3 * m.E) return;
  const Tables<double>& T = *m.tab;
  const int64_t e = gid / 3;
  const int D = (int)(gid % 3);
  const int ex = (int)(e % m.nx), ey = (int)((e / m.nx) % m.ny), ez = (int)(e / ((int64_t)m.nx * m.ny));
  int64_t nL, nH;
  if (D == 0) { nL = neighbour<0>(m, ex, ey, ez, 0); nH = neighbour<0>(m, ex, ey, ez, 1); }
  else if (D == 1) { nL = neighbour<1>(m, ex, ey, ez, 0); nH = neighbour<1>(m, ex, ey, ez, 1); }
  else { nL = neighbour<2>(m, ex, ey, ez, 0); nH = neighbour<2>(m, ex, ey, ez, 1); }
  const double K = m.K[e], GL = m.G[6 * e + 2 * D], GH = m.G[6 * e + 2 * D + 1];
  double L[kMaxN * kMaxN];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double u[N], uL[N], uH[N], b[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      u[i] = i == j ? 1.0 : 0.0;
      uL[i] = (nL == e && i == j) ? 1.0 : 0.0;
      uH[i] = (nH == e && i == j) ? 1.0 : 0.0;
    }
    line_op<N, double, false>(T, u, uL, uH, nL >= 0, nH >= 0, GL, GH, K * m.vs[D], m.ih[D], m.sg[D], m.At[D], true,
                              b);
#pragma unroll
    for (int i = 0; i < N; ++i) L[i * kMaxN + j] = b[i];
  }
  if (D == 2 && m.R) {
    const double cr = m.R[e] * m.vol;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) L[i * kMaxN + j] += cr * T.M[i * kMaxN + j];
  }
  // A' = C L C (symmetrised: L is symmetric up to rounding)
  double A[kMaxN * kMaxN], V[kMaxN * kMaxN], CL[kMaxN * kMaxN];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) s += T.Mis[i * kMaxN + k] * 0.5 * (L[k * kMaxN + j] + L[j * kMaxN + k]);
      CL[i * kMaxN + j] = s;
    }
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) s += CL[i * kMaxN + k] * T.Mis[k * kMaxN + j];
      A[i * kMaxN + j] = s;
    }
  sym_eig_jacobi<double>(N, A, V);
  double* q = Q + (e * 3 + D) * N * N;
  double* l = lam + (e * 3 + D) * N;
  float* q32 = Q32 + (e * 3 + D) * N * N;
  float* l32 = lam32 + (e * 3 + D) * N;
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) s += T.Mis[i * kMaxN + k] * V[k * kMaxN + j];
      q[i * N + j] = s;
      q32[i * N + j] = (float)s;
    }
    l[i] = A[i * kMaxN + i];
    l32[i] = (float)A[i * kMaxN + i];
  }
}

// z = P r with P = blockdiag(A_TT^-1) by fast diagonalisation, and the block
// partials {<z, r>, <r, r>}.  n^2 threads per element, one line each per
// phase: Q_x^T, Q_y^T, Q_z^T, the scaling by 1 / (l_x + l_y + l_z), Q_z,
// Q_y, Q_x.  TV: vector type (double / float), TQ: type of the stored Q, l.
// UPD: first the CG residual update r -= lambda q with lambda = rho[par] / pq
// from the solver state (r is rewritten), so that the update and the
// preconditioner take one pass over the residual.  FUSED (with UPD): pq is
// summed here from the apply's nbA partials (partA) by every block in the
// same order, so all blocks obtain the same lambda; block 0 records pq and
// the pending x update, or stops the solve on a breakdown (no block writes a
// state field that another block of this kernel reads).
template <int N, typename TV, typename TQ, bool UPD, bool FUSED>
__global__ __launch_bounds__(kBlock) void k_bj_apply(int64_t E, const TQ* __restrict__ Q, const TQ* __restrict__ lam,
                                                     TV* __restrict__ r, TV* __restrict__ z, double* partials,
                                                     const int* skip, const TV* __restrict__ q, CgState* st,
                                                     int par, const double* partA, int64_t nbA) {
  constexpr int NN = N * N, EPB = elems_per_block(N), PE = Lay<N, TV>::PE;
  __shared__ TV sT[EPB * PE];
  __shared__ TQ sQ[EPB][3 * NN], sL[EPB][3 * N];
  __shared__ double red[kBlock / 64];
  if (skip != nullptr && *skip) return;
  double lamb = 0.0;
  if constexpr (FUSED) {
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (st->done) {
      if (lead) st->xpend = 0;
      return;
    }
    double t[1];
    sum_partials<1, kBlock>(partA, nbA, t);
    const double pq = t[0];
    lamb = st->rho[par] / pq;
    if (!(pq > 0.0) || !(lamb == lamb && lamb - lamb == 0.0)) {  // not positive, or lambda not finite
      if (lead) {
        st->pq = pq;
        st->xpend = 0;
        st->breakdown = 1;
        st->done = 1;
      }
      return;
    }
    if (lead) {
      st->pq = pq;
      st->xpend = 1;
    }
  } else if constexpr (UPD) {
    lamb = st->rho[par] / st->pq;
  }
  const int tid = threadIdx.x, el = tid / NN, t = tid % NN, t1 = t % N, t2 = t / N;
  const int64_t e = (int64_t)blockIdx.x * EPB + el;
  const bool act = el < EPB && e < E;
  const int le = act ? el : 0;
  if (act) {
    for (int i = t; i < 3 * NN; i += NN) sQ[el][i] = Q[e * 3 * NN + i];
    for (int i = t; i < 3 * N; i += NN) sL[el][i] = lam[e * 3 * N + i];
  }
  __syncthreads();
  TV* tile = sT + le * PE;
  const TQ* qx = sQ[le];
  const TQ* qy = sQ[le] + NN;
  const TQ* qz = sQ[le] + 2 * NN;
  TV rl[N], a[N], b[N];
  // x-lines: w = Q_x^T r
  if (act) {
    glb_get<N, 0, TV, TV>(r, e, t1, t2, rl);
    if (UPD) {
      TV ql[N];
      glb_get<N, 0, TV, TV>(q, e, t1, t2, ql);
      TV* pr = r + e * NN * N;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        rl[i] = (TV)((double)rl[i] - lamb * (double)ql[i]);
        pr[lidx<N, 0>(t1, t2, i)] = rl[i];
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) rl[i] = TV(0);
  }
#pragma unroll
  for (int j = 0; j < N; ++j) {
    TV s = TV(0);
#pragma unroll
    for (int i = 0; i < N; ++i) s += (TV)qx[i * N + j] * rl[i];
    b[j] = s;
  }
  if (act) lds_put<N, 0>(tile, t1, t2, b);  // threads without an element write nothing
  __syncthreads();
  lds_get<N, 1>(tile, t1, t2, a);  // y-lines: Q_y^T
#pragma unroll
  for (int j = 0; j < N; ++j) {
    TV s = TV(0);
#pragma unroll
    for (int i = 0; i < N; ++i) s += (TV)qy[i * N + j] * a[i];
    b[j] = s;
  }
  if (act) lds_put<N, 1>(tile, t1, t2, b);
  __syncthreads();
  lds_get<N, 2>(tile, t1, t2, a);  // z-lines: Q_z^T, scale (modes j1 = t1, j2 = t2), Q_z
  {
    const TV lxy = (TV)sL[le][t1] + (TV)sL[le][N + t2];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      TV s = TV(0);
#pragma unroll
      for (int i = 0; i < N; ++i) s += (TV)qz[i * N + j] * a[i];
      b[j] = s / (lxy + (TV)sL[le][2 * N + j]);
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      TV s = TV(0);
#pragma unroll
      for (int j = 0; j < N; ++j) s += (TV)qz[i * N + j] * b[j];
      a[i] = s;
    }
  }
  if (act) lds_put<N, 2>(tile, t1, t2, a);
  __syncthreads();
  lds_get<N, 1>(tile, t1, t2, a);  // y-lines: Q_y
#pragma unroll
  for (int i = 0; i < N; ++i) {
    TV s = TV(0);
#pragma unroll
    for (int j = 0; j < N; ++j) s += (TV)qy[i * N + j] * a[j];
    b[i] = s;
  }
  if (act) lds_put<N, 1>(tile, t1, t2, b);
  __syncthreads();
  lds_get<N, 0>(tile, t1, t2, a);  // x-lines: Q_x, out
  double zr = 0.0, rr = 0.0;
  if (act) {
    TV* pz = z + e * NN * N;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      TV s = TV(0);
#pragma unroll
      for (int j = 0; j < N; ++j) s += (TV)qx[i * N + j] * a[j];
      pz[lidx<N, 0>(t1, t2, i)] = s;
      zr += (double)s * (double)rl[i];
      rr += (double)rl[i] * (double)rl[i];
    }
  }
  const double mine[2] = {block_sum<kBlock>(zr, red), block_sum<kBlock>(rr, red)};
  store_partials<2>(mine, partials, blockIdx.x);
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
  constexpr int NN = N * N, EPB = elems_per_block(N), PE = Lay<N, double>::PE;
  __shared__ double sU[EPB * PE], sV[EPB * PE], sW[EPB * PE], sX[EPB * PE];
  __shared__ double sF[EPB][2][NN];
  __shared__ double sPart[kBlock];
  const Tables<double>& T = *m.tab;
  const int tid = threadIdx.x, el = tid / NN, t = tid % NN, t1 = t % N, t2 = t / N;
  const int64_t e = (int64_t)blockIdx.x * EPB + el;
  const bool act = (el < EPB) && (e < m.E);
  const int le = act ? el : 0;
  double* U = sU + le * PE;
  double* V = sV + le * PE;
  double* W = sW + le * PE;
  double* X = sX + le * PE;
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
    line_op<N, double, false>(T, lv, z0, z0, false, false, 0.0, 0.0, m.vs[2], m.ih[2], m.sg[2], m.At[2], false, w);
    lds_put<N, 2>(W, t1, t2, w);
  }
  __syncthreads();
  if (act) {  // Y
    double lv[N], w[N];
    lds_get<N, 1>(V, t1, t2, lv);
    line_op<N, double, false>(T, lv, z0, z0, false, false, 0.0, 0.0, m.vs[1], m.ih[1], m.sg[1], m.At[1], false, w);
    lds_put<N, 1>(X, t1, t2, w);
  }
  __syncthreads();
  if (act) {  // X
    double lv[N], wx[N], wy[N], wz[N], c[N], ee[N];
    lds_get<N, 0>(V, t1, t2, lv);
    line_op<N, double, false>(T, lv, z0, z0, false, false, 0.0, 0.0, m.vs[0], m.ih[0], m.sg[0], m.At[0], false, wx);
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

// Face coefficients G[6e + 2d + s] = K K' / (K + K') (interior, = gamma_e / 2)
// or K (Dirichlet face), in FP64 and FP32.
__global__ void k_face_coef(MeshArgs<double> m, double* __restrict__ G64, float* __restrict__ G32) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.E) return;
  const int ex = (int)(e % m.nx), ey = (int)((e / m.nx) % m.ny), ez = (int)(e / ((int64_t)m.nx * m.ny));
  const double K = m.K[e];
#pragma unroll
  for (int D = 0; D < 3; ++D)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      int64_t nb;
      if (D == 0) nb = neighbour<0>(m, ex, ey, ez, s);
      else if (D == 1) nb = neighbour<1>(m, ex, ey, ez, s);
      else nb = neighbour<2>(m, ex, ey, ez, s);
      double g = K;
      if (nb >= 0) {
        const double Kn = m.K[nb];
        g = K * Kn / (K + Kn);
      }
      G64[6 * e + 2 * D + s] = g;
      G32[6 * e + 2 * D + s] = (float)g;
    }
}

hipError_t launch_face_coef(const MeshArgs<double>& m, double* G64, float* G32, hipStream_t s) {
  hipLaunchKernelGGL(k_face_coef, dim3((unsigned)((m.E + 255) / 256)), dim3(256), 0, s, m, G64, G32);
  return hipGetLastError();
}

// ---------------------------------------------------------------- launchers

int64_t element_blocks(int n, int64_t E) {
  const int epb = elems_per_block(n);
  return (E + epb - 1) / epb;
}

int64_t affine_tiles(int n, int nx, int ny, int nz) {
  const int bx = tile_x(n), by = tile_y(n), bz = tile_z(n);
  return (int64_t)((nx + bx - 1) / bx) * ((ny + by - 1) / by) * ((nz + bz - 1) / bz);
}

template <int N, typename TIN, typename TOUT, typename TC, bool TRANS, bool DOT>
static hipError_t run_apply(const MeshArgs<TC>& m, const void* x, void* y, double* partials, CgState* st,
                            int par, const int* skip, hipStream_t s, int nrhs = 1) {
  const int64_t nb = affine_tiles(N, m.nx, m.ny, m.nz);
  // 32-bit byte offsets when every vector and the face coefficients stay below 4 GiB
  const double nd = (double)m.E * N * N * N;
  const bool off32 = nd * (double)(sizeof(TIN) > sizeof(TOUT) ? sizeof(TIN) : sizeof(TOUT)) < 4294967296.0 &&
                     6.0 * (double)m.E * sizeof(TC) < 4294967296.0;
  hipError_t e;
  if (off32)
    hipLaunchKernelGGL((k_apply_affine<N, TIN, TOUT, TC, TRANS, DOT, true>), dim3((unsigned)nb, (unsigned)nrhs),
                       dim3(apply_block(N)), 0, s, m, (const TIN*)x, (TOUT*)y, partials, skip);
  else
    hipLaunchKernelGGL((k_apply_affine<N, TIN, TOUT, TC, TRANS, DOT, false>), dim3((unsigned)nb, (unsigned)nrhs),
                       dim3(apply_block(N)), 0, s, m, (const TIN*)x, (TOUT*)y, partials, skip);
  e = hipGetLastError();
  if (e != hipSuccess || !DOT || st == nullptr) return e;  // st == nullptr: partials only
  return launch_finish_dot(partials, nb, st, par, s);
}

template <int N, bool TRANS, bool DOT>
static hipError_t run_apply_prec(int prec, const MeshArgs<double>& m64, const MeshArgs<float>& m32,
                                 const void* x, void* y, double* partials, CgState* st, int par,
                                 const int* skip, hipStream_t s) {
  switch (prec) {
    case 0: return run_apply<N, double, double, double, TRANS, DOT>(m64, x, y, partials, st, par, skip, s);
    case 1: return run_apply<N, float, float, float, TRANS, DOT>(m32, x, y, partials, st, par, skip, s);
    case 2: return run_apply<N, uint16_t, float, float, TRANS, DOT>(m32, x, y, partials, st, par, skip, s);
    case 3: {  // BF16 input, tangential masses on MFMA (the operator is symmetric: A^T x is the same product)
      const int64_t nb = affine_tiles(N, m32.nx, m32.ny, m32.nz);
      hipError_t e = launch_apply_affine_mfma(N, DOT ? 1 : 0, m32, (const uint16_t*)x, (float*)y, partials, skip, s);
      if (e != hipSuccess || !DOT || st == nullptr) return e;
      return launch_finish_dot(partials, nb, st, par, s);
    }
  }
  return hipErrorInvalidValue;
}

template <int N>
static hipError_t run_apply_n(int prec, int trans, int dot, const MeshArgs<double>& m64,
                              const MeshArgs<float>& m32, const void* x, void* y, double* partials,
                              CgState* st, int par, const int* skip, hipStream_t s) {
  if (trans) {
    if (dot) return run_apply_prec<N, true, true>(prec, m64, m32, x, y, partials, st, par, skip, s);
    return run_apply_prec<N, true, false>(prec, m64, m32, x, y, partials, st, par, skip, s);
  }
  if (dot) return run_apply_prec<N, false, true>(prec, m64, m32, x, y, partials, st, par, skip, s);
  return run_apply_prec<N, false, false>(prec, m64, m32, x, y, partials, st, par, skip, s);
}

hipError_t launch_apply_affine(int n, int prec, int trans, int dot, const MeshArgs<double>& m64,
                               const MeshArgs<float>& m32, const void* x, void* y, double* partials,
                               CgState* st, int par, const int* skip, hipStream_t s) {
  switch (n) {
    case 2: return run_apply_n<2>(prec, trans, dot, m64, m32, x, y, partials, st, par, skip, s);
    case 3: return run_apply_n<3>(prec, trans, dot, m64, m32, x, y, partials, st, par, skip, s);
    case 4: return run_apply_n<4>(prec, trans, dot, m64, m32, x, y, partials, st, par, skip, s);
    case 5: return run_apply_n<5>(prec, trans, dot, m64, m32, x, y, partials, st, par, skip, s);
    case 6: return run_apply_n<6>(prec, trans, dot, m64, m32, x, y, partials, st, par, skip, s);
    case 7: return run_apply_n<7>(prec, trans, dot, m64, m32, x, y, partials, st, par, skip, s);
    case 8: return run_apply_n<8>(prec, trans, dot, m64, m32, x, y, partials, st, par, skip, s);
  }
  return hipErrorInvalidValue;
}

template <int N>
static hipError_t run_diag(const MeshArgs<double>& m, double* d, const int* run, hipStream_t s) {
  const int64_t tot = m.E * N * N * N;
  hipLaunchKernelGGL((k_diag_affine<N>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, m, d, run);
  return hipGetLastError();
}
hipError_t launch_diag_affine(int n, const MeshArgs<double>& m, double* d, const int* run, hipStream_t s) {
  switch (n) {
    case 2: return run_diag<2>(m, d, run, s);
    case 3: return run_diag<3>(m, d, run, s);
    case 4: return run_diag<4>(m, d, run, s);
    case 5: return run_diag<5>(m, d, run, s);
    case 6: return run_diag<6>(m, d, run, s);
    case 7: return run_diag<7>(m, d, run, s);
    case 8: return run_diag<8>(m, d, run, s);
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

// ------------------------------------------------------------ multi-vector apply
template <int N, bool TRANS>
static hipError_t run_multi(int prec, int nrhs, const MeshArgs<double>& m64, const MeshArgs<float>& m32, const void* x,
                            void* y, hipStream_t s) {
  switch (prec) {
    case 0: return run_apply<N, double, double, double, TRANS, false>(m64, x, y, nullptr, nullptr, 0, nullptr, s, nrhs);
    case 1: return run_apply<N, float, float, float, TRANS, false>(m32, x, y, nullptr, nullptr, 0, nullptr, s, nrhs);
    case 2: return run_apply<N, uint16_t, float, float, TRANS, false>(m32, x, y, nullptr, nullptr, 0, nullptr, s, nrhs);
    case 3: return launch_apply_affine_mfma(N, 0, m32, (const uint16_t*)x, (float*)y, nullptr, nullptr, s, nrhs);
  }
  return hipErrorInvalidValue;
}
template <int N>
static hipError_t run_multi_n(int prec, int trans, int nrhs, const MeshArgs<double>& m64, const MeshArgs<float>& m32,
                              const void* x, void* y, hipStream_t s) {
  return trans ? run_multi<N, true>(prec, nrhs, m64, m32, x, y, s) : run_multi<N, false>(prec, nrhs, m64, m32, x, y, s);
}
hipError_t launch_apply_affine_multi(int n, int prec, int trans, int nrhs, const MeshArgs<double>& m64,
                                     const MeshArgs<float>& m32, const void* x, void* y, hipStream_t s) {
  switch (n) {
    case 2: return run_multi_n<2>(prec, trans, nrhs, m64, m32, x, y, s);
    case 3: return run_multi_n<3>(prec, trans, nrhs, m64, m32, x, y, s);
    case 4: return run_multi_n<4>(prec, trans, nrhs, m64, m32, x, y, s);
    case 5: return run_multi_n<5>(prec, trans, nrhs, m64, m32, x, y, s);
    case 6: return run_multi_n<6>(prec, trans, nrhs, m64, m32, x, y, s);
    case 7: return run_multi_n<7>(prec, trans, nrhs, m64, m32, x, y, s);
    case 8: return run_multi_n<8>(prec, trans, nrhs, m64, m32, x, y, s);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------ block-Jacobi launchers
template <int N>
static hipError_t run_bj_setup(const MeshArgs<double>& m, double* Q, double* lam, float* Q32, float* lam32,
                               hipStream_t s) {
  hipLaunchKernelGGL((k_bj_setup<N>), dim3((unsigned)((3 * m.E + 255) / 256)), dim3(256), 0, s, m, Q, lam, Q32, lam32);
  return hipGetLastError();
}
hipError_t launch_bj_setup(int n, const MeshArgs<double>& m, double* Q, double* lam, float* Q32, float* lam32,
                           hipStream_t s) {
  switch (n) {
    case 2: return run_bj_setup<2>(m, Q, lam, Q32, lam32, s);
    case 3: return run_bj_setup<3>(m, Q, lam, Q32, lam32, s);
    case 4: return run_bj_setup<4>(m, Q, lam, Q32, lam32, s);
    case 5: return run_bj_setup<5>(m, Q, lam, Q32, lam32, s);
    case 6: return run_bj_setup<6>(m, Q, lam, Q32, lam32, s);
    case 7: return run_bj_setup<7>(m, Q, lam, Q32, lam32, s);
    case 8: return run_bj_setup<8>(m, Q, lam, Q32, lam32, s);
  }
  return hipErrorInvalidValue;
}
template <int N, typename TV, typename TQ>
static hipError_t run_bj_apply(int64_t E, const TQ* Q, const TQ* lam, TV* r, TV* z, double* partials,
                               const int* skip, const TV* q, CgState* st, int par, const double* partA, int64_t nbA,
                               hipStream_t s) {
  const dim3 grid((unsigned)element_blocks(N, E));
  if (q != nullptr && partA != nullptr)
    hipLaunchKernelGGL((k_bj_apply<N, TV, TQ, true, true>), grid, dim3(kBlock), 0, s, E, Q, lam, r, z, partials,
                       skip, q, st, par, partA, nbA);
  else if (q != nullptr)
    hipLaunchKernelGGL((k_bj_apply<N, TV, TQ, true, false>), grid, dim3(kBlock), 0, s, E, Q, lam, r, z, partials,
                       skip, q, st, par, partA, nbA);
  else
    hipLaunchKernelGGL((k_bj_apply<N, TV, TQ, false, false>), grid, dim3(kBlock), 0, s, E, Q, lam, r, z, partials,
                       skip, q, st, par, partA, nbA);
  return hipGetLastError();
}
template <typename TV, typename TQ>
hipError_t launch_bj_apply(int n, int64_t E, const TQ* Q, const TQ* lam, TV* r, TV* z, double* partials,
                           const int* skip, hipStream_t s, const TV* q, CgState* st, int par, const double* partA,
                           int64_t nbA) {
  switch (n) {
    case 2: return run_bj_apply<2, TV, TQ>(E, Q, lam, r, z, partials, skip, q, st, par, partA, nbA, s);
    case 3: return run_bj_apply<3, TV, TQ>(E, Q, lam, r, z, partials, skip, q, st, par, partA, nbA, s);
    case 4: return run_bj_apply<4, TV, TQ>(E, Q, lam, r, z, partials, skip, q, st, par, partA, nbA, s);
    case 5: return run_bj_apply<5, TV, TQ>(E, Q, lam, r, z, partials, skip, q, st, par, partA, nbA, s);
    case 6: return run_bj_apply<6, TV, TQ>(E, Q, lam, r, z, partials, skip, q, st, par, partA, nbA, s);
    case 7: return run_bj_apply<7, TV, TQ>(E, Q, lam, r, z, partials, skip, q, st, par, partA, nbA, s);
    case 8: return run_bj_apply<8, TV, TQ>(E, Q, lam, r, z, partials, skip, q, st, par, partA, nbA, s);
  }
  return hipErrorInvalidValue;
}
template hipError_t launch_bj_apply<double, double>(int, int64_t, const double*, const double*, double*, double*,
                                                    double*, const int*, hipStream_t, const double*, CgState*, int,
                                                    const double*, int64_t);
template hipError_t launch_bj_apply<float, float>(int, int64_t, const float*, const float*, float*, float*, double*,
                                                  const int*, hipStream_t, const float*, CgState*, int,
                                                  const double*, int64_t);

}  // namespace dg
