// dg_ppd.hip -- sum-factorised SWIPDG apply on meshes whose elements are all
// the same parallelepiped: an affine image x = J xi of the axis-parallel grid
// (problem B of Sec. 3.3: affine geometries, coefficients per cell).
//
// With the constant metric G = |det J| J^-1 J^-T the element form is the
// axis-parallel one with a full 3 x 3 coefficient: on the reference grid
//
//     K grad u . grad v |det J| = K sum_ab G_ab d_a u d_b v,
//
// and on a face normal to axis d the area-weighted conormal is G e_d.  The
// diagonal entries G_dd, the face areas |J e_a x J e_b| and the penalty
// sigma_e = sig_hat / h_d (h_d = 1 / n_d, as on axis-parallel meshes) enter
// the 1D line operators L_d of the axis-parallel apply unchanged (volume
// scale G_dd, normal-flux scale G_dd, penalty area |F_d|).  Each
// off-diagonal entry G_ab (a < b, c the third axis) adds
//
//     G_ab M_c (x) P_ab,
//
// P_ab the mixed-derivative part of the form in the (a, b) plane: the volume
// term K (C_a (x) C_b^T + C_a^T (x) C_b) with C_ij = int l_i l_j', and the
// tangential parts of the consistency and symmetry terms on the a- and
// b-faces.  Since C + C^T = E = diag(-1, 0, ..., 0, 1) (integration by
// parts on GLL nodes), the volume term is -2 K C_a (x) C_b plus E terms on
// the element's faces, and face by face the three pieces combine to
//
//     a-face at the upper end:  C_b X_hi + G_hi E_b (U_hi - u_hi),
//     a-face at the lower end: -C_b X_lo + G_lo E_b (u_lo - U_lo),
//     X = K u - 2 G U,
//
// with u the element's trace on the face, U the neighbour's (0 on a
// Dirichlet face), G the face coefficient (gamma / 2 on interior faces, K on
// Dirichlet faces).  So
//
//     P_ab = C_b (-2 K C_a u + a-face rows X) + C_a (b-face rows X) + corners,
//
// the a-face rows riding on the a-line contraction, the b-face rows needing
// one contraction along a of the face row, and the E terms landing on the
// four edges of the (a, b) plane.  The transpose is the same operator (the
// form is symmetric).
//
// Phases (one more LDS tile than the axis-parallel apply, S3, and small
// per-element exchange rows; P_ab is symmetric in a and b, so each pair is
// formed in the phase whose lines suit it):
//   X : b_x -> S1; x-face rows X and jumps
//   Y : b_y -> S2; S1 <- M_y S1; c_y = -2K C u + y-face rows -> S3; y-face jumps
//   X2: S1 <- S1 + M_x S2 + G_xy P_xy,  P_xy = C_x c_y + C_y (x-face rows) + corners
//   Z : b_z -> S2; r = M_z S1; S1 <- P_yz = C_z c_y + C_y (z-face rows) + corners;
//       c_z = -2K C u + z-face rows -> S3
//   X3: S2 <- M_x S2 + G_xz P_xz,  P_xz = C_x c_z + C_z (x-face rows) + corners;
//       S1 <- G_yz M_x S1
//   Y3: S2 <- M_y S2
//   Z2: y = r + S2 + S1
// so that y = M_z (M_y b_x + M_x b_y + G_xy P_xy) + M_y (M_x b_z + G_xz P_xz)
//         + G_yz M_x P_yz.
#include "dg_internal.hpp"
#include "dg_kernels.hpp"
#include "dg_lines.hpp"
#include "dg_faces.hpp"

namespace dg {

// out = C a along the line (C centro-antisymmetric: even-odd halves from n = 4,
// where they cost no more operations and hold half the table in scalar registers)
template <int N, typename TC>
__device__ __forceinline__ void cd_line(const Tables<TC>& T, const TC (&a)[N], TC (&out)[N]) {
  if constexpr (N >= 4) {
    contract_eo<N, TC, -1>(T.eC, a, out);
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      TC s = TC(0);
#pragma unroll
      for (int j = 0; j < N; ++j) s += T.Cd[i * kMaxN + j] * a[j];
      out[i] = s;
    }
  }
}

__host__ __device__ constexpr size_t lds_units(size_t bytes) { return (bytes + 1023) / 1024 * 1024; }

template <int N, typename TIN, typename TOUT, typename TC, bool DOT, bool OFF32>
__global__ __launch_bounds__(apply_block(N)) void k_apply_ppd(MeshArgs<TC> m, const TIN* __restrict__ x,
                                                              TOUT* __restrict__ y, double* partials,
                                                              const int* skip) {
  constexpr int NN = N * N, N3 = NN * N;
  constexpr int BX = tile_x(N), BY = tile_y(N), BZ = tile_z(N), TE = BX * BY * BZ;
  constexpr int LV = 1;  // the denser tile layout: LDS bounds this kernel's occupancy
  constexpr int PE = Lay<N, TC, LV>::PE;
  constexpr bool F_IN_S2 = 4 * NN <= PE;
  constexpr int FS = F_IN_S2 ? PE : 4 * NN;
  constexpr int BLOCK = apply_block(N);
  static_assert(TE * NN <= BLOCK && BLOCK <= kBlock, "brick too large");
  // an element's threads lie in one wavefront (ELEM), and so does each x-row
  // of the brick (XROW): exchanges inside an element then need only
  // wavefront-level synchronisation (every exchange outside the face phases is)
  constexpr bool ELEM = 64 % NN == 0, XROW = 64 % (BX * NN) == 0;
  // padding lanes repeat the work of the brick's last element lane for lane
  // (same values to the same LDS words, in the same wavefront)
  static_assert(TE * NN == BLOCK || BLOCK - (TE - 1) * NN <= 64, "padding lanes and their twins share a wavefront");
  // per element, lower and upper side each: x-face rows X, y-face jumps, z-face rows X, z-face jumps.
  // The z-face rows live only inside the Z phase: where moving them into the
  // element's face-scalar slot (free once the Z face scalars have been read,
  // at the cost of one or two more barriers) lets one more workgroup fit in a
  // CU's LDS, they go there (ZR_IN_F) and sP keeps six rows
  constexpr size_t LDS_BASE = (3 * TE * PE + (F_IN_S2 ? 1 : TE * 4 * NN) + NN) * sizeof(TC) + BLOCK / 64 * 8;
  // (a CU holds at most 32 waves and 160 KB of LDS, granted in 1 KB units as
  // measured: 54.1 KB per workgroup left room for two at n = 7, 53.3 KB for three)
  constexpr size_t LDS_CU = 160 * 1024, MAX_WG = 32 / (BLOCK / 64);
  constexpr size_t WG6 = LDS_CU / lds_units(LDS_BASE + TE * 6 * NN * sizeof(TC));
  constexpr size_t WG8 = LDS_CU / lds_units(LDS_BASE + TE * 8 * NN * sizeof(TC));
  constexpr bool ZR_IN_F = (WG6 < MAX_WG ? WG6 : MAX_WG) > (WG8 < MAX_WG ? WG8 : MAX_WG);
  constexpr int PR = ZR_IN_F ? 6 : 8;  // rows per element in sP
  constexpr int JZ = ZR_IN_F ? 4 : 6;  // first z-face jump row
  __shared__ TC sS1[TE * PE], sS2[TE * PE], sS3[TE * PE];
  __shared__ TC sFx[F_IN_S2 ? 1 : TE * 4 * NN];
  __shared__ TC sP[TE * PR * NN];
  __shared__ TC sC[NN];  // C, row-major, for lane-indexed rows
  __shared__ double red[BLOCK / 64];
  if (skip != nullptr && *skip) return;
  // vector blockIdx.y of a multi-vector apply (the vectors follow each other)
  x += (size_t)blockIdx.y * (size_t)m.E * N3;
  y += (size_t)blockIdx.y * (size_t)m.E * N3;
  TC* F = F_IN_S2 ? sS2 : sFx;
  // The 1D tables are read through the scalar cache.  Each phase re-derives
  // their address, which keeps the compiler from holding every table in
  // scalar registers across the whole kernel (at n >= 4 they do not fit and
  // spill into vector-register lanes): a phase loads the tables it uses.
  auto tabs = [&]() -> const Tables<TC>& {
    uint64_t a = (uint64_t)m.tab;
    asm volatile("" : "+s"(a));
    typedef const __attribute__((address_space(4))) Tables<TC>* ConstTab;
    return *(const Tables<TC>*)(ConstTab)a;
  };
  const int tb = (int)xcd_remap(blockIdx.x, gridDim.x);
  int o[3];
  brick_origin<BX, BY, BZ>(tb, m.nx, m.ny, m.nz, o);
  const int Nd[3] = {m.nx, m.ny, m.nz};
  const int tid = threadIdx.x, el0 = tid / NN, t = tid - el0 * NN, t1 = t % N, t2 = t / N;
  const int el = min(el0, TE - 1);
  const int lx = el % BX, ly = (el / BX) % BY, lz = el / (BX * BY);
  const int cu[3] = {o[0] + lx, o[1] + ly, o[2] + lz};
  // own: the lane's element lies in the mesh (overhanging elements compute on
  // the nearest mesh element without neighbours); act: own and not padding
  const bool own = cu[0] < m.nx && cu[1] < m.ny && cu[2] < m.nz;
  const bool act = el0 < TE && own;
  const int c[3] = {min(cu[0], m.nx - 1), min(cu[1], m.ny - 1), min(cu[2], m.nz - 1)};
  TC* S1 = sS1 + el * PE;
  TC* S2 = sS2 + el * PE;
  TC* S3 = sS3 + el * PE;
  TC* Fe = F + el * FS;
  TC* P = sP + el * PR * NN;
  TC* ZR = ZR_IN_F ? Fe : P + 4 * NN;  // the element's z-face rows: lower side, then upper side
  if (tid < NN) sC[tid] = tabs().Cd[(tid / N) * kMaxN + tid % N];
  const int64_t e = c[0] + (int64_t)m.nx * (c[1] + (int64_t)m.ny * c[2]);
  const uint32_t eo = (uint32_t)e * (uint32_t)N3;  // the element's first entry (N_dof < 2^31)
  const TC K = m.K[e], K2 = TC(-2) * K;
  auto gco = [&](int f) { return OFF32 ? m.G[(uint32_t)(6 * e + f)] : m.G[6 * e + f]; };
  const TC gxy = m.go[0], gxz = m.go[1], gyz = m.go[2];
  TC b[N], v[N], w[N], u[N], tr[2];
  TC jxl, jxh;  // this thread's x-face jumps at (y, z) = (t1, t2), used again in X2 and X3
  // ---------------- X: b_x -> S1, x-face rows and jumps
  {
    const Tables<TC>& T = tabs();
    const TC GL = gco(0), GH = gco(1);
    face_phase<N, 0, BX, BY, BZ, FS, TC, TIN, false, OFF32>(m, T, x, own, eo, c, o, Nd, t, t1, t2, Fe, K, GL, GH,
                                                            TC(0), b, u, tr);
    lds_put<N, 0, TC, LV>(S1, t1, t2, b);
    P[0 * NN + t] = K * u[0] - TC(2) * GL * tr[0];
    P[1 * NN + t] = K * u[N - 1] - TC(2) * GH * tr[1];
    jxl = GL * (u[0] - tr[0]);
    jxh = GH * (tr[1] - u[N - 1]);
  }
  lds_sync<XROW>();  // F (read by the x-neighbours) is rewritten by the next phase
  // ---------------- Y: b_y -> S2, S1 <- M_y S1, c_y -> S3, y-face jumps
  {
    const Tables<TC>& T = tabs();
    const TC GL = gco(2), GH = gco(3);
    face_phase<N, 1, BX, BY, BZ, FS, TC, TIN, false, OFF32>(m, T, x, own, eo, c, o, Nd, t, t1, t2, Fe, K, GL, GH,
                                                            TC(0), b, u, tr);
    lds_get<N, 1, TC, LV>(S1, t1, t2, v);
    mass_line<N, TC, false>(T, v, w);
    cd_line<N, TC>(T, u, v);
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] *= K2;
    v[N - 1] += K * u[N - 1] - TC(2) * GH * tr[1];  // the y-face rows ride on c_y
    v[0] -= K * u[0] - TC(2) * GL * tr[0];
    P[2 * NN + t] = GL * (u[0] - tr[0]);  // y-face jumps at (x, z) = (t1, t2)
    P[3 * NN + t] = GH * (tr[1] - u[N - 1]);
    if (F_IN_S2) __syncthreads();  // the face scalars in S2 have been read
    lds_put<N, 1, TC, LV>(S2, t1, t2, b);
    lds_put<N, 1, TC, LV>(S1, t1, t2, w);
    lds_put<N, 1, TC, LV>(S3, t1, t2, v);
  }
  lds_sync<ELEM>();
  // ---------------- X2: S1 <- S1 + M_x S2 + G_xy P_xy,  P_xy = C_x c_y + C_y (x-face rows) + corners
  {
    const Tables<TC>& T = tabs();
    lds_get<N, 0, TC, LV>(S2, t1, t2, v);
    lds_get<N, 0, TC, LV>(S1, t1, t2, w);
    mass_line<N, TC, false>(T, v, b);
#pragma unroll
    for (int i = 0; i < N; ++i) w[i] += b[i];
    lds_get<N, 0, TC, LV>(S3, t1, t2, v);
    TC p[N];
    cd_line<N, TC>(T, v, p);
    TC sh = TC(0), sl = TC(0);  // x-face rows contracted along y, at y = t1
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const TC cj = sC[t1 * N + j];
      sh += cj * P[1 * NN + j + N * t2];
      sl += cj * P[0 * NN + j + N * t2];
    }
    p[N - 1] += sh;
    p[0] -= sl;
    if (t1 == N - 1) {  // edges of the (x, y) plane: own x-face jumps, y-face jumps at x = 0 / n-1
      p[N - 1] += jxh + P[3 * NN + (N - 1) + N * t2];
      p[0] += jxl - P[3 * NN + N * t2];
    } else if (t1 == 0) {
      p[N - 1] += P[2 * NN + (N - 1) + N * t2] - jxh;
      p[0] -= jxl + P[2 * NN + N * t2];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) w[i] += gxy * p[i];
    lds_put<N, 0, TC, LV>(S1, t1, t2, w);
  }
  lds_sync<ELEM>();
  // ---------------- Z: b_z -> S2, r = M_z S1, P_yz -> S1, c_z -> S3, z-face rows and jumps
  TC r[N];
  {
    const Tables<TC>& T = tabs();
    const TC GL = gco(4), GH = gco(5);
    const TC cr = m.R ? m.R[e] * m.vol : TC(0);
    face_phase<N, 2, BX, BY, BZ, FS, TC, TIN, false, OFF32>(m, T, x, own, eo, c, o, Nd, t, t1, t2, Fe, K, GL, GH,
                                                            cr, b, u, tr);
    lds_get<N, 2, TC, LV>(S1, t1, t2, v);
    mass_line<N, TC, false>(T, v, r);
    const TC Xlo = K * u[0] - TC(2) * GL * tr[0], Xhi = K * u[N - 1] - TC(2) * GH * tr[1];
    const TC jzl = GL * (u[0] - tr[0]), jzh = GH * (tr[1] - u[N - 1]);
    if constexpr (!ZR_IN_F) {  // z-face rows and jumps at (x, y) = (t1, t2)
      ZR[t] = Xlo;
      ZR[NN + t] = Xhi;
    }
    P[JZ * NN + t] = jzl;
    P[(JZ + 1) * NN + t] = jzh;
    TC p[N];
    lds_get<N, 2, TC, LV>(S3, t1, t2, v);
    cd_line<N, TC>(T, v, p);  // P_yz = C_z c_y + ...
    cd_line<N, TC>(T, u, w);  // c_z
#pragma unroll
    for (int i = 0; i < N; ++i) w[i] *= K2;
    w[N - 1] += Xhi;
    w[0] -= Xlo;
    // the face scalars (in S2 or in their own slots) have been read; the
    // z-face rows are published
    if (F_IN_S2 || ZR_IN_F) __syncthreads();
    else lds_sync<ELEM>();
    if constexpr (ZR_IN_F) {  // into the face-scalar slot, free from here on
      ZR[t] = Xlo;
      ZR[NN + t] = Xhi;
      lds_sync<ELEM>();
    }
    TC sh = TC(0), sl = TC(0);  // z-face rows contracted along y, at y = t2
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const TC cj = sC[t2 * N + j];
      sh += cj * ZR[NN + t1 + N * j];
      sl += cj * ZR[t1 + N * j];
    }
    p[N - 1] += sh;
    p[0] -= sl;
    if (t2 == N - 1) {  // edges of the (y, z) plane: y-face jumps at z = 0 / n-1, own z-face jumps
      p[N - 1] += P[3 * NN + t1 + N * (N - 1)] + jzh;
      p[0] += jzl - P[3 * NN + t1];
    } else if (t2 == 0) {
      p[N - 1] += P[2 * NN + t1 + N * (N - 1)] - jzh;
      p[0] -= P[2 * NN + t1] + jzl;
    }
    if constexpr (ZR_IN_F && F_IN_S2) lds_sync<ELEM>();  // the rows in S2 have been read
    lds_put<N, 2, TC, LV>(S2, t1, t2, b);
    lds_put<N, 2, TC, LV>(S1, t1, t2, p);  // the thread's own z-lines of S1 and S3 were read above
    lds_put<N, 2, TC, LV>(S3, t1, t2, w);
  }
  lds_sync<ELEM>();
  // ---------------- X3: S2 <- M_x S2 + G_xz P_xz (P_xz = C_x c_z + C_z (x-face rows) + corners),
  //                      S1 <- G_yz M_x S1
  {
    const Tables<TC>& T = tabs();
    lds_get<N, 0, TC, LV>(S2, t1, t2, v);
    mass_line<N, TC, false>(T, v, w);
    lds_get<N, 0, TC, LV>(S3, t1, t2, v);
    TC p[N];
    cd_line<N, TC>(T, v, p);
    TC sh = TC(0), sl = TC(0);  // x-face rows contracted along z, at z = t2
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const TC cj = sC[t2 * N + j];
      sh += cj * P[1 * NN + t1 + N * j];
      sl += cj * P[0 * NN + t1 + N * j];
    }
    p[N - 1] += sh;
    p[0] -= sl;
    if (t2 == N - 1) {  // edges of the (x, z) plane: own x-face jumps, z-face jumps at x = 0 / n-1
      p[N - 1] += jxh + P[(JZ + 1) * NN + (N - 1) + N * t1];
      p[0] += jxl - P[(JZ + 1) * NN + N * t1];
    } else if (t2 == 0) {
      p[N - 1] += P[JZ * NN + (N - 1) + N * t1] - jxh;
      p[0] -= jxl + P[JZ * NN + N * t1];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) w[i] += gxz * p[i];
    lds_put<N, 0, TC, LV>(S2, t1, t2, w);
    lds_get<N, 0, TC, LV>(S1, t1, t2, v);
    mass_line<N, TC, false>(T, v, w);
#pragma unroll
    for (int i = 0; i < N; ++i) w[i] *= gyz;
    lds_put<N, 0, TC, LV>(S1, t1, t2, w);
  }
  lds_sync<ELEM>();
  // ---------------- Y3: S2 <- M_y S2
  {
    const Tables<TC>& T = tabs();
    lds_get<N, 1, TC, LV>(S2, t1, t2, v);
    mass_line<N, TC, false>(T, v, w);
    lds_put<N, 1, TC, LV>(S2, t1, t2, w);
  }
  lds_sync<ELEM>();
  // ---------------- Z2: y = r + S2 + S1
  double part = 0.0;
  lds_get<N, 2, TC, LV>(S2, t1, t2, v);
  lds_get<N, 2, TC, LV>(S1, t1, t2, w);
  if (act) {
    const uint32_t yb = (eo + (uint32_t)lidx<N, 2>(t1, t2, 0)) * (uint32_t)sizeof(TOUT);
    TOUT* py = y + e * N3;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const TOUT yv = (TOUT)(r[i] + v[i] + w[i]);
      TOUT* dst = OFF32 ? (TOUT*)((char*)y + (yb + (uint32_t)(lidx<N, 2>(0, 0, i) * sizeof(TOUT))))
                        : &py[lidx<N, 2>(t1, t2, i)];
      __builtin_nontemporal_store(yv, dst);
      if (DOT) part += (double)u[i] * (double)yv;
    }
  }
  if (DOT) {
    const double mine[1] = {block_sum<BLOCK>(part, red)};
    store_partials<1>(mine, partials, blockIdx.x);
  }
}

// ---------------------------------------------------------------- launchers
template <int N, typename TIN, typename TOUT, typename TC, bool DOT>
static hipError_t run_ppd(const MeshArgs<TC>& m, const void* x, void* y, double* partials, CgState* st, int par,
                          const int* skip, hipStream_t s, int nrhs = 1) {
  const int64_t nb = affine_tiles(N, m.nx, m.ny, m.nz);
  const double nd = (double)m.E * N * N * N;
  const bool off32 = nd * (double)(sizeof(TIN) > sizeof(TOUT) ? sizeof(TIN) : sizeof(TOUT)) < 4294967296.0 &&
                     6.0 * (double)m.E * sizeof(TC) < 4294967296.0;
  if (off32)
    hipLaunchKernelGGL((k_apply_ppd<N, TIN, TOUT, TC, DOT, true>), dim3((unsigned)nb, (unsigned)nrhs),
                       dim3(apply_block(N)), 0, s, m, (const TIN*)x, (TOUT*)y, partials, skip);
  else
    hipLaunchKernelGGL((k_apply_ppd<N, TIN, TOUT, TC, DOT, false>), dim3((unsigned)nb, (unsigned)nrhs),
                       dim3(apply_block(N)), 0, s, m, (const TIN*)x, (TOUT*)y, partials, skip);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess || !DOT || st == nullptr) return e;
  return launch_finish_dot(partials, nb, st, par, s);
}

template <int N, bool DOT>
static hipError_t run_ppd_prec(int prec, const MeshArgs<double>& m64, const MeshArgs<float>& m32, const void* x,
                               void* y, double* partials, CgState* st, int par, const int* skip, hipStream_t s) {
  switch (prec) {
    case 0: return run_ppd<N, double, double, double, DOT>(m64, x, y, partials, st, par, skip, s);
    case 1: return run_ppd<N, float, float, float, DOT>(m32, x, y, partials, st, par, skip, s);
    case 2: return run_ppd<N, uint16_t, float, float, DOT>(m32, x, y, partials, st, par, skip, s);
    default: return hipErrorInvalidValue;
  }
}

template <int N>
static hipError_t run_ppd_n(int prec, int dot, const MeshArgs<double>& m64, const MeshArgs<float>& m32,
                            const void* x, void* y, double* partials, CgState* st, int par, const int* skip,
                            hipStream_t s) {
  return dot ? run_ppd_prec<N, true>(prec, m64, m32, x, y, partials, st, par, skip, s)
             : run_ppd_prec<N, false>(prec, m64, m32, x, y, partials, st, par, skip, s);
}

template <int N>
static hipError_t run_ppd_multi(int prec, int nrhs, const MeshArgs<double>& m64, const MeshArgs<float>& m32,
                                const void* x, void* y, hipStream_t s) {
  switch (prec) {
    case 0: return run_ppd<N, double, double, double, false>(m64, x, y, nullptr, nullptr, 0, nullptr, s, nrhs);
    case 1: return run_ppd<N, float, float, float, false>(m32, x, y, nullptr, nullptr, 0, nullptr, s, nrhs);
    case 2: return run_ppd<N, uint16_t, float, float, false>(m32, x, y, nullptr, nullptr, 0, nullptr, s, nrhs);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_apply_ppd_multi(int n, int prec, int nrhs, const MeshArgs<double>& m64, const MeshArgs<float>& m32,
                                  const void* x, void* y, hipStream_t s) {
  switch (n) {
    case 2: return run_ppd_multi<2>(prec, nrhs, m64, m32, x, y, s);
    case 3: return run_ppd_multi<3>(prec, nrhs, m64, m32, x, y, s);
    case 4: return run_ppd_multi<4>(prec, nrhs, m64, m32, x, y, s);
    case 5: return run_ppd_multi<5>(prec, nrhs, m64, m32, x, y, s);
    case 6: return run_ppd_multi<6>(prec, nrhs, m64, m32, x, y, s);
    case 7: return run_ppd_multi<7>(prec, nrhs, m64, m32, x, y, s);
    case 8: return run_ppd_multi<8>(prec, nrhs, m64, m32, x, y, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_apply_ppd(int n, int prec, int dot, const MeshArgs<double>& m64, const MeshArgs<float>& m32,
                            const void* x, void* y, double* partials, CgState* st, int par, const int* skip,
                            hipStream_t s) {
  switch (n) {
    case 2: return run_ppd_n<2>(prec, dot, m64, m32, x, y, partials, st, par, skip, s);
    case 3: return run_ppd_n<3>(prec, dot, m64, m32, x, y, partials, st, par, skip, s);
    case 4: return run_ppd_n<4>(prec, dot, m64, m32, x, y, partials, st, par, skip, s);
    case 5: return run_ppd_n<5>(prec, dot, m64, m32, x, y, partials, st, par, skip, s);
    case 6: return run_ppd_n<6>(prec, dot, m64, m32, x, y, partials, st, par, skip, s);
    case 7: return run_ppd_n<7>(prec, dot, m64, m32, x, y, partials, st, par, skip, s);
    case 8: return run_ppd_n<8>(prec, dot, m64, m32, x, y, partials, st, par, skip, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dg
