// dg_mfma.hip -- BF16-input apply y = A x on affine (axis-parallel box)
// meshes with the tangential mass contractions on the matrix cores.
//
// The affine operator (Sec. 4.1 forms on box elements, Sec. 3.3 sum
// factorisation) is a sum over the axes d of tensor products
//     A = sum_d  (M (x) M)_perp(d) (x) L_d ,
// the 1D mass matrix M on the two axes tangential to d and the 1D DG
// operator L_d (stiffness plus the two faces normal to d) along d.  The two
// factors act on different axes, so the tangential mass can be applied first:
// with z_d = (M (x) M)_perp(d) x on every element (and on the neighbours that
// share a face normal to d),
//     (A x)_T = sum_d L_d z_d ,
// where the face terms of L_d read the neighbour's z_d at the shared face (its
// trace and normal derivative), exactly as they read x in the other kernels.
//
// z_d is a dense product: for each layer l of an element along d, the
// (n^2 x n^2) matrix M (x) M times the n^2 values of x on that plane.  x is
// stored in BF16, so the plane values are exact BF16 operands; the matrix is
// split into three BF16 terms, M (x) M = hi + mid + lo (each the rounding of
// what the previous ones leave, so the sum carries the FP32 value to about
// 2^-27 of an entry), and v_mfma_f32_32x32x16_bf16 accumulates hi x + mid x +
// lo x in FP32 (the product of two BF16 numbers is exact in FP32): the
// arithmetic error is that of an FP32 contraction.
// The rest -- the 1D operators L_d on the lines of z_d with their face terms,
// the reaction term and the output -- runs on the VALU in FP32, on data in LDS.
//
// MFMA operand layout (32x32x16, checked with an in-bounds probe on gfx950):
// A row r = lane % 32 holds A[r][8 (lane / 32) + j], j = 0..7; B column
// c = lane % 32 holds B[8 (lane / 32) + j][c]; the 16 accumulators of a lane
// are D[8 q + 4 (lane / 32) + i][lane % 32], q, i = 0..3.  Here the rows and
// K index the n^2 positions of a plane (k = a + n b for tangential indices
// (a, b)), the columns are planes (element slot, layer), 32 per instruction.
//
// A workgroup owns a brick of elements (the same bricks and brick order as
// the VALU kernel, so the fused <x, y> partials are counted the same way)
// plus a halo: the face neighbours outside the brick, loaded whole.  Per
// axis d: MFMA for the planes perpendicular to d of the brick and of its
// halo along d -> z_d in LDS; then one thread per line along d of an own
// element applies L_d (own line and the two neighbour lines from LDS) and
// adds the result to the element's output tile in LDS.  Finally the tile
// is written to y (and <x, y> formed when asked).
#include "dg_internal.hpp"
#include "dg_kernels.hpp"
#include "dg_lines.hpp"

namespace dg {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

__device__ __forceinline__ __bf16 as_bf16(uint16_t v) { return __builtin_bit_cast(__bf16, v); }

template <int N>
struct MfmaGeom {
  static constexpr int NN = N * N, N3 = NN * N;
  static constexpr int KCH = (NN + 15) / 16;  // K chunks of 16 (NN <= 32: one row block)
  static constexpr int ZS = 36;               // floats per plane column of z in LDS (32 rows + pad)
  // 32-bit words per element slot of x in LDS: the element's N^3 BF16 values
  // start 0 or 2 bytes into the slot (the global element block is 2-byte aligned)
  static constexpr int XW = (2 * N3 + 2 + 3) / 4;
  static_assert(NN <= 32, "one 32-row block per plane");
};

// halo elements along axis d of a BX x BY x BZ brick (both sides), and the
// offset of axis d's halo among the halo slots
template <int BX, int BY, int BZ>
__host__ __device__ constexpr int halo_n(int d) { return d == 0 ? 2 * BY * BZ : (d == 1 ? 2 * BX * BZ : 2 * BX * BY); }
template <int BX, int BY, int BZ>
__host__ __device__ constexpr int halo_off(int d) {
  return d == 0 ? 0 : (d == 1 ? halo_n<BX, BY, BZ>(0) : halo_n<BX, BY, BZ>(0) + halo_n<BX, BY, BZ>(1));
}
__device__ __forceinline__ int pick3(int d, int a0, int a1, int a2) { return d == 0 ? a0 : (d == 1 ? a1 : a2); }

// Per-block state shared by the three axis passes.
struct MfmaBrick {
  int o[3], act[3];
};

// One axis D of the apply: z_D on the MFMA units, then y (+)= L_D z_D on the
// VALU.  Every thread of the block calls it (two workgroup barriers).
template <int N, int BX, int BY, int BZ, int D, int KCH>
__device__ __forceinline__ void mfma_axis(const MeshArgs<float>& m, const Tables<float>& T, const MfmaBrick& br,
                                          const uint16_t* sX16, const int* sEl, const int* sOff, float* sZ,
                                          float* sY, const bf16x8_t (&Ahi)[KCH], const bf16x8_t (&Amid)[KCH],
                                          const bf16x8_t (&Alo)[KCH]) {
  using G = MfmaGeom<N>;
  constexpr int NN = G::NN, N3 = G::N3, ZS = G::ZS, XW = G::XW;
  constexpr int TE = BX * BY * BZ, HDD = halo_n<BX, BY, BZ>(D), HOD = halo_off<BX, BY, BZ>(D);
  constexpr int TA = D == 0 ? 1 : 0, TB = D == 2 ? 1 : 2;  // tangential axes, TA fastest
  constexpr int BA = TA == 0 ? BX : BY, BD = D == 0 ? BX : (D == 1 ? BY : BZ);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // ---------------- z_D = (M (x) M) x on the planes perpendicular to D
  {
    constexpr int ncol = (TE + HDD) * N;
    constexpr int nblk = (ncol + 31) / 32;
    const int h = lane >> 5;
    // offsets (16-bit units, relative to layer 0 of the column's element) of
    // this lane's 8 K entries per chunk; -1 past the n^2 plane positions
    int koff[KCH][8];
#pragma unroll
    for (int kc = 0; kc < KCH; ++kc)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k0 = 16 * kc + j, k1 = k0 + 8;  // the two possible K indices (lane half 0 / 1)
        const int o0 = D == 0 ? N * (k0 % N) + NN * (k0 / N) : (D == 1 ? (k0 % N) + NN * (k0 / N) : (k0 % N) + N * (k0 / N));
        const int o1 = D == 0 ? N * (k1 % N) + NN * (k1 / N) : (D == 1 ? (k1 % N) + NN * (k1 / N) : (k1 % N) + N * (k1 / N));
        const int a0 = k0 < NN ? o0 : -1, a1 = k1 < NN ? o1 : -1;
        koff[kc][j] = h ? a1 : a0;
      }
    constexpr int LSTR = D == 0 ? 1 : (D == 1 ? N : NN);  // stride of the layer index l
    for (int cb = wave; cb < nblk; cb += kBlock / 64) {  // uniform per wave
      const int col = cb * 32 + (lane & 31);
      const int cc = col < ncol ? col : 0;  // columns past the end compute on column 0
      const int zs = cc / N, l = cc - zs * N;
      const int xs = zs < TE ? zs : TE + HOD + (zs - TE);
      const int base = (xs * XW * 4 + sOff[xs]) >> 1;  // in 16-bit units
      f32x16_t acc = {};
#pragma unroll
      for (int kc = 0; kc < KCH; ++kc) {
        // plane perpendicular to D at layer l: (i2, i3) at i1 = l (D = 0),
        // (i1, i3) at i2 = l (D = 1), (i1, i2) at i3 = l (D = 2)
        bf16x8_t bv;
        const int lb = base + LSTR * l;
#pragma unroll
        for (int j = 0; j < 8; ++j) bv[j] = as_bf16(koff[kc][j] >= 0 ? sX16[lb + koff[kc][j]] : (uint16_t)0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Alo[kc], bv, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Amid[kc], bv, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ahi[kc], bv, acc, 0, 0, 0);
      }
      if (col < ncol) {
        float* zc = sZ + (zs * N + l) * ZS;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r0 = 8 * q + 4 * h;
          if (r0 < NN) *(float4*)(zc + r0) = make_float4(acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]);
        }
      }
    }
  }
  __syncthreads();
  // ---------------- y (+)= L_D z_D on the lines along D of the brick's elements
  const int oD = pick3(D, br.o[0], br.o[1], br.o[2]), actD = pick3(D, br.act[0], br.act[1], br.act[2]);
  const int NdD = pick3(D, m.nx, m.ny, m.nz);
  for (int li = tid; li < TE * NN; li += kBlock) {
    const int s = li / NN, t = li - s * NN, t1 = t % N, t2 = t / N;
    const int e = sEl[s];
    if (e < 0) continue;
    const int c0 = s % BX, c1 = (s / BX) % BY, c2 = s / (BX * BY);
    const int cD = pick3(D, c0, c1, c2), cA = pick3(TA, c0, c1, c2), cB = pick3(TB, c0, c1, c2);
    float u[N], b[N];
#pragma unroll
    for (int i = 0; i < N; ++i) u[i] = sZ[(s * N + i) * ZS + t];
    // neighbour along D on each side: an own slot when its (wrapped)
    // coordinate lies in the brick's active range, else the halo slot
    float UL = 0.f, GLr = 0.f, UH = 0.f, GHr = 0.f;
    bool hasL = false, hasH = false;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int gn = nb_coord(oD + cD, side, NdD, m.periodic);
      if (gn < 0) continue;
      int zs;
      if (gn >= oD && gn < oD + actD) {
        zs = s + (gn - oD - cD) * (D == 0 ? 1 : (D == 1 ? BX : BX * BY));
      } else {
        zs = TE + side * (HDD / 2) + cA + BA * cB;
      }
      float v[N];
#pragma unroll
      for (int i = 0; i < N; ++i) v[i] = sZ[(zs * N + i) * ZS + t];
      if (side == 0) {
        hasL = true;
        UL = v[N - 1];
        GLr = dot_end<N, float, 1>(T, v);
      } else {
        hasH = true;
        UH = v[0];
        GHr = dot_end<N, float, 0>(T, v);
      }
    }
    const float K = m.K[e];
    const float GL = m.G[6 * (int64_t)e + 2 * D], GH = m.G[6 * (int64_t)e + 2 * D + 1];
    line_op_s<N, float, false>(T, u, dot_end<N, float, 0>(T, u), dot_end<N, float, 1>(T, u), UL, GLr, UH, GHr,
                               hasL, hasH, GL, GH, K * m.vs[D], m.ih[D], m.sg[D], m.At[D], b);
    if (D == 2 && m.R) {  // reaction c |T| M (x) M (x) M x: the last mass along z
      float mu[N];
      mass_line<N, float, false>(T, u, mu);
      const float cr = m.R[e] * m.vol;
#pragma unroll
      for (int i = 0; i < N; ++i) b[i] += cr * mu[i];
    }
    float* ys = sY + s * N3;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int off = lidx<N, D>(t1, t2, i);
      if (D == 0) ys[off] = b[i];
      else ys[off] += b[i];
    }
  }
  __syncthreads();
  (void)BD;
}

template <int N, int BX, int BY, int BZ, bool DOT>
__global__ __launch_bounds__(kBlock) void k_apply_affine_mfma(MeshArgs<float> m, const uint16_t* __restrict__ x,
                                                              float* __restrict__ y, double* partials,
                                                              const int* skip) {
  using G = MfmaGeom<N>;
  constexpr int NN = G::NN, N3 = G::N3, KCH = G::KCH, ZS = G::ZS, XW = G::XW;
  constexpr int TE = BX * BY * BZ;
  constexpr int H0 = halo_n<BX, BY, BZ>(0), H1 = halo_n<BX, BY, BZ>(1), H2 = halo_n<BX, BY, BZ>(2);
  constexpr int HT = H0 + H1 + H2;
  constexpr int HMAX = H0 > H1 ? (H0 > H2 ? H0 : H2) : (H1 > H2 ? H1 : H2);
  constexpr int XS = TE + HT;       // x slots: the brick, then the halo along x, y, z
  constexpr int ZSL = TE + HMAX;    // z slots: the brick, then the halo along the current axis
  __shared__ uint32_t sX[XS * XW];
  __shared__ float sZ[ZSL * N * ZS];
  __shared__ float sY[TE * N3];
  __shared__ int sEl[XS], sOff[XS];
  __shared__ double red[kBlock / 64];
  if (skip != nullptr && *skip) return;
  // vector blockIdx.y of a multi-vector apply (the vectors follow each other)
  x += (size_t)blockIdx.y * (size_t)m.E * N3;
  y += (size_t)blockIdx.y * (size_t)m.E * N3;
  const Tables<float>& T = *m.tab;
  const int tid = threadIdx.x, lane = tid & 63;
  const int tb = (int)xcd_remap(blockIdx.x, gridDim.x);
  MfmaBrick br;
  brick_origin<BX, BY, BZ>(tb, m.nx, m.ny, m.nz, br.o);
  br.act[0] = min(BX, m.nx - br.o[0]);
  br.act[1] = min(BY, m.ny - br.o[1]);
  br.act[2] = min(BZ, m.nz - br.o[2]);

  // ---- slot -> global element (-1: none) and the byte offset of its BF16
  // block inside the 4-byte aligned window that is copied to LDS
  for (int s = tid; s < XS; s += kBlock) {
    int c0, c1, c2, e = -1;
    if (s < TE) {
      c0 = s % BX;
      c1 = (s / BX) % BY;
      c2 = s / (BX * BY);
      if (c0 < br.act[0] && c1 < br.act[1] && c2 < br.act[2])
        e = (br.o[0] + c0) + m.nx * ((br.o[1] + c1) + m.ny * (br.o[2] + c2));
    } else {
      const int hh = s - TE;
      const int d = hh < H0 ? 0 : (hh < H0 + H1 ? 1 : 2);
      const int r = hh - (d == 0 ? 0 : (d == 1 ? H0 : H0 + H1));
      const int half = (d == 0 ? H0 : (d == 1 ? H1 : H2)) / 2, side = r / half, q = r % half;
      const int ta = d == 0 ? 1 : 0, tbx = d == 2 ? 1 : 2;
      const int Ba = ta == 0 ? BX : BY;
      const int a = q % Ba, b = q / Ba;
      if (a < pick3(ta, br.act[0], br.act[1], br.act[2]) && b < pick3(tbx, br.act[0], br.act[1], br.act[2])) {
        const int od = pick3(d, br.o[0], br.o[1], br.o[2]), ad = pick3(d, br.act[0], br.act[1], br.act[2]);
        const int Ndd = pick3(d, m.nx, m.ny, m.nz);
        int g = side ? od + ad : od - 1;
        bool ok = true;
        if (g < 0 || g >= Ndd) {
          if (m.periodic) g = g < 0 ? Ndd - 1 : 0;
          else ok = false;
        }
        if (ok) {
          const int ca = pick3(ta, br.o[0], br.o[1], br.o[2]) + a, cb = pick3(tbx, br.o[0], br.o[1], br.o[2]) + b;
          int cc[3];
          cc[0] = d == 0 ? g : ca;
          cc[1] = d == 1 ? g : (d == 0 ? ca : cb);
          cc[2] = d == 2 ? g : cb;
          e = cc[0] + m.nx * (cc[1] + m.ny * cc[2]);
        }
      }
    }
    sEl[s] = e;
    sOff[s] = e >= 0 ? (int)(((uintptr_t)x + (uintptr_t)e * (2 * N3)) & 3) : 0;
  }
  __syncthreads();
  // ---- x of every slot into LDS: the 4-byte words of the aligned window
  // around the element's BF16 block (the bytes outside the block belong to
  // neighbouring elements and are not used).  Only a word that would reach
  // before the start or past the end of x itself is read as its 16-bit half
  // inside x.  All loads of a thread are issued before any is stored.
  {
    constexpr int NW = XS * XW, IT = (NW + kBlock - 1) / kBlock;
    const uintptr_t xs0 = (uintptr_t)x, xs1 = xs0 + (uintptr_t)m.E * (2 * N3);
    uint32_t v[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int w = tid + it * kBlock;
      v[it] = 0;
      if (w < NW) {
        const int sl = w / XW, i = w - sl * XW;
        const int e = sEl[sl];
        if (e >= 0) {
          const uintptr_t wb = (((uintptr_t)x + (uintptr_t)e * (2 * N3)) & ~(uintptr_t)3) + 4 * (uintptr_t)i;
          if (wb >= xs0 && wb + 4 <= xs1) v[it] = *(const uint32_t*)wb;
          else if (wb + 2 == xs0) v[it] = (uint32_t)(*(const uint16_t*)xs0) << 16;  // x starts 2 bytes into a word
          else if (wb + 2 == xs1) v[it] = (uint32_t)(*(const uint16_t*)wb);  // x ends mid-word
        }
      }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int w = tid + it * kBlock;
      if (w < NW) sX[w] = v[it];
    }
  }
  // ---- A operand: M (x) M split into BF16 hi + mid + lo, rows / K = plane positions
  bf16x8_t Ahi[KCH], Amid[KCH], Alo[KCH];
  {
    const int r = lane & 31, h = lane >> 5;
#pragma unroll
    for (int kc = 0; kc < KCH; ++kc)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = 16 * kc + 8 * h + j;
        float v = 0.0f;
        if (r < NN && k < NN) v = T.M[(r % N) * kMaxN + (k % N)] * T.M[(r / N) * kMaxN + (k / N)];
        const uint16_t hb = f32_to_bf16(v);
        const float r1 = v - bf16_to_f32(hb);
        const uint16_t mb = f32_to_bf16(r1);
        const uint16_t lb = f32_to_bf16(r1 - bf16_to_f32(mb));
        Ahi[kc][j] = as_bf16(hb);
        Amid[kc][j] = as_bf16(mb);
        Alo[kc][j] = as_bf16(lb);
      }
  }
  __syncthreads();
  const uint16_t* sX16 = (const uint16_t*)sX;
  mfma_axis<N, BX, BY, BZ, 0, KCH>(m, T, br, sX16, sEl, sOff, sZ, sY, Ahi, Amid, Alo);
  mfma_axis<N, BX, BY, BZ, 1, KCH>(m, T, br, sX16, sEl, sOff, sZ, sY, Ahi, Amid, Alo);
  mfma_axis<N, BX, BY, BZ, 2, KCH>(m, T, br, sX16, sEl, sOff, sZ, sY, Ahi, Amid, Alo);
  // ---------------- y (nontemporal: written once) and the fused <x, y>
  double part = 0.0;
  for (int w = tid; w < TE * N3; w += kBlock) {
    const int s = w / N3, i = w - s * N3;
    const int e = sEl[s];
    if (e < 0) continue;
    const float yv = sY[w];
    __builtin_nontemporal_store(yv, &y[(int64_t)e * N3 + i]);
    if (DOT) part += (double)bf16_to_f32(sX16[((s * XW * 4 + sOff[s]) >> 1) + i]) * (double)yv;
  }
  if (DOT) {
    const double mine[1] = {block_sum<kBlock>(part, red)};
    store_partials<1>(mine, partials, blockIdx.x);
  }
  (void)ZS;
}

template <int N, bool DOT>
static hipError_t run_mfma(const MeshArgs<float>& m, const uint16_t* x, float* y, double* partials, const int* skip,
                           hipStream_t s, int nrhs) {
  const int64_t nb = affine_tiles(N, m.nx, m.ny, m.nz);
  hipLaunchKernelGGL((k_apply_affine_mfma<N, tile_x(N), tile_y(N), tile_z(N), DOT>), dim3((unsigned)nb, (unsigned)nrhs),
                     dim3(kBlock), 0, s, m, x, y, partials, skip);
  return hipGetLastError();
}

bool mfma_apply_supported(int n) { return n >= 2 && n <= 5; }

hipError_t launch_apply_affine_mfma(int n, int dot, const MeshArgs<float>& m, const uint16_t* x, float* y,
                                    double* partials, const int* skip, hipStream_t s, int nrhs) {
  switch (n) {
    case 2: return dot ? run_mfma<2, true>(m, x, y, partials, skip, s, 1) : run_mfma<2, false>(m, x, y, partials, skip, s, nrhs);
    case 3: return dot ? run_mfma<3, true>(m, x, y, partials, skip, s, 1) : run_mfma<3, false>(m, x, y, partials, skip, s, nrhs);
    case 4: return dot ? run_mfma<4, true>(m, x, y, partials, skip, s, 1) : run_mfma<4, false>(m, x, y, partials, skip, s, nrhs);
    case 5: return dot ? run_mfma<5, true>(m, x, y, partials, skip, s, 1) : run_mfma<5, false>(m, x, y, partials, skip, s, nrhs);
  }
  return hipErrorInvalidValue;
}

}  // namespace dg
