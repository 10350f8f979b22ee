// dg_faces.hpp -- the face-aware line phase shared by the affine applies:
// neighbour face scalars of a line (from the brick's LDS exchange area or
// from HBM) and the 1D DG operator on the thread's line.
#pragma once

#include "dg_internal.hpp"
#include "dg_lines.hpp"

namespace dg {

// Neighbour face scalars along axis D for both sides.  In-brick neighbours
// publish their own face scalars in F (written by their threads in this
// phase), out-of-brick neighbours come from HBM, Dirichlet sides are absent.
template <int N, int D, int BX, int BY, int BZ, typename TC, typename TIN, bool OFF32 = false>
struct AxisNeighbours {
  bool inL, inH, glL, glH, hasL, hasH;
  int fL, fH;  // exchange-slot offsets of in-brick neighbours from the own slot
  uint32_t eoL, eoH;  // first entries of the neighbour elements
  TC gL[N], gH[N];
  // eo: the element's first entry (element index times n^3, below 2^31);
  // FS: element stride of the exchange slots
  template <int FS>
  __device__ __forceinline__ void locate(int nx, int ny, uint32_t eo, const int (&c)[3], const int (&o)[3],
                                         const int (&Nd)[3], int periodic, bool slot = true) {
    constexpr int Bd = D == 0 ? BX : (D == 1 ? BY : BZ);
    constexpr int sD = D == 0 ? 1 : (D == 1 ? BX : BX * BY);
    const int cl = nb_coord(c[D], 0, Nd[D], periodic), ch = nb_coord(c[D], 1, Nd[D], periodic);
    hasL = slot && cl >= 0;
    hasH = slot && ch >= 0;
    const int ll = cl - o[D], lh = ch - o[D];
    inL = hasL && ll >= 0 && ll < Bd;
    inH = hasH && lh >= 0 && lh < Bd;
    glL = hasL && !inL;
    glH = hasH && !inH;
    // an in-brick neighbour is the next slot along D, or across the brick
    // when the brick spans the periodic axis (uniform choices, no multiply)
    fL = c[D] > 0 ? -sD * FS : (Nd[D] - 1) * sD * FS;
    fH = c[D] < Nd[D] - 1 ? sD * FS : -(Nd[D] - 1) * sD * FS;
    // the neighbours' first entries as uniform offsets from the element's: one
    // element stride along D, or the periodic wrap across the mesh (no
    // per-lane multiply; unused on a side without neighbour)
    constexpr uint32_t N3 = N * N * N;
    const uint32_t sd = D == 0 ? N3 : (D == 1 ? (uint32_t)nx * N3 : (uint32_t)nx * (uint32_t)ny * N3);
    const uint32_t wrap = (uint32_t)(Nd[D] - 1) * sd;
    eoL = c[D] > 0 ? eo - sd : eo + wrap;
    eoH = c[D] < Nd[D] - 1 ? eo + sd : eo - wrap;
  }
  // issue the HBM loads (before the own work of the phase, to hide latency)
  __device__ __forceinline__ void fetch(const TIN* __restrict__ x, int t1, int t2) {
    if (glL) glb_get_at<N, D, TC, TIN, OFF32>(x, eoL, t1, t2, gL);
    if (glH) glb_get_at<N, D, TC, TIN, OFF32>(x, eoH, t1, t2, gH);
  }
  // the HBM neighbour lines reduced to their face scalars (frees the lines)
  TC uL, dL, uH, dH;
  __device__ __forceinline__ void reduce(const Tables<TC>& T) {
    uL = dL = uH = dH = TC(0);
    if (glL) {
      uL = gL[N - 1];
      dL = dot_end<N, TC, 1>(T, gL);
    }
    if (glH) {
      uH = gH[0];
      dH = dot_end<N, TC, 0>(T, gH);
    }
  }
  // neighbour scalars: low side -> its upper-face (U, d1.u), high side -> its lower-face (U, d0.u);
  // Fe: the own element's exchange slot
  __device__ __forceinline__ void scalars(const TC* Fe, int t, TC& UL, TC& GLr, TC& UH, TC& GHr) const {
    constexpr int NN = N * N;
    UL = uL;
    GLr = dL;
    UH = uH;
    GHr = dH;
    if (inL) {
      UL = Fe[fL + 2 * NN + t];
      GLr = Fe[fL + 3 * NN + t];
    }
    if (inH) {
      UH = Fe[fH + 0 * NN + t];
      GHr = Fe[fH + 1 * NN + t];
    }
  }
};

// Barrier over the threads that exchange data through LDS at one point of
// the apply.  WAVE: every thread whose LDS writes the readers depend on lies
// in the reader's wavefront (the lanes of a wavefront execute together and
// its LDS operations complete in order), so only the compiler has to be kept
// from moving LDS accesses across it; otherwise the workgroup barrier.
template <bool WAVE>
__device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// One face-aware direction of the affine apply: b = L_D u on this thread's
// line along axis D (own line from HBM, neighbour face scalars from the
// brick's exchange area or from HBM; Fe: the element's own slot in that
// area).  Contains one barrier; every thread of the block calls it.
// act == false: the lane's element overhangs the mesh (it computes on a
// clamped element, sees no neighbours, and its result is discarded).
template <int N, int D, int BX, int BY, int BZ, int FS, typename TC, typename TIN, bool TRANS, bool OFF32>
__device__ __forceinline__ void face_phase(const MeshArgs<TC>& m, const Tables<TC>& T, const TIN* __restrict__ x,
                                           bool act, uint32_t eo, const int (&c)[3], const int (&o)[3],
                                           const int (&Nd)[3], int t, int t1, int t2, TC* Fe, TC K, TC GL,
                                           TC GH, TC cr, TC (&b)[N], TC* own = nullptr, TC* nbt = nullptr) {
  constexpr int NN = N * N;
  AxisNeighbours<N, D, BX, BY, BZ, TC, TIN, OFF32> nb;
  TC u[N], g0, g1;
  {
    nb.template locate<FS>(m.nx, m.ny, eo, c, o, Nd, m.periodic, act);
    nb.fetch(x, t1, t2);
    glb_get_at<N, D, TC, TIN, OFF32>(x, eo, t1, t2, u);
    nb.reduce(T);
    g0 = dot_end<N, TC, 0>(T, u);
    g1 = dot_end<N, TC, 1>(T, u);
    Fe[0 * NN + t] = u[0];
    Fe[1 * NN + t] = g0;
    Fe[2 * NN + t] = u[N - 1];
    Fe[3 * NN + t] = g1;
  }
  // x-neighbours inside the brick share the wavefront when a brick row does
  lds_sync<D == 0 && 64 % (BX * NN) == 0>();
  {
    TC UL, GLr, UH, GHr;
    nb.scalars(Fe, t, UL, GLr, UH, GHr);
    line_op_s<N, TC, TRANS>(T, u, g0, g1, UL, GLr, UH, GHr, nb.hasL, nb.hasH, GL, GH, K * m.vs[D], m.ih[D],
                            m.sg[D], m.At[D], b);
    if (own != nullptr) {  // the caller keeps the line (x along D at (t1, t2))
#pragma unroll
      for (int i = 0; i < N; ++i) own[i] = u[i];
    }
    if (nbt != nullptr) {  // the caller keeps the neighbours' traces at the shared ends
      nbt[0] = UL;
      nbt[1] = UH;
    }
    if (cr != TC(0)) {  // reaction c |T| M u along this line (the other two masses follow)
      TC mu[N];
      mass_line<N, TC, false>(T, u, mu);
#pragma unroll
      for (int i = 0; i < N; ++i) b[i] += cr * mu[i];
    }
  }
}

}  // namespace dg
