// dg_vec.hip -- vector kernels of the Krylov solvers (Alg. "PCG", Sec. 2.4)
// and of the FP64 defect correction around an FP32-vector PCG.
//
// The CG scalars live in device memory (CgState); every kernel reads them
// there, so a solve needs no host round trip per iteration.  Reductions are
// deterministic: fixed thread-to-data mapping, fixed-order tree per block,
// block partials summed in block order by a single-block finish kernel.  The
// convergence norm <r, r> is computed in the same reduction as <z, r> (the
// merged check of Sec. 2.4), so an iteration has two reductions: <p, q>
// (fused into the operator application) and {<z, r>, <r, r>}.
#include "dg_internal.hpp"
#include "dg_kernels.hpp"

namespace dg {

constexpr int kVecPerThread = 4;

int64_t vec_blocks(int64_t n) {
  int64_t b = (n + (int64_t)kBlock * kVecPerThread - 1) / ((int64_t)kBlock * kVecPerThread);
  return b < 1 ? 1 : (b > kMaxVecBlocks ? kMaxVecBlocks : b);
}

template <typename TP>
__device__ __forceinline__ double p_load(const TP* p, int64_t i) { return (double)p[i]; }
template <>
__device__ __forceinline__ double p_load<uint16_t>(const uint16_t* p, int64_t i) {
  return (double)bf16_to_f32(p[i]);
}
template <typename TP>
__device__ __forceinline__ void p_store(TP* p, int64_t i, double v) { p[i] = (TP)v; }
template <>
__device__ __forceinline__ void p_store<uint16_t>(uint16_t* p, int64_t i, double v) {
  p[i] = f32_to_bf16((float)v);
}

__device__ __forceinline__ bool finite_d(double v) { return v == v && v - v == 0.0; }

// Grid-stride loop over chunks of kBlock * kVecPerThread entries; within a
// chunk consecutive threads take consecutive entries (coalesced) and each
// thread handles kVecPerThread of them (unrolled, independent loads).
#define DG_VEC_LOOP(i, k, n)                                                                          \
  for (int64_t base_ = (int64_t)blockIdx.x * kBlock * kVecPerThread; base_ < (n);                     \
       base_ += (int64_t)gridDim.x * kBlock * kVecPerThread)                                          \
    _Pragma("unroll") for (int k = 0; k < kVecPerThread; ++k)                                         \
      for (int64_t i = base_ + (int64_t)k * kBlock + threadIdx.x; i < (n); i = (n))

// r = b - q; z = Dinv r; p = z;  partials {<z,r>, <r,r>, <b,b>}
template <typename TB, typename TV, typename TP, typename TD>
__global__ __launch_bounds__(kBlock) void k_cg_init(int64_t n, const TB* __restrict__ b,
                                                    const TV* __restrict__ q, TV* __restrict__ r,
                                                    TP* __restrict__ p, const TD* __restrict__ dinv,
                                                    double* partials) {
  __shared__ double red[kBlock / 64];
  double zr = 0.0, rr = 0.0, bb = 0.0;
  DG_VEC_LOOP(i, k, n) {
    const double bi = (double)b[i];
    const TV ri = (TV)(bi - (double)q[i]);
    r[i] = ri;
    const double z = dinv ? (double)dinv[i] * (double)ri : (double)ri;
    p_store<TP>(p, i, z);
    zr += z * (double)ri;
    rr += (double)ri * (double)ri;
    bb += bi * bi;
  }
  const double mine[3] = {block_sum<kBlock>(zr, red), block_sum<kBlock>(rr, red), block_sum<kBlock>(bb, red)};
  store_partials<3>(mine, partials, blockIdx.x);
}

// inner solve: d = 0; z = Dinv r; p = z;  partials {<z,r>, <r,r>}
template <typename TV, typename TP, typename TD>
__global__ __launch_bounds__(kBlock) void k_cg_init_inner(int64_t n, const TV* __restrict__ r,
                                                          TV* __restrict__ d, TP* __restrict__ p,
                                                          const TD* __restrict__ dinv, double* partials) {
  __shared__ double red[kBlock / 64];
  double zr = 0.0, rr = 0.0;
  DG_VEC_LOOP(i, k, n) {
    const double ri = (double)r[i];
    const double z = dinv ? (double)dinv[i] * ri : ri;
    d[i] = (TV)0;
    p_store<TP>(p, i, z);
    zr += z * ri;
    rr += ri * ri;
  }
  const double mine[2] = {block_sum<kBlock>(zr, red), block_sum<kBlock>(rr, red)};
  store_partials<2>(mine, partials, blockIdx.x);
}

// lambda = rho / <p, q>;  r -= lambda q;  partials {<z,r>, <r,r>}, z = Dinv r.
// The matching x += lambda p is deferred to k_cg_pupdate, which reads p anyway.
// DINV: Jacobi preconditioner present (a template parameter rather than a
// test inside the loop, so that all loads of an entry are issued together).
template <typename TV, typename TD, bool DINV>
__device__ __forceinline__ void cg_update_body(int64_t n, TV* __restrict__ r, const TV* __restrict__ q,
                                               const TD* __restrict__ dinv, double lam, double* partials) {
  __shared__ double red[kBlock / 64];
  double zr = 0.0, rr = 0.0;
  DG_VEC_LOOP(i, k, n) {
    const double qi = (double)q[i], ro = (double)r[i], di = DINV ? (double)dinv[i] : 1.0;
    const TV ri = (TV)(ro - lam * qi);
    r[i] = ri;
    const double z = DINV ? di * (double)ri : (double)ri;
    zr += z * (double)ri;
    rr += (double)ri * (double)ri;
  }
  const double mine[2] = {block_sum<kBlock>(zr, red), block_sum<kBlock>(rr, red)};
  store_partials<2>(mine, partials, blockIdx.x);
}
// SEQ: the loads of an entry in program order with the preconditioner test
// inside the loop.  Measured faster than issuing all loads of an entry
// together for FP64 vectors that stream from HBM (187 vs 197 us at 32.8M
// entries); for FP32 vectors, and for FP64 vectors that stay in the
// last-level cache, the batched form is faster (FP32 92 vs 98 us).
template <typename TV, typename TD>
__device__ __forceinline__ void cg_update_seq(int64_t n, TV* __restrict__ r, const TV* __restrict__ q,
                                              const TD* __restrict__ dinv, double lam, double* partials) {
  __shared__ double red[kBlock / 64];
  double zr = 0.0, rr = 0.0;
  DG_VEC_LOOP(i, k, n) {
    const TV ri = (TV)((double)r[i] - lam * (double)q[i]);
    r[i] = ri;
    const double z = dinv ? (double)dinv[i] * (double)ri : (double)ri;
    zr += z * (double)ri;
    rr += (double)ri * (double)ri;
  }
  const double mine[2] = {block_sum<kBlock>(zr, red), block_sum<kBlock>(rr, red)};
  store_partials<2>(mine, partials, blockIdx.x);
}
template <typename TV, typename TD, bool SEQ>
__global__ __launch_bounds__(kBlock) void k_cg_update(int64_t n, TV* __restrict__ r, const TV* __restrict__ q,
                                                      const TD* __restrict__ dinv, int par,
                                                      const CgState* st, double* partials) {
  if (st->done) return;
  const double lam = st->rho[par] / st->pq;
  if constexpr (SEQ) {
    cg_update_seq<TV, TD>(n, r, q, dinv, lam, partials);
  } else {
    if (dinv) cg_update_body<TV, TD, true>(n, r, q, dinv, lam, partials);
    else cg_update_body<TV, TD, false>(n, r, q, dinv, lam, partials);
  }
}

// x += lambda p when this iteration's update ran (st->xpend), then, unless the
// solve has stopped, p = z + (rho[par^1] / rho[par]) p with z = Dinv r.
// force_p: only the p update, with rho[par^1] just replaced by the residual
// replacement of the defect correction (the direction is kept).  XU, PU and
// DINV select the work once per kernel, outside the loop, so that every load
// of an entry is issued before any is used.
template <typename TX, typename TV, typename TP, typename TD, bool XU, bool PU, bool DINV>
__device__ __forceinline__ void cg_pupdate_body(int64_t n, TX* __restrict__ x, const TV* __restrict__ r,
                                                TP* __restrict__ p, const TD* __restrict__ dinv, double lam,
                                                double beta) {
  DG_VEC_LOOP(i, k, n) {
    const double pi = p_load<TP>(p, i);
    const double xi = XU ? (double)x[i] : 0.0;
    const double ri = PU ? (double)r[i] : 0.0;
    const double di = PU && DINV ? (double)dinv[i] : 1.0;
    if (XU) x[i] = (TX)(xi + lam * pi);
    if (PU) p_store<TP>(p, i, (DINV ? di * ri : ri) + beta * pi);
  }
}
template <typename TX, typename TV, typename TP, typename TD, bool SEQ>
__global__ __launch_bounds__(kBlock) void k_cg_pupdate(int64_t n, TX* __restrict__ x, const TV* __restrict__ r,
                                                       TP* __restrict__ p, const TD* __restrict__ dinv,
                                                       int par, const CgState* st, int force_p) {
  const bool xu = !force_p && st->xpend;
  const bool pu = force_p ? true : !st->done;
  if (!xu && !pu) return;
  const double lam = xu ? st->rho[par] / st->pq : 0.0;
  const double beta = pu ? st->rho[par ^ 1] / st->rho[par] : 0.0;
  if constexpr (SEQ) {  // x first, then r (HBM-resident FP64: 290 vs 302 us at 32.8M entries)
    DG_VEC_LOOP(i, k, n) {
      const double pi = p_load<TP>(p, i);
      if (xu) x[i] = (TX)((double)x[i] + lam * pi);
      if (pu) {
        const double ri = (double)r[i];
        const double z = dinv ? (double)dinv[i] * ri : ri;
        p_store<TP>(p, i, z + beta * pi);
      }
    }
  } else if (xu && pu) {
    if (dinv) cg_pupdate_body<TX, TV, TP, TD, true, true, true>(n, x, r, p, dinv, lam, beta);
    else cg_pupdate_body<TX, TV, TP, TD, true, true, false>(n, x, r, p, dinv, lam, beta);
  } else if (xu) {
    cg_pupdate_body<TX, TV, TP, TD, true, false, false>(n, x, r, p, dinv, lam, beta);
  } else {
    if (dinv) cg_pupdate_body<TX, TV, TP, TD, false, true, true>(n, x, r, p, dinv, lam, beta);
    else cg_pupdate_body<TX, TV, TP, TD, false, true, false>(n, x, r, p, dinv, lam, beta);
  }
}

// FP64 PCG without the single-workgroup finish kernels, for problems whose
// block partials are few (the vectors then sit in the last-level cache and
// a finish launch is a large part of an iteration).  Every block of the
// consuming kernel sums the producer's partials itself, in the same fixed
// order, so all blocks obtain bit-identical scalars; block 0 records them in
// the state.  No block writes a state field that other blocks of the same
// kernel read.
//
// update: pq = sum of the apply's partials (partA), lambda = rho / pq; on a
// breakdown block 0 stops the solve; otherwise r -= lambda q with partials
// {<z, r>, <r, r>} into partB, and block 0 records pq and a pending x update.
template <typename TV, typename TD, bool SEQ>
__global__ __launch_bounds__(kBlock) void k_cg_update_fused(int64_t n, TV* __restrict__ r, const TV* __restrict__ q,
                                                            const TD* __restrict__ dinv, int par, CgState* st,
                                                            const double* partA, int64_t nbA, double* partB) {
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (st->done) {
    if (lead) st->xpend = 0;
    return;
  }
  double t[1];
  sum_partials<1, kBlock>(partA, nbA, t);
  const double pq = t[0], lam = st->rho[par] / pq;
  if (!(pq > 0.0) || !finite_d(lam)) {
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
  __syncthreads();  // the partial-sum scratch of sum_partials is reused below
  if constexpr (SEQ) {
    cg_update_seq<TV, TD>(n, r, q, dinv, lam, partB);
  } else {
    if (dinv) cg_update_body<TV, TD, true>(n, r, q, dinv, lam, partB);
    else cg_update_body<TV, TD, false>(n, r, q, dinv, lam, partB);
  }
}

// x/p update: when the update ran (xpend), rho' = <z, r> and <r, r> from
// partB decide convergence; x += lambda p and, unless the solve stops,
// p = z + (rho' / rho) p.  Block 0 records rho', <r, r>, the iteration count
// and the stop (xpend is cleared by the next update).
template <typename TX, typename TV, typename TP, typename TD, bool SEQ>
__global__ __launch_bounds__(kBlock) void k_cg_pupdate_fused(int64_t n, TX* __restrict__ x, const TV* __restrict__ r,
                                                             TP* __restrict__ p, const TD* __restrict__ dinv,
                                                             int par, CgState* st, const double* partB,
                                                             int64_t nbB) {
  if (!st->xpend) return;
  double t[2];
  sum_partials<2, kBlock>(partB, nbB, t);
  const double rz = t[0], rr = t[1];
  const bool bad = !finite_d(rz) || !finite_d(rr);
  const bool conv = rr <= st->tol2;
  const bool pu = !(conv || bad);
  const double lam = st->rho[par] / st->pq;
  const double beta = pu ? rz / st->rho[par] : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->rho[par ^ 1] = rz;
    st->rr = rr;
    st->iters += 1;
    if (conv) st->done = 1;
    if (bad) {
      st->breakdown = 1;
      st->done = 1;
    }
  }
  if constexpr (SEQ) {
    DG_VEC_LOOP(i, k, n) {
      const double pi = p_load<TP>(p, i);
      x[i] = (TX)((double)x[i] + lam * pi);
      if (pu) {
        const double ri = (double)r[i];
        const double z = dinv ? (double)dinv[i] * ri : ri;
        p_store<TP>(p, i, z + beta * pi);
      }
    }
  } else if (pu) {
    if (dinv) cg_pupdate_body<TX, TV, TP, TD, true, true, true>(n, x, r, p, dinv, lam, beta);
    else cg_pupdate_body<TX, TV, TP, TD, true, true, false>(n, x, r, p, dinv, lam, beta);
  } else {
    cg_pupdate_body<TX, TV, TP, TD, true, false, false>(n, x, r, p, dinv, lam, beta);
  }
}

// FP64 outer residual of the defect correction: r64 = b - q64, r32 = fp32(r64);
// partials {<r64, r64>, <b, b>}
__global__ __launch_bounds__(kBlock) void k_dc_residual(int64_t n, const double* __restrict__ b,
                                                        const double* __restrict__ q,
                                                        float* __restrict__ r32, double* partials) {
  __shared__ double red[kBlock / 64];
  double rr = 0.0, bb = 0.0;
  DG_VEC_LOOP(i, k, n) {
    const double bi = b[i];
    const double ri = bi - q[i];
    r32[i] = (float)ri;
    rr += ri * ri;
    bb += bi * bi;
  }
  const double mine[2] = {block_sum<kBlock>(rr, red), block_sum<kBlock>(bb, red)};
  store_partials<2>(mine, partials, blockIdx.x);
}

// x += d (FP64 solution update from the FP32 correction); d = 0
__global__ __launch_bounds__(kBlock) void k_dc_update(int64_t n, double* __restrict__ x, float* __restrict__ d) {
  DG_VEC_LOOP(i, k, n) {
    x[i] += (double)d[i];
    d[i] = 0.0f;
  }
}

// Residual replacement of the defect correction that keeps the inner search
// direction: r64 = b - q64, r32 = fp32(r64), z = Dinv r32;
// partials {<r64, r64>, <b, b>, <z, r32>}
__global__ __launch_bounds__(kBlock) void k_dc_replace(int64_t n, const double* __restrict__ b,
                                                       const double* __restrict__ q,
                                                       const float* __restrict__ dinv,
                                                       float* __restrict__ r32, double* partials) {
  __shared__ double red[kBlock / 64];
  double rr = 0.0, bb = 0.0, zr = 0.0;
  DG_VEC_LOOP(i, k, n) {
    const double bi = b[i];
    const double ri = bi - q[i];
    const float r32i = (float)ri;
    r32[i] = r32i;
    const double z = dinv ? (double)dinv[i] * (double)r32i : (double)r32i;
    rr += ri * ri;
    bb += bi * bi;
    zr += z * (double)r32i;
  }
  const double mine[3] = {block_sum<kBlock>(rr, red), block_sum<kBlock>(bb, red), block_sum<kBlock>(zr, red)};
  store_partials<3>(mine, partials, blockIdx.x);
}

// partials {<b - q, b - q>, <b, b>} (true residual check)
__global__ __launch_bounds__(kBlock) void k_resid_norm(int64_t n, const double* __restrict__ b,
                                                       const double* __restrict__ q, double* partials) {
  __shared__ double red[kBlock / 64];
  double rr = 0.0, bb = 0.0;
  DG_VEC_LOOP(i, k, n) {
    const double ri = b[i] - q[i];
    rr += ri * ri;
    bb += b[i] * b[i];
  }
  const double mine[2] = {block_sum<kBlock>(rr, red), block_sum<kBlock>(bb, red)};
  store_partials<2>(mine, partials, blockIdx.x);
}

// Single-reduction PCG (Chronopoulos-Gear form of the CG recurrences): with
// alpha, beta from the previous finish,
//   p = z + beta p,  s = w + beta s  (s = A p by recurrence),  x += alpha p,
//   r -= alpha s,  z = Dinv r;  partials {<r, z>, <r, r>}.
template <bool DINV>
__device__ __forceinline__ void cg2_update_body(int64_t n, double* __restrict__ x, double* __restrict__ r,
                                                double* __restrict__ z, double* __restrict__ p,
                                                double* __restrict__ s, const double* __restrict__ w,
                                                const double* __restrict__ dinv, double al, double be,
                                                double* partials) {
  __shared__ double red[kBlock / 64];
  double zr = 0.0, rr = 0.0;
  DG_VEC_LOOP(i, k, n) {
    const double zo = z[i], po = p[i], wo = w[i], so = s[i], xo = x[i], ro = r[i];
    const double di = DINV ? dinv[i] : 1.0;
    const double pi = zo + be * po;
    const double si = wo + be * so;
    p[i] = pi;
    s[i] = si;
    x[i] = xo + al * pi;
    const double ri = ro - al * si;
    r[i] = ri;
    const double zi = DINV ? di * ri : ri;
    z[i] = zi;
    zr += zi * ri;
    rr += ri * ri;
  }
  const double mine[2] = {block_sum<kBlock>(zr, red), block_sum<kBlock>(rr, red)};
  store_partials<2>(mine, partials, blockIdx.x);
}
__global__ __launch_bounds__(kBlock) void k_cg2_update(int64_t n, double* __restrict__ x, double* __restrict__ r,
                                                       double* __restrict__ z, double* __restrict__ p,
                                                       double* __restrict__ s, const double* __restrict__ w,
                                                       const double* __restrict__ dinv, const CgState* st,
                                                       double* partials) {
  if (st->done) return;
  const double al = st->alpha, be = st->beta;
  if (dinv) cg2_update_body<true>(n, x, r, z, p, s, w, dinv, al, be, partials);
  else cg2_update_body<false>(n, x, r, z, p, s, w, dinv, al, be, partials);
}

// mode 0 (after the first apply): delta = <z, w> (partB) -> alpha = gamma / delta,
// beta = 0 (gamma = rho[0] from the initial residual).  mode 1: gamma' = <r, z>,
// <r, r> (partA) and delta = <z, w> (partB): iteration count, convergence on
// <r, r>, beta = gamma' / gamma, alpha = gamma' / (delta - beta gamma' / alpha).
__global__ __launch_bounds__(1024) void k_cg2_finish(const double* partA, int64_t nbA, const double* partB,
                                                     int64_t nbB, CgState* st, int mode) {
  if (st->done) return;
  double tA[2] = {0.0, 0.0}, tB[1];
  if (mode == 1) sum_partials<2, 1024>(partA, nbA, tA);
  __syncthreads();
  sum_partials<1, 1024>(partB, nbB, tB);
  if (threadIdx.x != 0) return;
  const double delta = tB[0];
  double gam, be, den;
  if (mode == 0) {
    gam = st->rho[0];
    be = 0.0;
    den = delta;
  } else {
    gam = tA[0];
    st->rr = tA[1];
    st->iters += 1;
    be = gam / st->rho[0];
    den = delta - be * gam / st->alpha;
    if (tA[1] <= st->tol2) st->done = 1;
  }
  const double al = gam / den;
  st->rho[0] = gam;
  st->alpha = al;
  st->beta = be;
  if (!st->done && (!(den > 0.0) || !finite_d(al) || !finite_d(be))) {
    st->breakdown = 1;
    st->done = 1;
  }
}

// ---------------------------------------------------------------- finish kernels
// mode: what the totals mean and which state fields they set
enum FinishMode {
  FIN_DOT = 0,       // 1 value: pq
  FIN_INIT = 1,      // 3 values: rho[0], rr (= rr0), bb; tol2 = rtol^2 bb
  FIN_INIT_INNER = 2,// 2 values: rho[0], rr (= rr0 = bb); tol2 = rtol^2 rr
  FIN_UPDATE = 3,    // 2 values: rho[par^1], rr; iters++; done when rr <= tol2
  FIN_DC = 4,        // 2 values: rr, bb
  FIN_TRUE = 5,      // 2 values: true_rr, true_bb
  FIN_REPLACE = 6,   // 3 values: true_rr (= rr), true_bb, rho[par^1]; restarts the inner stop test
  FIN_BJ = 7         // 2 values: rho[par] = <z, r> of the block-Jacobi z (skipped once stopped)
};

constexpr int kFinishBlock = 1024;

template <int NV, int MODE>
__global__ __launch_bounds__(kFinishBlock) void k_finish(const double* partials, int64_t nblocks, CgState* st,
                                                         int par, double rtol, double aux) {
  if (MODE == FIN_DOT) {
    // a new iteration starts: the deferred x update of the last one has been applied
    if (threadIdx.x == 0) st->xpend = 0;
  }
  if (MODE == FIN_DOT || MODE == FIN_UPDATE || MODE == FIN_BJ) {
    if (st->done) return;
  }
  double t[NV];
  sum_partials<NV, kFinishBlock>(partials, nblocks, t);
  if (threadIdx.x != 0) return;
  if (MODE == FIN_DOT) {
    st->pq = t[0];
    const double lam = st->rho[par] / t[0];
    if (!(t[0] > 0.0) || !finite_d(lam)) {
      st->breakdown = 1;
      st->done = 1;
    }
  } else if (MODE == FIN_INIT || MODE == FIN_INIT_INNER) {
    st->rho[0] = t[0];
    st->rr = t[1];
    st->rr0 = t[1];
    st->bb = MODE == FIN_INIT ? t[2] : t[1];
    st->tol2 = rtol * rtol * st->bb;
    st->iters = 0;
    st->breakdown = 0;
    st->xpend = 0;
    st->done = (t[1] <= st->tol2) ? 1 : 0;
    if (!finite_d(t[0]) || !finite_d(t[1])) {
      st->breakdown = 1;
      st->done = 1;
    }
  } else if (MODE == FIN_UPDATE) {
    st->rho[par ^ 1] = t[0];
    st->rr = t[1];
    st->iters += 1;
    st->xpend = 1;
    if (t[1] <= st->tol2) st->done = 1;
    if (!finite_d(t[0]) || !finite_d(t[1])) {
      st->breakdown = 1;
      st->done = 1;
    }
  } else if (MODE == FIN_BJ) {
    st->rho[par] = t[0];
    if (!finite_d(t[0]) || !(t[0] > 0.0)) {
      st->breakdown = 1;
      st->done = 1;
    }
  } else if (MODE == FIN_DC) {
    st->rr = t[0];
    st->bb = t[1];
  } else if (MODE == FIN_TRUE) {
    st->true_rr = t[0];
    st->true_bb = t[1];
  } else {
    // rtol: outer tolerance; aux: reduction asked of the next inner segment.
    // The segment stops at aux * ||r|| or at half the outer target, whichever is larger.
    st->true_rr = t[0];
    st->true_bb = t[1];
    st->rr = t[0];
    st->rr0 = t[0];
    st->rho[par ^ 1] = t[2];
    const double a = aux * aux * t[0], o = 0.25 * rtol * rtol * t[1];
    st->tol2 = a > o ? a : o;
    st->iters = 0;
    st->xpend = 0;
    st->breakdown = 0;
    st->done = 0;
    if (!finite_d(t[0]) || !finite_d(t[2]) || !(t[2] > 0.0)) {
      st->breakdown = 1;
      st->done = 1;
    }
  }
}

template <int NV, int MODE>
static hipError_t finish(const double* partials, int64_t nb, CgState* st, int par, double rtol, hipStream_t s,
                         double aux = 0.0) {
  hipLaunchKernelGGL((k_finish<NV, MODE>), dim3(1), dim3(kFinishBlock), 0, s, partials, nb, st, par, rtol, aux);
  return hipGetLastError();
}

hipError_t launch_finish_dot(const double* partials, int64_t nblocks, CgState* st, int par, hipStream_t s) {
  return finish<1, FIN_DOT>(partials, nblocks, st, par, 0.0, s);
}
hipError_t launch_update_finish(const double* partials, int64_t nb, CgState* st, int par, hipStream_t s) {
  return finish<2, FIN_UPDATE>(partials, nb, st, par, 0.0, s);
}
hipError_t launch_bj_finish(const double* partials, int64_t nblocks, CgState* st, int idx, hipStream_t s) {
  return finish<2, FIN_BJ>(partials, nblocks, st, idx, 0.0, s);
}

// ---------------------------------------------------------------- launchers
#define DG_TRY(expr)                     \
  do {                                   \
    hipError_t e_ = (expr);              \
    if (e_ != hipSuccess) return e_;     \
  } while (0)

template <typename TB, typename TV, typename TP, typename TD>
hipError_t launch_cg_init(int64_t n, const TB* b, const TV* q, TV* r, TP* p, const TD* dinv, double rtol,
                          CgState* st, double* partials, hipStream_t s) {
  const int64_t nb = vec_blocks(n);
  hipLaunchKernelGGL((k_cg_init<TB, TV, TP, TD>), dim3((unsigned)nb), dim3(kBlock), 0, s, n, b, q, r, p, dinv,
                     partials);
  DG_TRY(hipGetLastError());
  return finish<3, FIN_INIT>(partials, nb, st, 0, rtol, s);
}
template <typename TV, typename TP, typename TD>
hipError_t launch_cg_init_inner(int64_t n, const TV* r, TV* d, TP* p, const TD* dinv, double rtol,
                                CgState* st, double* partials, hipStream_t s) {
  const int64_t nb = vec_blocks(n);
  hipLaunchKernelGGL((k_cg_init_inner<TV, TP, TD>), dim3((unsigned)nb), dim3(kBlock), 0, s, n, r, d, p, dinv,
                     partials);
  DG_TRY(hipGetLastError());
  return finish<2, FIN_INIT_INNER>(partials, nb, st, 0, rtol, s);
}
// the in-order loop form of the CG update kernels for vectors of 8-byte
// entries above 24 MB (streamed from HBM rather than held in the 256 MB
// last-level cache with the other CG vectors)
template <typename TV>
static bool seq_form(int64_t n) {
  return sizeof(TV) >= 8 && (double)n * sizeof(TV) > 24e6;
}

template <typename TV, typename TD>
hipError_t launch_cg_update(int64_t n, TV* r, const TV* q, const TD* dinv, int par, CgState* st,
                            double* partials, hipStream_t s) {
  const int64_t nb = vec_blocks(n);
  if (seq_form<TV>(n))
    hipLaunchKernelGGL((k_cg_update<TV, TD, true>), dim3((unsigned)nb), dim3(kBlock), 0, s, n, r, q, dinv, par,
                       st, partials);
  else
    hipLaunchKernelGGL((k_cg_update<TV, TD, false>), dim3((unsigned)nb), dim3(kBlock), 0, s, n, r, q, dinv, par,
                       st, partials);
  DG_TRY(hipGetLastError());
  return finish<2, FIN_UPDATE>(partials, nb, st, par, 0.0, s);
}
template <typename TX, typename TV, typename TP, typename TD>
hipError_t launch_cg_pupdate(int64_t n, TX* x, const TV* r, TP* p, const TD* dinv, int par, const CgState* st,
                             int force_p, hipStream_t s) {
  if (seq_form<TV>(n))
    hipLaunchKernelGGL((k_cg_pupdate<TX, TV, TP, TD, true>), dim3((unsigned)vec_blocks(n)), dim3(kBlock), 0, s, n,
                       x, r, p, dinv, par, st, force_p);
  else
    hipLaunchKernelGGL((k_cg_pupdate<TX, TV, TP, TD, false>), dim3((unsigned)vec_blocks(n)), dim3(kBlock), 0, s, n,
                       x, r, p, dinv, par, st, force_p);
  return hipGetLastError();
}

template <typename TV, typename TD>
hipError_t launch_cg_update_fused(int64_t n, TV* r, const TV* q, const TD* dinv, int par, CgState* st,
                                  const double* partA, int64_t nbA, double* partB, hipStream_t s) {
  const int64_t nb = vec_blocks(n);
  if (seq_form<TV>(n))
    hipLaunchKernelGGL((k_cg_update_fused<TV, TD, true>), dim3((unsigned)nb), dim3(kBlock), 0, s, n, r, q, dinv,
                       par, st, partA, nbA, partB);
  else
    hipLaunchKernelGGL((k_cg_update_fused<TV, TD, false>), dim3((unsigned)nb), dim3(kBlock), 0, s, n, r, q, dinv,
                       par, st, partA, nbA, partB);
  return hipGetLastError();
}
template <typename TX, typename TV, typename TP, typename TD>
hipError_t launch_cg_pupdate_fused(int64_t n, TX* x, const TV* r, TP* p, const TD* dinv, int par, CgState* st,
                                   const double* partB, hipStream_t s, int64_t nbB) {
  const int64_t nb = vec_blocks(n);
  if (nbB < 0) nbB = nb;
  if (seq_form<TV>(n))
    hipLaunchKernelGGL((k_cg_pupdate_fused<TX, TV, TP, TD, true>), dim3((unsigned)nb), dim3(kBlock), 0, s, n, x, r,
                       p, dinv, par, st, partB, nbB);
  else
    hipLaunchKernelGGL((k_cg_pupdate_fused<TX, TV, TP, TD, false>), dim3((unsigned)nb), dim3(kBlock), 0, s, n, x,
                       r, p, dinv, par, st, partB, nbB);
  return hipGetLastError();
}
template hipError_t launch_cg_update_fused<double, double>(int64_t, double*, const double*, const double*, int,
                                                           CgState*, const double*, int64_t, double*, hipStream_t);
template hipError_t launch_cg_update_fused<float, float>(int64_t, float*, const float*, const float*, int, CgState*,
                                                         const double*, int64_t, double*, hipStream_t);
template hipError_t launch_cg_pupdate_fused<double, double, double, double>(int64_t, double*, const double*, double*,
                                                                            const double*, int, CgState*,
                                                                            const double*, hipStream_t, int64_t);
template hipError_t launch_cg_pupdate_fused<float, float, float, float>(int64_t, float*, const float*, float*,
                                                                       const float*, int, CgState*, const double*,
                                                                       hipStream_t, int64_t);
template hipError_t launch_cg_pupdate_fused<float, float, uint16_t, float>(int64_t, float*, const float*, uint16_t*,
                                                                          const float*, int, CgState*,
                                                                          const double*, hipStream_t, int64_t);

// explicit instantiations used by the host solvers
template hipError_t launch_cg_init<double, double, double, double>(int64_t, const double*, const double*,
                                                                   double*, double*, const double*, double,
                                                                   CgState*, double*, hipStream_t);
template hipError_t launch_cg_update<double, double>(int64_t, double*, const double*, const double*, int,
                                                     CgState*, double*, hipStream_t);
template hipError_t launch_cg_pupdate<double, double, double, double>(int64_t, double*, const double*, double*,
                                                                      const double*, int, const CgState*, int,
                                                                      hipStream_t);
template hipError_t launch_cg_init_inner<float, float, float>(int64_t, const float*, float*, float*,
                                                              const float*, double, CgState*, double*,
                                                              hipStream_t);
template hipError_t launch_cg_init_inner<float, uint16_t, float>(int64_t, const float*, float*, uint16_t*,
                                                                 const float*, double, CgState*, double*,
                                                                 hipStream_t);
template hipError_t launch_cg_update<float, float>(int64_t, float*, const float*, const float*, int, CgState*,
                                                   double*, hipStream_t);
template hipError_t launch_cg_pupdate<float, float, float, float>(int64_t, float*, const float*, float*,
                                                                  const float*, int, const CgState*, int,
                                                                  hipStream_t);
template hipError_t launch_cg_pupdate<float, float, uint16_t, float>(int64_t, float*, const float*, uint16_t*,
                                                                     const float*, int, const CgState*, int,
                                                                     hipStream_t);

hipError_t launch_dc_residual(int64_t n, const double* b, const double* q, float* r32, CgState* st,
                              double* partials, hipStream_t s) {
  const int64_t nb = vec_blocks(n);
  hipLaunchKernelGGL(k_dc_residual, dim3((unsigned)nb), dim3(kBlock), 0, s, n, b, q, r32, partials);
  DG_TRY(hipGetLastError());
  return finish<2, FIN_DC>(partials, nb, st, 0, 0.0, s);
}
hipError_t launch_dc_update(int64_t n, double* x, float* d, hipStream_t s) {
  hipLaunchKernelGGL(k_dc_update, dim3((unsigned)vec_blocks(n)), dim3(kBlock), 0, s, n, x, d);
  return hipGetLastError();
}
hipError_t launch_dc_replace(int64_t n, const double* b, const double* q, const float* dinv, float* r32,
                             CgState* st, int par, double rtol, double reduction, double* partials,
                             hipStream_t s) {
  const int64_t nb = vec_blocks(n);
  hipLaunchKernelGGL(k_dc_replace, dim3((unsigned)nb), dim3(kBlock), 0, s, n, b, q, dinv, r32, partials);
  DG_TRY(hipGetLastError());
  return finish<3, FIN_REPLACE>(partials, nb, st, par, rtol, s, reduction);
}
hipError_t launch_cg2_update(int64_t n, double* x, double* r, double* z, double* p, double* s, const double* w,
                             const double* dinv, const CgState* st, double* partials, hipStream_t st_) {
  hipLaunchKernelGGL(k_cg2_update, dim3((unsigned)vec_blocks(n)), dim3(kBlock), 0, st_, n, x, r, z, p, s, w, dinv, st,
                     partials);
  return hipGetLastError();
}
hipError_t launch_cg2_finish(const double* partA, int64_t nbA, const double* partB, int64_t nbB, CgState* st,
                             int mode, hipStream_t s) {
  hipLaunchKernelGGL(k_cg2_finish, dim3(1), dim3(1024), 0, s, partA, nbA, partB, nbB, st, mode);
  return hipGetLastError();
}
hipError_t launch_resid_norm(int64_t n, const double* b, const double* q, CgState* st, double* partials,
                             hipStream_t s) {
  const int64_t nb = vec_blocks(n);
  hipLaunchKernelGGL(k_resid_norm, dim3((unsigned)nb), dim3(kBlock), 0, s, n, b, q, partials);
  DG_TRY(hipGetLastError());
  return finish<2, FIN_TRUE>(partials, nb, st, 0, 0.0, s);
}

// inner solve with a stored preconditioned residual: p = z, d = 0
template <typename TP>
__global__ __launch_bounds__(kBlock) void k_inner_start(int64_t n, const float* __restrict__ z, float* __restrict__ d,
                                                        TP* __restrict__ p, const CgState* st) {
  if (st->done) return;
  DG_VEC_LOOP(i, k, n) {
    p_store<TP>(p, i, (double)z[i]);
    d[i] = 0.0f;
  }
}
template <typename TP>
hipError_t launch_inner_start(int64_t n, const float* z, float* d, TP* p, const CgState* st, hipStream_t s) {
  hipLaunchKernelGGL((k_inner_start<TP>), dim3((unsigned)vec_blocks(n)), dim3(kBlock), 0, s, n, z, d, p, st);
  return hipGetLastError();
}
template hipError_t launch_inner_start<float>(int64_t, const float*, float*, float*, const CgState*, hipStream_t);
template hipError_t launch_inner_start<uint16_t>(int64_t, const float*, float*, uint16_t*, const CgState*,
                                                 hipStream_t);
// {<z, r>, <r, r>} partials of the block preconditioner as the start of an
// inner solve: rho[0], rr = rr0 = bb, tol2 = rtol^2 rr (FIN_INIT_INNER)
hipError_t launch_init_inner_finish(const double* partials, int64_t nb, CgState* st, double rtol, hipStream_t s) {
  return finish<2, FIN_INIT_INNER>(partials, nb, st, 0, rtol, s);
}

// ---------------------------------------------------------------- elementwise helpers
// K = exp(theta).  changed != nullptr: set *changed = 1 when any coefficient
// differs bitwise from the one it replaces (every writer stores the same value).
__global__ void k_exp(int64_t n, const double* __restrict__ th, double* __restrict__ K64,
                      float* __restrict__ K32, int* changed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double k = th ? exp(th[i]) : 1.0;
  if (changed != nullptr && __double_as_longlong(K64[i]) != __double_as_longlong(k)) *changed = 1;
  K64[i] = k;
  K32[i] = (float)k;
}
__global__ void k_set_flag(int* f, int v) {
  if (threadIdx.x == 0) *f = v;
}
// run != nullptr && *run == 0: nothing to do (the diagonal is unchanged)
__global__ void k_inv_diag(int64_t n, const double* __restrict__ d, double* __restrict__ i64,
                           float* __restrict__ i32, const int* run) {
  if (run != nullptr && *run == 0) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = 1.0 / d[i];
  i64[i] = v;
  i32[i] = (float)v;
}
__global__ void k_to_f32(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

hipError_t launch_exp(int64_t n, const double* th, double* K64, float* K32, int* changed, hipStream_t s) {
  if (changed != nullptr) {
    hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(64), 0, s, changed, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_exp, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, th, K64, K32, changed);
  return hipGetLastError();
}
hipError_t launch_inv_diag(int64_t n, const double* d, double* i64, float* i32, const int* run, hipStream_t s) {
  hipLaunchKernelGGL(k_inv_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, d, i64, i32, run);
  return hipGetLastError();
}
hipError_t launch_to_f32(int64_t n, const double* a, float* b, hipStream_t s) {
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, a, b);
  return hipGetLastError();
}

}  // namespace dg
