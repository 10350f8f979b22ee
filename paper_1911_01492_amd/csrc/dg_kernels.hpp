// dg_kernels.hpp -- host-side launchers of the libdg kernels.
#pragma once

#include "dg_internal.hpp"

namespace dg {

// Scalars of one running CG solve, kept in device memory.
struct CgState {
  double rho[2];    // <z, r> of the current and of the next iteration (by parity)
  double pq;        // <p, A p>
  double rr;        // <r, r>
  double rr0;       // <r0, r0>
  double bb;        // <b, b>
  double tol2;      // squared absolute tolerance on <r, r>
  double true_rr;   // ||b - A x||^2 of the last true-residual check
  double true_bb;   // ||b||^2
  int done;         // 1 once converged or broken down: later kernels of the loop return at once
  int breakdown;    // 1 on a non-positive / non-finite CG scalar
  int iters;        // iterations completed
  int xpend;        // 1 after an update: the deferred x += lambda p of that iteration is due
  unsigned counter; // arrival counter of the grid reductions (reset by the last block)
  unsigned pad1;
  double alpha;     // single-reduction CG: step length and direction coefficient of the next update
  double beta;
};

constexpr int kMaxVecBlocks = 2048;

// grid size of the per-element kernels (one block per elems_per_block(n)
// elements), of the brick-tiled affine apply, and of the vector kernels
int64_t element_blocks(int n, int64_t E);
int64_t affine_tiles(int n, int nx, int ny, int nz);
int64_t vec_blocks(int64_t n);

// y = A x (trans: A^T x) on affine meshes; prec: 0 f64, 1 f32, 2 bf16 in / f32 out.
// dot != 0: <x, y> -> st->pq (block partials, then a single-block finish kernel;
// sets st->breakdown / st->done when <p, A p> is not positive, par selects rho).
// skip: device flag; when nonzero the kernels do nothing.
hipError_t launch_apply_affine(int n, int prec, int trans, int dot, const MeshArgs<double>& m64,
                               const MeshArgs<float>& m32, const void* x, void* y, double* partials,
                               CgState* st, int par, const int* skip, hipStream_t s);
// BF16-input affine apply with the tangential masses on MFMA (n = 2..5):
// partials only (one per brick, as launch_apply_affine); the caller finishes.
bool mfma_apply_supported(int n);
hipError_t launch_apply_affine_mfma(int n, int dot, const MeshArgs<float>& m, const uint16_t* x, float* y,
                                    double* partials, const int* skip, hipStream_t s, int nrhs = 1);
// Y = A X for nrhs vectors stored one after another (affine meshes, no fused
// dot): the vectors are the second grid dimension of the apply kernels
hipError_t launch_apply_affine_multi(int n, int prec, int trans, int nrhs, const MeshArgs<double>& m64,
                                     const MeshArgs<float>& m32, const void* x, void* y, hipStream_t s);
// element block-Jacobi (axis-parallel affine meshes): per element and axis the
// fast-diagonalisation factors Q_d (n x n) and l_d (n), FP64 and FP32 copies;
// z = P r with the block partials {<z, r>, <r, r>} (element_blocks(n, E) of them);
// q != nullptr: first r -= (rho[par] / pq) q from st (r rewritten), the CG update
hipError_t launch_bj_setup(int n, const MeshArgs<double>& m, double* Q, double* lam, float* Q32, float* lam32,
                           hipStream_t s);
// partA != nullptr (with q): the CG update sums the apply's nbA partials of
// <p, q> itself (every block, in the same order) instead of reading st->pq
// from a finish kernel, records pq and the pending x update in st, and stops
// the solve on a breakdown (the counterpart of launch_cg_update_fused)
template <typename TV, typename TQ>
hipError_t launch_bj_apply(int n, int64_t E, const TQ* Q, const TQ* lam, TV* r, TV* z, double* partials,
                           const int* skip, hipStream_t s, const TV* q = nullptr, CgState* st = nullptr,
                           int par = 0, const double* partA = nullptr, int64_t nbA = 0);
// FIN_UPDATE on {<z, r>, <r, r>} partials (rho[par^1], rr, iteration count, convergence)
hipError_t launch_update_finish(const double* partials, int64_t nb, CgState* st, int par, hipStream_t s);
// st->rho[idx] = <z, r> from the block-Jacobi partials (nothing once the solve stopped)
hipError_t launch_bj_finish(const double* partials, int64_t nblocks, CgState* st, int idx, hipStream_t s);
// inner solve started from a stored preconditioned residual z: p = z, d = 0
// (skipped when st->done), and the finish that turns the block preconditioner's
// {<z, r>, <r, r>} partials into the start state of the inner solve
template <typename TP>
hipError_t launch_inner_start(int64_t n, const float* z, float* d, TP* p, const CgState* st, hipStream_t s);
hipError_t launch_init_inner_finish(const double* partials, int64_t nb, CgState* st, double rtol, hipStream_t s);
hipError_t launch_face_coef(const MeshArgs<double>& m, double* G64, float* G32, hipStream_t s);
hipError_t launch_finish_dot(const double* partials, int64_t nblocks, CgState* st, int par, hipStream_t s);
// diagonal kernels: run != nullptr && *run == 0 makes them return at once
hipError_t launch_diag_affine(int n, const MeshArgs<double>& m, double* d, const int* run, hipStream_t s);
hipError_t launch_dA_affine(int n, const MeshArgs<double>& m, const double* u, const double* v, double* g,
                            hipStream_t s);

// trilinear meshes
hipError_t launch_apply_trilinear(int n, int prec, int trans, int dot, const MeshArgs<double>& m64,
                                  const MeshArgs<float>& m32, const void* x, void* y, double* partials,
                                  CgState* st, int par, const int* skip, hipStream_t s);
// meshes of equal parallelepipeds (constant metric; m64 / m32 carry the
// metric scalars): y = A x, the form being symmetric also A^T x
hipError_t launch_apply_ppd(int n, int prec, int dot, const MeshArgs<double>& m64, const MeshArgs<float>& m32,
                            const void* x, void* y, double* partials, CgState* st, int par, const int* skip,
                            hipStream_t s);
// Y = A X for nrhs vectors stored one after another (the vector index is the
// second grid dimension; no fused dot)
hipError_t launch_apply_ppd_multi(int n, int prec, int nrhs, const MeshArgs<double>& m64, const MeshArgs<float>& m32,
                                  const void* x, void* y, hipStream_t s);
hipError_t launch_diag_trilinear(int n, const MeshArgs<double>& m, double* d, const int* run, hipStream_t s);
// g_T = u^T dA/dtheta_T v on trilinear meshes; parts: 7 E doubles of scratch
hipError_t launch_dA_trilinear(int n, const MeshArgs<double>& m, const double* u, const double* v, double* parts,
                               double* g, hipStream_t s);

// geometry / load vector (any mesh)
hipError_t launch_quad_points(int n, const MeshArgs<double>& m, double* xq, hipStream_t s);
hipError_t launch_load_vector(int n, const MeshArgs<double>& m, const double* fq, double* b,
                              hipStream_t s);

// Krylov vector kernels
template <typename TB, typename TV, typename TP, typename TD>
hipError_t launch_cg_init(int64_t n, const TB* b, const TV* q, TV* r, TP* p, const TD* dinv, double rtol,
                          CgState* st, double* partials, hipStream_t s);
template <typename TV, typename TP, typename TD>
hipError_t launch_cg_init_inner(int64_t n, const TV* r, TV* d, TP* p, const TD* dinv, double rtol,
                                CgState* st, double* partials, hipStream_t s);
template <typename TV, typename TD>
hipError_t launch_cg_update(int64_t n, TV* r, const TV* q, const TD* dinv, int par, CgState* st,
                            double* partials, hipStream_t s);
template <typename TX, typename TV, typename TP, typename TD>
hipError_t launch_cg_pupdate(int64_t n, TX* x, const TV* r, TP* p, const TD* dinv, int par, const CgState* st,
                             int force_p, hipStream_t s);
hipError_t launch_dc_residual(int64_t n, const double* b, const double* q, float* r32, CgState* st,
                              double* partials, hipStream_t s);
hipError_t launch_dc_update(int64_t n, double* x, float* d, hipStream_t s);
// single-reduction (Chronopoulos-Gear) PCG in FP64: fused update of p, s, x, r, z
// with the partials {<r, z>, <r, r>}, and the finish over these and the <z, w>
// partials of the apply (mode 0: after the first apply, 1: every iteration)
hipError_t launch_cg2_update(int64_t n, double* x, double* r, double* z, double* p, double* s, const double* w,
                             const double* dinv, const CgState* st, double* partials, hipStream_t st_);
// PCG update kernels that sum the producer's block partials themselves
// (no finish kernels): partA = the apply's <p, q> partials (nbA of them),
// partB = the update's {<z, r>, <r, r>} partials (disjoint from partA)
template <typename TV, typename TD>
hipError_t launch_cg_update_fused(int64_t n, TV* r, const TV* q, const TD* dinv, int par, CgState* st,
                                  const double* partA, int64_t nbA, double* partB, hipStream_t s);
// nbB: number of {<z, r>, <r, r>} partial pairs in partB (< 0: those of
// launch_cg_update_fused, one per vector block)
template <typename TX, typename TV, typename TP, typename TD>
hipError_t launch_cg_pupdate_fused(int64_t n, TX* x, const TV* r, TP* p, const TD* dinv, int par, CgState* st,
                                   const double* partB, hipStream_t s, int64_t nbB = -1);
hipError_t launch_cg2_finish(const double* partA, int64_t nbA, const double* partB, int64_t nbB, CgState* st,
                             int mode, hipStream_t s);
hipError_t launch_dc_replace(int64_t n, const double* b, const double* q, const float* dinv, float* r32,
                             CgState* st, int par, double rtol, double reduction, double* partials,
                             hipStream_t s);
hipError_t launch_resid_norm(int64_t n, const double* b, const double* q, CgState* st, double* partials,
                             hipStream_t s);
// K = exp(theta); changed != nullptr: *changed = 1 if any K differs from before, else 0
hipError_t launch_exp(int64_t n, const double* th, double* K64, float* K32, int* changed, hipStream_t s);
hipError_t launch_inv_diag(int64_t n, const double* d, double* i64, float* i32, const int* run, hipStream_t s);
hipError_t launch_to_f32(int64_t n, const double* a, float* b, hipStream_t s);

}  // namespace dg
