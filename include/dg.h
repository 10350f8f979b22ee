/*
 * dg.h -- C ABI of libdg: matrix-free, sum-factorised application of the
 * symmetric weighted interior-penalty (SWIPDG) operator for
 * -div(K grad u) = f (optionally -div(K grad u) + c u = f, dg_set_reaction)
 * on structured hexahedral meshes of the unit cube, with a
 * tensor-product Q_k Lagrange basis on Gauss-Lobatto nodes, on one AMD
 * Instinct MI355X (gfx950).
 *
 * The operator is the bilinear form of Sec. 4.1 ("Continuous problem and
 * discretization": element integrals of K grad u . grad v plus the face forms
 * b_h^e of SWIPDG), with these readings: minus signs on both consistency
 * terms, jump [w] = w^- - w^+ with the normal from T^- (lower index along the
 * face normal) to T^+, weighted average and penalty with the harmonic mean
 * gamma_e = 2 K^- K^+ / (K^- + K^+), penalty sigma_e = penalty_hat / h_d with
 * h_d = 1/n_d, weak Dirichlet u = 0 on boundary faces (-K grad u.n v -
 * K grad v.n u + sigma K u v) or periodic wrap in all directions, and
 * (k+1)-point Gauss quadrature per direction on volumes and faces.
 *
 * Vectors use the element-blocked ("DG codepath") layout of Sec. 3.3: the
 * (k+1)^3 values of element e = ex + nx (ey + ny ez) are contiguous, local
 * index i1 + n (i2 + n i3) with i1 along x fastest; the kernels read and
 * write the caller's global vectors in place, without gather/scatter copies.
 *
 * Conventions for every call:
 *   - Pointers named device are device pointers (e.g. from a contiguous
 *     torch tensor on the GPU); they are borrowed for the call only.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *     work on it and return without synchronising, except dg_setup and
 *     dg_cg_solve, which synchronise `stream` before returning.
 *   - Return values: DG_OK (0), solver outcomes > 0, errors < 0.  Errors
 *     leave outputs untouched where the arguments were rejected; the message
 *     is available from dg_last_error.  Nothing throws across the ABI.
 *   - A context is used by one host thread at a time.
 *   - The library allocates no device memory: everything it keeps lives in
 *     the caller's workspace (dg_query_workspace), which must outlive the
 *     context, except the static scratch array of dg_dA_dtheta_noalloc
 *     (16 MiB per GPU, part of the library's code object).
 */
#ifndef DG_H
#define DG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_ctx dg_ctx;

enum dg_status {
  DG_OK = 0,
  DG_NOT_CONVERGED = 1, /* dg_cg_solve hit maxit; the last iterate is in x            */
  DG_BREAKDOWN = 2,     /* dg_cg_solve met a non-positive or non-finite CG scalar     */
  DG_ERR_ARG = -1,      /* null / misaligned / aliased pointer, bad size or option    */
  DG_ERR_UNSUPPORTED = -2, /* degree or precision not built into the library        */
  DG_ERR_DEVICE = -3    /* a HIP call failed                                          */
};

enum dg_precision {
  DG_F64 = 0,  /* x: double, y: double; FP64 arithmetic                              */
  DG_F32 = 1,  /* x: float,  y: float;  FP32 arithmetic, FP32 tables and K          */
  DG_BF16 = 2, /* x: bfloat16 (uint16_t bit patterns), y: float; FP32 accumulation   */
  DG_BF16_MFMA = 3 /* as DG_BF16, with the tangential mass contractions (M (x) M on  *
                    * the n^2 points of every element plane) on the matrix cores:     *
                    * exact BF16 x operands, the matrix as a three-term BF16 sum,     *
                    * FP32 accumulation; the 1D operators along each axis in FP32.    *
                    * Affine meshes, k <= 4 (DG_ERR_UNSUPPORTED otherwise).           */
};

enum dg_bc { DG_BC_DIRICHLET0 = 0, DG_BC_PERIODIC = 1 };
/* DG_PC_JACOBI: M = diag(A)^-1.  DG_PC_BLOCK_JACOBI: M = blockdiag(A)^-1 over the
 * element blocks (Sec. 3.4's block preconditioners from the element blocks of
 * the DG matrix), inverted exactly by fast diagonalisation: on axis-parallel
 * box elements the block is a Kronecker sum of per-element 1D operators.
 * Affine meshes and DG_CG_STANDARD only (DG_ERR_UNSUPPORTED otherwise); in the
 * FP64 PCG and in the FP32-vector inner PCG of the defect correction. */
enum dg_preconditioner { DG_PC_NONE = 0, DG_PC_JACOBI = 1, DG_PC_BLOCK_JACOBI = 2 };

typedef struct {
  int32_t nx, ny, nz;        /* elements per direction, >= 1                              */
  int32_t degree;            /* k, 1 <= k <= 7                                             */
  int32_t bc;                /* enum dg_bc                                                 */
  int32_t reserved;          /* must be 0                                                  */
  double penalty_hat;        /* sigma_e * h_d; <= 0 selects 2 (k+1)^2                     */
  const double* vertices;    /* device, (nx+1)(ny+1)(nz+1) x 3 doubles, x-index fastest:   *
                              * trilinear elements; NULL = uniform grid (affine elements).  *
                              * Copied at setup.                                            */
  const double* theta;       /* device, nx*ny*nz doubles, K_T = exp(theta_T); NULL: K = 1.   *
                              * Copied at setup.                                            */
  void* workspace;           /* device, >= dg_query_workspace bytes, 256-byte aligned       */
  size_t workspace_bytes;
} dg_mesh_desc;

/* Bytes of device workspace the context for this mesh needs (pointers in the
 * descriptor are not read).  DG_ERR_ARG / DG_ERR_UNSUPPORTED on bad sizes. */
int dg_query_workspace(const dg_mesh_desc* mesh, size_t* bytes);

/* Build a context for the discrete problem of Sec. 4.1 ("Continuous problem
 * and discretization": the mesh T_h of the unit cube, the broken polynomial
 * space, the coefficient K) in the cell-blocked storage of the Sec. 3.3 DG
 * codepath: 1D tables (Gauss-Lobatto nodes, Gauss points, basis values and
 * derivatives) in FP64 on the host, K = exp(theta) in FP64 and FP32,
 * geometry, Jacobi diagonal.  With vertices, setup checks whether every
 * element is the same parallelepiped (the grid under one affine map, problem
 * B of Sec. 3.3) and then applies the operator with the constant-metric
 * kernel; dg_apply_kernel reports the choice.  Synchronises `stream`.  *out receives the
 * context (host memory owned by the library until dg_destroy).  Errors:
 * DG_ERR_ARG for a bad descriptor or a workspace below dg_query_workspace,
 * DG_ERR_UNSUPPORTED for a degree outside 1..7, DG_ERR_DEVICE for a failed HIP
 * call; *out is NULL then. */
int dg_setup(const dg_mesh_desc* mesh, dg_ctx** out, void* stream);

/* Replace the coefficient K of the form of Sec. 4.1: K_T = exp(theta_T)
 * (device, nx*ny*nz doubles), face coefficients and Jacobi diagonal.  When
 * every new K_T equals the current one bit for bit, the diagonal kernels find
 * that out on the device and return at once (no host synchronisation).
 * Asynchronous on `stream`.  Errors: DG_ERR_ARG for NULL pointers. */
int dg_set_theta(dg_ctx* ctx, const double* theta, void* stream);

/* Add a reaction term int c_T u v to the form (the diffusion-reaction problems
 * whose operator throughput Sec. 3.3 reports): c (device, nx*ny*nz doubles,
 * c_T >= 0 for a definite operator) is copied into the workspace; c == NULL
 * removes the term (the default after dg_setup).  The Jacobi diagonal is
 * recomputed; dg_dA_dtheta is unaffected (c does not depend on theta).
 * Asynchronous on `stream`. */
int dg_set_reaction(dg_ctx* ctx, const double* c, void* stream);

/* y = A x (Sec. 3.3 operator application; form of Sec. 4.1).  x and y are
 * device vectors of N_dof = nx*ny*nz*(k+1)^3 entries of the types given by
 * `prec` (enum dg_precision); x == y is rejected (DG_ERR_ARG).  On trilinear
 * meshes (other than equal parallelepipeds) the apply runs in two passes that
 * exchange face data through the context's workspace, so applies (and solves)
 * on one such context must not overlap in time: issue them on one stream or
 * order them with events. */
int dg_apply(dg_ctx* ctx, int prec, const void* x, void* y, void* stream);

/* y = A^T x, the operator of the adjoint problems.  The symmetric weighted
 * interior-penalty form of Sec. 4.1 is symmetric in its two arguments (the
 * consistency and symmetry terms are mirror images and the penalty term is
 * symmetric), so A^T = A.  Affine meshes: evaluated from the transposed 1D
 * operators and the transposed face algebra (equal to A x up to rounding);
 * parallelepiped and trilinear meshes: the apply itself.  Arguments and errors
 * as dg_apply. */
int dg_apply_transpose(dg_ctx* ctx, int prec, const void* x, void* y, void* stream);

/* Y = A X (transpose = 1: A^T X) for nrhs vectors at once, the multiple
 * right-hand sides of the block Krylov methods of Sec. 3.5 ("Horizontal
 * vectorization of Block Krylov methods").  X and Y hold nrhs device vectors of
 * N_dof entries each, one after another (vector j starts at entry j N_dof),
 * of the types given by `prec`; 1 <= nrhs <= 65535.  Affine meshes and meshes
 * of equal parallelepipeds: one launch with the vectors as the second grid
 * dimension; other trilinear meshes: one apply per vector.  Errors as dg_apply
 * (overlap of the X and Y ranges: DG_ERR_ARG). */
int dg_apply_multi(dg_ctx* ctx, int prec, int transpose, int nrhs, const void* X, void* Y, void* stream);

/* g_T = u^T (dA / dtheta_T) v for every element T (device: u, v N_dof
 * doubles, g nx*ny*nz doubles).  In the form of Sec. 4.1 the coefficient
 * enters through K_T in the element integrals and through the harmonic face
 * weights gamma_e of the face terms; this is the derivative of that form with
 * respect to theta_T = log K_T, as the gradient of an inverse problem
 * (Sec. 3.5 names optimisation and inverse problems among the users of
 * repeated solves) needs it: the volume form with K_T and each face form
 * of T with d gamma_e / d theta_T = gamma_e K_other / (K^- + K^+) (boundary:
 * K_T); the reaction term does not depend on theta.  FP64, affine and
 * trilinear meshes (on trilinear meshes the context's CG work space holds
 * per-element partial forms, so the call must not overlap a dg_cg_solve on
 * the same context). */
int dg_dA_dtheta(dg_ctx* ctx, const double* u, const double* v, double* g, void* stream);

/* For callers that cannot allocate device memory while they run (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * dg_dA_dtheta with its scratch in a static device array of the library
 * instead of the context's workspace.  Same arguments, results and errors as
 * dg_dA_dtheta (bit-identical g); no allocation of any kind.  On trilinear
 * meshes the per-element partial forms (7 doubles per element) go to a 16 MiB
 * array that each GPU holds until the process ends, so such meshes are limited
 * to 299593 elements (DG_ERR_ARG above that); affine meshes need no scratch.
 * All calls on one GPU share that array and every call overwrites it: calls
 * that overlap in time on one GPU (other streams, other contexts, other host
 * threads) race and must be ordered by the caller. */
int dg_dA_dtheta_noalloc(dg_ctx* ctx, const double* u, const double* v, double* g, void* stream);

/* d = diag(A) (device, N_dof doubles), FP64: the point-Jacobi choice of the
 * preconditioner M that Alg. "PCG" of Sec. 2.4 leaves open (the smallest of
 * the block-diagonal preconditioners Sec. 3.4 builds from the element
 * blocks).  Errors: DG_ERR_ARG for NULL pointers. */
int dg_diagonal(dg_ctx* ctx, double* d, void* stream);

/* Physical coordinates of the (k+1)^3 volume Gauss points of every element
 * (device, N_dof x 3 doubles, element-blocked, point index q1 + n(q2 + n q3)). */
int dg_quadrature_points(dg_ctx* ctx, double* xq, void* stream);

/* Load vector b_i = int f phi_i by (k+1)-point Gauss quadrature from the
 * values of f at the points of dg_quadrature_points (device, N_dof doubles). */
int dg_load_vector(dg_ctx* ctx, const double* fq, double* b, void* stream);

/* How the FP64 defect correction (prec_inner DG_F32 / DG_BF16) continues
 * after an outer step x += d, r = b - A x (FP64):
 *  DG_DC_RESTART  a fresh inner PCG on A d = r from d = 0 (default inner_rtol
 *                 1e-5 for DG_F32, 1e-2 for DG_BF16; default max_outer 30);
 *  DG_DC_KEEP     the FP64 residual replaces the inner one and CG continues
 *                 along its current direction (p = z + beta p with the new
 *                 residual); an inner segment ends when its residual fell by
 *                 inner_rtol (default 0.1) or below half the outer target
 *                 (default max_outer 200).  Falls back to a fresh direction
 *                 after an inner breakdown. */
enum dg_dc_mode { DG_DC_RESTART = 0, DG_DC_KEEP = 1 };

/* DG_CG_STANDARD: Alg. "PCG" of Sec. 2.4 with the norm check merged into the
 * <z, r> reduction (two reductions per iteration).  DG_CG_SINGLE_REDUCTION:
 * the same iterates (up to rounding) from the single-reduction recurrences of
 * Chronopoulos and Gear cited in Sec. 2.4 (s = A p carried by recurrence, w = A z
 * applied; one reduction of {<r, z>, <r, r>, <z, w>} per iteration, two more
 * streamed vectors).  FP64 solves only. */
enum dg_cg_variant { DG_CG_STANDARD = 0, DG_CG_SINGLE_REDUCTION = 1 };

typedef struct {
  int prec_inner;     /* DG_F64: FP64 PCG.  DG_F32 / DG_BF16: FP64 defect correction  *
                       * whose inner PCG runs on FP32 vectors with that apply          */
  int precond;        /* enum dg_preconditioner                                       */
  int transpose;      /* 1: solve A^T x = b                                            */
  double rtol;        /* stop when ||b - A x||_2 <= rtol ||b||_2 (true FP64 residual)  */
  double inner_rtol;  /* inner PCG reduction for prec_inner != DG_F64; <= 0: default   */
  int maxit;          /* total (inner) CG iterations allowed                          */
  int max_outer;      /* outer corrections allowed (mixed precision)                  */
  int check_every;    /* host looks at the device convergence flag every this many     *
                       * iterations (>= 1; <= 0: default 32; up to this many - 1       *
                       * iterations after convergence run as no-op launches)           */
  int dc_mode;        /* enum dg_dc_mode (mixed precision only; must be valid always)  */
  int cg_variant;     /* enum dg_cg_variant (prec_inner DG_F64 only for the second)   */
} dg_cg_opts;

typedef struct {
  int status;               /* DG_OK, DG_NOT_CONVERGED or DG_BREAKDOWN                  */
  int iters;                /* CG iterations performed (inner iterations in total)     */
  int outer_iters;          /* defect-correction steps (0 for FP64 PCG)                */
  int restarts;             /* FP64 PCG restarts after a failed true-residual check    */
  double rel_true_residual; /* ||b - A x|| / ||b|| in FP64 at return                   */
  double seconds;           /* wall time of the call                                  */
} dg_cg_info;

/* Solve A x = b (or A^T x = b) with Alg. "PCG" of Sec. 2.4 (Jacobi or no
 * preconditioner; the norm check merged into the <z, r> reduction, so two
 * reductions per iteration) in FP64, or with FP64 defect correction around
 * an FP32-vector PCG (prec_inner DG_F32 / DG_BF16).  b and x are device FP64
 * vectors; x holds x0 on entry and the result on exit.  Synchronises
 * `stream`; info is always filled when the arguments are accepted. */
int dg_cg_solve(dg_ctx* ctx, const dg_cg_opts* opts, const double* b, double* x, dg_cg_info* info,
                void* stream);

/* N_dof, element count and nodes per direction of a context. */
int64_t dg_num_dofs(const dg_ctx* ctx);
int64_t dg_num_elements(const dg_ctx* ctx);
int dg_nodes_per_dir(const dg_ctx* ctx);

/* The apply kernel dg_setup chose for the mesh (Sec. 3.3 benchmarks the
 * operator on axis-parallel grids, problem A, and on affine geometries,
 * problem B):  DG_KERNEL_AFFINE for axis-parallel boxes (no vertices given),
 * DG_KERNEL_TRILINEAR for general trilinear element maps (Jacobian at every
 * quadrature point), DG_KERNEL_PARALLELEPIPED when every element is the same
 * parallelepiped (the grid under one affine map: constant metric, the
 * axis-parallel kernel plus the mixed-derivative terms).  -1 for a NULL
 * context. */
enum dg_kernel { DG_KERNEL_AFFINE = 0, DG_KERNEL_TRILINEAR = 1, DG_KERNEL_PARALLELEPIPED = 2 };
int dg_apply_kernel(const dg_ctx* ctx);

/* Release the context's host memory (the caller frees the workspace). */
void dg_destroy(dg_ctx* ctx);

/* Message of the last failed call on ctx (or of the last failed dg_setup /
 * dg_query_workspace when ctx is NULL).  Valid until the next call. */
const char* dg_last_error(const dg_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* DG_H */
