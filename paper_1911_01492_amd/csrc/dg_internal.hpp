// dg_internal.hpp -- shared definitions of the libdg HIP sources (gfx950).
//
// Everything here belongs to the GPU library; nothing is shared with the CPU
// oracle.  Notation: n = k+1 nodes per direction, N3 = n^3 values per element,
// element-blocked vectors (Sec. 3.3, DG codepath), local index
// i1 + n (i2 + n i3) with i1 along x.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dg {

constexpr int kMaxN = 8;  // k <= 7

// 1D reference operators on [0,1] (n GLL nodes, n Gauss points).
// An n x n matrix A with A[n-1-i][n-1-j] = SIGN A[i][j] (centro-symmetric,
// SIGN = +1, or centro-antisymmetric, SIGN = -1), as the 1D tables on the
// symmetric Gauss-Lobatto and Gauss points are, stored by its even-odd halves
// (h = n / 2; m = h is the middle index when n is odd):
//   E[i][j] = (A[i][j] + A[i][n-1-j]) / 2,  O[i][j] = (A[i][j] - A[i][n-1-j]) / 2  (i, j < h),
//   C[i] = A[i][m],  R[j] = A[m][j],  mm = A[m][m]                                 (n odd).
// A contraction then needs half the table and about 3/4 of the operations.
constexpr int kMaxH = kMaxN / 2;
template <typename T>
struct EvenOdd {
  T E[kMaxH * kMaxH];
  T O[kMaxH * kMaxH];
  T C[kMaxH];
  T R[kMaxH];
  T mm;
};

template <typename T>
struct Tables {
  T M[kMaxN * kMaxN];   // mass       M_ij = sum_q w_q l_i(x_q) l_j(x_q)
  T S[kMaxN * kMaxN];   // stiffness  S_ij = sum_q w_q l_i'(x_q) l_j'(x_q)
  T B[kMaxN * kMaxN];   // interpolation GLL -> Gauss, B_qi = l_i(x_q)
  T D[kMaxN * kMaxN];   // derivative at the Gauss points, D_qi = l_i'(x_q)
  T d0[kMaxN];          // l_i'(0)
  T d1[kMaxN];          // l_i'(1)
  T gw[kMaxN];          // Gauss weights on [0,1]
  T gx[kMaxN];          // Gauss points on [0,1]
  EvenOdd<T> eM, eS;    // M and S (symmetric, centro-symmetric)
  EvenOdd<T> eB, eBt;   // B and B^T (centro-symmetric)
  EvenOdd<T> eDg, eDgt; // Dg and Dg^T, Dg the collocation derivative on the Gauss
                        // points (Dg B = D; centro-antisymmetric)
  T Mis[kMaxN * kMaxN]; // M^{-1/2} (symmetric), for the generalized eigenproblems of
                        // the element block-Jacobi preconditioner
  T Cd[kMaxN * kMaxN];  // mixed matrix C_ij = sum_q w_q l_i(x_q) l_j'(x_q) = int l_i l_j'
  EvenOdd<T> eC;        // C by its even-odd halves (centro-antisymmetric)
};

// Eigen-decomposition of a symmetric n x n matrix (row stride kMaxN) by the
// cyclic Jacobi method (Jacobi 1846; the row-cyclic ordering with the
// symmetric 2 x 2 Schur rotation as in Golub and Van Loan, Matrix
// Computations, Sec. 8.5): a is overwritten (its diagonal holds the
// eigenvalues), v receives the eigenvectors as columns.  Sweeps stop when
// every off-diagonal entry is negligible against its two diagonal entries.
template <typename T>
__host__ __device__ inline void sym_eig_jacobi(int n, T* a, T* v) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) v[i * kMaxN + j] = i == j ? T(1) : T(0);
  for (int sweep = 0; sweep < 40; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const T apq = a[p * kMaxN + q];
        const T app = a[p * kMaxN + p], aqq = a[q * kMaxN + q];
        if (apq == T(0) || (T)1e-17 * (T)1e-17 * app * aqq >= apq * apq) continue;
        rotated = true;
        const T tau = (aqq - app) / (T(2) * apq);
        const T t = (tau >= T(0) ? T(1) : T(-1)) / ((tau >= T(0) ? tau : -tau) + sqrt(T(1) + tau * tau));
        const T c = T(1) / sqrt(T(1) + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q of a J
          const T akp = a[k * kMaxN + p], akq = a[k * kMaxN + q];
          a[k * kMaxN + p] = c * akp - s * akq;
          a[k * kMaxN + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q of J^T (a J)
          const T apk = a[p * kMaxN + k], aqk = a[q * kMaxN + k];
          a[p * kMaxN + k] = c * apk - s * aqk;
          a[q * kMaxN + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {  // v J
          const T vkp = v[k * kMaxN + p], vkq = v[k * kMaxN + q];
          v[k * kMaxN + p] = c * vkp - s * vkq;
          v[k * kMaxN + q] = s * vkp + c * vkq;
        }
      }
    if (!rotated) break;
  }
}

// Mesh data passed by value to the kernels.
template <typename T>
struct MeshArgs {
  int nx, ny, nz;
  int periodic;         // 1: periodic wrap, 0: weak Dirichlet
  int64_t E;            // elements
  T hx, hy, hz;         // 1/nx, 1/ny, 1/nz
  T sig_hat;            // penalty_hat (sigma_e = sig_hat / h_d)
  const T* K;           // E coefficients K_T = exp(theta_T)
  const T* G;           // 6 per element: face coefficient of face (d, s) at [6e + 2d + s]:
                        // gamma_e / 2 = K K' / (K + K') on interior faces, K on Dirichlet faces
  const T* vert;        // trilinear meshes: (nx+1)(ny+1)(nz+1) x 3 vertex coordinates
  const Tables<T>* tab; // 1D tables
  T ih[3];              // 1 / h_d
  T sg[3];              // sigma_e = sig_hat / h_d
  T At[3];              // face area h_t1 h_t2 of faces normal to d
  T vs[3];              // At_d / h_d (volume stiffness scale along d, without K)
  const T* R;           // E reaction coefficients c_T, or nullptr (no reaction term)
  T vol;                // h_x h_y h_z (affine element volume; |det J| on parallelepipeds)
  T go[3];              // parallelepiped meshes: the off-diagonal metric entries G_xy, G_xz,
                        // G_yz of G = |det J| J^-1 J^-T (zero on axis-parallel boxes)
  int affg;             // trilinear meshes: 1 when every element is a parallelepiped
  T* fb;                // trilinear meshes: per element and axis d, the 2 n^2 line scalars of
                        // its lower face (d, 0), written by the neighbour that evaluates the
                        // face in the first pass of the apply ([(3 e + d) 2 + k] n^2 + t)
};

// Block -> logical tile: consecutive logical tiles go to the same XCD (the
// hardware deals workgroups round-robin over the 8 XCDs), so each XCD works on
// a contiguous slab of elements and its L2 catches the neighbour re-reads.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
  const int64_t full = (nb / 8) * 8;
  if (b >= full) return b;
  return (b % 8) * (full / 8) + b / 8;
}

// bfloat16 (uint16 storage) <-> float
__device__ __forceinline__ float bf16_to_f32(uint16_t v) {
  return __uint_as_float(((uint32_t)v) << 16);
}
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)0x7fc0;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);                                // round to nearest even
  return (uint16_t)(u >> 16);
}

template <typename TC, typename TIN>
__device__ __forceinline__ TC load_as(const TIN* p) {
  return (TC)(*p);
}
template <>
__device__ __forceinline__ float load_as<float, uint16_t>(const uint16_t* p) {
  return bf16_to_f32(*p);
}
template <>
__device__ __forceinline__ double load_as<double, uint16_t>(const uint16_t* p) {
  return (double)bf16_to_f32(*p);
}

// Threads per block of the element kernels (always a multiple of the wave
// size) and elements per block for n nodes per direction (n^2 line threads
// per element; the remaining threads of the block idle).
constexpr int kBlock = 256;
__host__ __device__ constexpr int elems_per_block(int n) { return kBlock / (n * n); }

// wave64 sum of a double (all 64 lanes must be present)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic block reduction of one double: every thread passes its value;
// thread 0 gets the sum (fixed order: wave sums, then waves in index order).
template <int BLOCK>
__device__ double block_sum(double v, double* red /* BLOCK/64 entries */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (BLOCK + 63) / 64; ++i) s += red[i];
  }
  __syncthreads();
  return s;
}

// Per-block partial sums are written with plain stores and summed by a
// separate single-block kernel launched next on the same stream (kernel
// boundaries make them visible).  This avoids device-scope fences inside
// the producing kernels, which on gfx950 would write back the XCD's L2.
template <int NV>
__device__ __forceinline__ void store_partials(const double (&mine)[NV], double* partials, int64_t myblock) {
  if (threadIdx.x == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) partials[myblock * NV + v] = mine[v];
  }
}

// Deterministic sum of nblocks x NV partials by one block of BLOCK threads:
// fixed assignment of partials to threads, wave sums, then waves in order.
template <int NV, int BLOCK>
__device__ void sum_partials(const double* partials, int64_t nblocks, double (&tot)[NV]) {
  // U loads per thread are issued before any is added, so a batch costs one
  // memory latency (the partials come from every XCD and are not in this L2)
  constexpr int U = 8;
  __shared__ double red[NV][BLOCK / 64];
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  for (int64_t b0 = threadIdx.x; b0 < nblocks; b0 += (int64_t)BLOCK * U) {
    double val[U][NV];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t b = b0 + (int64_t)u * BLOCK;
#pragma unroll
      for (int v = 0; v < NV; ++v) val[u][v] = b < nblocks ? partials[b * NV + v] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += val[u][v];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double s = wave_sum(acc[v]);
    if (lane == 0) red[v][w] = s;
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    tot[v] = 0.0;
    for (int i = 0; i < BLOCK / 64; ++i) tot[v] += red[v][i];
  }
}

}  // namespace dg
