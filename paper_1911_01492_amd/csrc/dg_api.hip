// dg_api.hip -- host side of libdg: the C ABI declared in include/dg.h.
//
// Holds the context (mesh, 1D tables, pointers into the caller's workspace),
// validates arguments, dispatches kernels by (geometry, n, precision) and
// drives the Krylov solvers: Alg. "PCG" of Sec. 2.4 in FP64 and an FP64
// defect correction around an FP32-vector PCG.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/dg.h"
#include "dg_internal.hpp"
#include "dg_kernels.hpp"

using namespace dg;

struct dg_ctx {
  dg_mesh_desc desc;
  int n;                 // nodes per direction
  int64_t E, ndof;
  bool trilinear;
  // workspace regions
  Tables<double>* tab64;
  Tables<float>* tab32;
  double* K64;
  float* K32;
  double* G64;           // face coefficients, 6 per element
  float* G32;
  double* R64;           // reaction coefficients, 1 per element (used when `reaction`)
  float* R32;
  bool reaction;
  bool affine_geom;      // trilinear mesh whose elements are all parallelepipeds
  bool ppd;              // ... and all the same parallelepiped (an affine image of the grid):
                         // the apply takes the constant-metric kernel
  double pG[6];          // its metric |det J| J^-1 J^-T: xx, yy, zz, xy, xz, yz
  double parea[3];       // face areas |J e_a x J e_b| of the faces normal to d
  double pdet;           // det J
  double* vert64;
  float* vert32;
  double* dinv64;
  float* dinv32;
  double *bjQ64, *bjL64;  // block-Jacobi factors (affine meshes): Q_d and l_d per element and axis
  float *bjQ32, *bjL32;
  double *r64, *p64, *q64;
  double *z64, *s64, *w64;   // single-reduction CG
  float *r32, *d32, *p32, *q32, *z32;
  uint16_t* p16;
  void* fb;              // trilinear meshes: lower-face line scalars between the two apply passes
  double* partials;
  CgState* st;           // [0]: outer / FP64 solve, [1]: inner solve
  int* coef_changed;     // set by dg_set_theta's exp kernel when K changed (device)
  double* scratch;       // this device's copy of the static scratch array (dg_dA_dtheta_noalloc)
  std::string err;
};

// ------------------------------------------------------------------ static scratch
// Scratch of dg_dA_dtheta_noalloc: the per-element partial forms of trilinear
// meshes (7 doubles per element) live in this file-scope device array instead
// of the caller's workspace.  Every GPU the library runs on holds its own copy
// until the process ends.  In host code the name `scratch` is only a stand-in
// for the symbol: its device address is looked up once per device (at the
// first dg_setup with that device current) and only that address is used.
static constexpr size_t kScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];
static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (resolved once per device)
static hipError_t scratch_address(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

namespace {

thread_local std::string g_err;

int fail(dg_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  else g_err = msg;
  return code;
}

#define HIP_TRY(c, expr)                                                                    \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail((c), DG_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

// ------------------------------------------------------------------ 1D tables
// Gauss-Legendre points by the Golub-Welsch method (eigenvalues of the
// symmetric tridiagonal Jacobi matrix of the Legendre recurrence, weights from
// the first eigenvector components), and the interior Gauss-Lobatto nodes as
// the Gauss points of the Jacobi weight (1-x^2) (roots of P^(1,1)_{n-2}, i.e.
// of P'_{n-1}).  Eigen-decomposition: the implicit QL algorithm with
// Wilkinson shifts for symmetric tridiagonal matrices, as published by
// Bowdler, Martin, Reinsch and Wilkinson (procedure tql2, Numer. Math. 11,
// 1968; Handbook for Automatic Computation, Vol. II), restricted here to the
// first row of the eigenvector matrix.

// diag d[0..m), off-diagonal e[1..m) (e[0] unused); on exit d = eigenvalues,
// z[0..m) = first components of the normalised eigenvectors.
bool tridiag_ql(std::vector<double>& d, std::vector<double> e, std::vector<double>& z0) {
  const int m = (int)d.size();
  std::vector<double> Z((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) Z[(size_t)i * m + i] = 1.0;
  for (int i = 1; i < m; ++i) e[i - 1] = e[i];
  if (m > 0) e[m - 1] = 0.0;
  for (int l = 0; l < m; ++l) {
    int iter = 0, mm;
    do {
      for (mm = l; mm < m - 1; ++mm) {
        const double dd = std::fabs(d[mm]) + std::fabs(d[mm + 1]);
        if (std::fabs(e[mm]) <= 1e-17 * dd) break;
      }
      if (mm != l) {
        if (++iter > 60) return false;
        double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
        double r = std::hypot(g, 1.0);
        g = d[mm] - d[l] + e[l] / (g + (g >= 0 ? std::fabs(r) : -std::fabs(r)));
        double s = 1.0, c = 1.0, p = 0.0;
        int i;
        for (i = mm - 1; i >= l; --i) {
          double f = s * e[i], b = c * e[i];
          r = std::hypot(f, g);
          e[i + 1] = r;
          if (r == 0.0) {
            d[i + 1] -= p;
            e[mm] = 0.0;
            break;
          }
          s = f / r;
          c = g / r;
          g = d[i + 1] - p;
          r = (d[i] - g) * s + 2.0 * c * b;
          p = s * r;
          d[i + 1] = g + p;
          g = c * r - b;
          for (int k = 0; k < m; ++k) {
            f = Z[(size_t)k * m + i + 1];
            Z[(size_t)k * m + i + 1] = s * Z[(size_t)k * m + i] + c * f;
            Z[(size_t)k * m + i] = c * Z[(size_t)k * m + i] - s * f;
          }
        }
        if (r == 0.0 && i >= l) continue;
        d[l] -= p;
        e[l] = g;
        e[mm] = 0.0;
      }
    } while (mm != l);
  }
  z0.assign(m, 0.0);
  for (int j = 0; j < m; ++j) z0[j] = Z[j];  // row 0 of the eigenvector matrix
  return true;
}

// q-point Gauss-Legendre on [0,1], ascending
bool gauss01(int q, std::vector<double>& x, std::vector<double>& w) {
  std::vector<double> d(q, 0.0), e(q, 0.0), z;
  for (int k = 1; k < q; ++k) e[k] = k / std::sqrt(4.0 * k * k - 1.0);
  if (!tridiag_ql(d, e, z)) return false;
  std::vector<int> idx(q);
  for (int i = 0; i < q; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
  x.resize(q);
  w.resize(q);
  for (int i = 0; i < q; ++i) {
    x[i] = 0.5 * (d[idx[i]] + 1.0);
    w[i] = z[idx[i]] * z[idx[i]];  // 2 z^2 on [-1,1], halved on [0,1]
  }
  return true;
}

// n Gauss-Lobatto nodes on [0,1]: 0, the n-2 roots of P^(1,1)_{n-2}, 1
bool lobatto01(int n, std::vector<double>& x) {
  const int m = n - 2;
  x.assign(n, 0.0);
  x[n - 1] = 1.0;
  if (m <= 0) return true;
  std::vector<double> d(m, 0.0), e(m, 0.0), z;
  for (int k = 1; k < m; ++k) e[k] = std::sqrt((double)k * (k + 2) / ((2.0 * k + 1) * (2.0 * k + 3)));
  if (!tridiag_ql(d, e, z)) return false;
  std::sort(d.begin(), d.end());
  for (int i = 0; i < m; ++i) x[i + 1] = 0.5 * (d[i] + 1.0);
  return true;
}

// Lagrange basis on nodes xs, barycentric form: values at points, and the
// differentiation matrix at the nodes Dn[k][i] = l_i'(xs_k).
struct Bary {
  std::vector<double> xs, w;
  explicit Bary(const std::vector<double>& nodes) : xs(nodes), w(nodes.size(), 1.0) {
    for (size_t i = 0; i < xs.size(); ++i)
      for (size_t j = 0; j < xs.size(); ++j)
        if (i != j) w[i] /= (xs[i] - xs[j]);
  }
  void values(double x, std::vector<double>& l) const {
    const size_t n = xs.size();
    l.assign(n, 0.0);
    for (size_t i = 0; i < n; ++i)
      if (x == xs[i]) {
        l[i] = 1.0;
        return;
      }
    double den = 0.0;
    for (size_t i = 0; i < n; ++i) den += w[i] / (x - xs[i]);
    for (size_t i = 0; i < n; ++i) l[i] = (w[i] / (x - xs[i])) / den;
  }
  void diff_matrix(std::vector<double>& Dn) const {
    const size_t n = xs.size();
    Dn.assign(n * n, 0.0);
    for (size_t k = 0; k < n; ++k) {
      double s = 0.0;
      for (size_t i = 0; i < n; ++i)
        if (i != k) {
          Dn[k * n + i] = (w[i] / w[k]) / (xs[k] - xs[i]);
          s += Dn[k * n + i];
        }
      Dn[k * n + k] = -s;
    }
  }
};

// Even-odd halves of an n x n matrix A (row-major, stride n) with
// A[n-1-i][n-1-j] = sign A[i][j]; false if A lacks that symmetry (beyond
// rounding), which would make the halves describe another matrix.
bool even_odd(int n, const std::vector<double>& A, int sign, EvenOdd<double>& eo) {
  double amax = 0.0;
  for (double a : A) amax = std::max(amax, std::fabs(a));
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (std::fabs(A[(n - 1 - i) * n + (n - 1 - j)] - sign * A[i * n + j]) > 1e-13 * amax) return false;
  const int h = n / 2, m = h;
  for (int i = 0; i < h; ++i) {
    for (int j = 0; j < h; ++j) {
      eo.E[i * kMaxH + j] = 0.5 * (A[i * n + j] + A[i * n + (n - 1 - j)]);
      eo.O[i * kMaxH + j] = 0.5 * (A[i * n + j] - A[i * n + (n - 1 - j)]);
    }
    if (n & 1) {
      eo.C[i] = A[i * n + m];
      eo.R[i] = A[m * n + i];
    }
  }
  if (n & 1) eo.mm = A[m * n + m];
  return true;
}

void even_odd_to_f32(const EvenOdd<double>& a, EvenOdd<float>& b) {
  for (int i = 0; i < kMaxH * kMaxH; ++i) {
    b.E[i] = (float)a.E[i];
    b.O[i] = (float)a.O[i];
  }
  for (int i = 0; i < kMaxH; ++i) {
    b.C[i] = (float)a.C[i];
    b.R[i] = (float)a.R[i];
  }
  b.mm = (float)a.mm;
}

bool build_tables(int n, Tables<double>& T) {
  std::memset(&T, 0, sizeof(T));
  std::vector<double> gll, gx, gw;
  if (!lobatto01(n, gll) || !gauss01(n, gx, gw)) return false;
  Bary L(gll), G(gx);
  std::vector<double> Dn, Dg, l;
  L.diff_matrix(Dn);  // Dn[k][i] = l_i'(gll_k)
  G.diff_matrix(Dg);  // Gauss-point collocation derivative
  // B[q][i] = l_i(x_q), D[q][i] = l_i'(x_q) = sum_k l_k(x_q) Dn[k][i]
  std::vector<double> B((size_t)n * n), D((size_t)n * n, 0.0);
  for (int q = 0; q < n; ++q) {
    L.values(gx[q], l);
    for (int i = 0; i < n; ++i) {
      B[q * n + i] = l[i];
      for (int k = 0; k < n; ++k) D[q * n + i] += l[k] * Dn[k * n + i];
    }
  }
  std::vector<double> Mv((size_t)n * n), Sv((size_t)n * n), Cv((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double m = 0.0, s = 0.0, cm = 0.0;
      for (int q = 0; q < n; ++q) {
        m += gw[q] * B[q * n + i] * B[q * n + j];
        s += gw[q] * D[q * n + i] * D[q * n + j];
        cm += gw[q] * B[q * n + i] * D[q * n + j];
      }
      T.M[i * kMaxN + j] = m;
      T.S[i * kMaxN + j] = s;
      T.Cd[i * kMaxN + j] = cm;
      Mv[i * n + j] = m;
      Sv[i * n + j] = s;
      Cv[i * n + j] = cm;
      T.B[i * kMaxN + j] = B[i * n + j];
      T.D[i * kMaxN + j] = D[i * n + j];
    }
  for (int i = 0; i < n; ++i) {
    T.d0[i] = Dn[0 * n + i];
    T.d1[i] = Dn[(size_t)(n - 1) * n + i];
    T.gw[i] = gw[i];
    T.gx[i] = gx[i];
  }
  std::vector<double> Bt((size_t)n * n), Dgt((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      Bt[i * n + j] = B[j * n + i];
      Dgt[i * n + j] = Dg[j * n + i];
    }
  {  // M^{-1/2} = V diag(mu^{-1/2}) V^T from the eigen-decomposition of M
    double a[kMaxN * kMaxN], v[kMaxN * kMaxN];
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) a[i * kMaxN + j] = Mv[i * n + j];
    sym_eig_jacobi<double>(n, a, v);
    for (int i = 0; i < n; ++i) {
      if (!(a[i * kMaxN + i] > 0.0)) return false;
      for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += v[i * kMaxN + k] * v[j * kMaxN + k] / std::sqrt(a[k * kMaxN + k]);
        T.Mis[i * kMaxN + j] = s;
      }
    }
  }
  return even_odd(n, Mv, 1, T.eM) && even_odd(n, Sv, 1, T.eS) && even_odd(n, B, 1, T.eB) &&
         even_odd(n, Bt, 1, T.eBt) && even_odd(n, Dg, -1, T.eDg) && even_odd(n, Dgt, -1, T.eDgt) &&
         even_odd(n, Cv, -1, T.eC);
}

void tables_to_f32(const Tables<double>& a, Tables<float>& b) {
  for (int i = 0; i < kMaxN * kMaxN; ++i) {
    b.M[i] = (float)a.M[i];
    b.Mis[i] = (float)a.Mis[i];
    b.S[i] = (float)a.S[i];
    b.B[i] = (float)a.B[i];
    b.D[i] = (float)a.D[i];
    b.Cd[i] = (float)a.Cd[i];
  }
  for (int i = 0; i < kMaxN; ++i) {
    b.d0[i] = (float)a.d0[i];
    b.d1[i] = (float)a.d1[i];
    b.gw[i] = (float)a.gw[i];
    b.gx[i] = (float)a.gx[i];
  }
  even_odd_to_f32(a.eM, b.eM);
  even_odd_to_f32(a.eS, b.eS);
  even_odd_to_f32(a.eB, b.eB);
  even_odd_to_f32(a.eBt, b.eBt);
  even_odd_to_f32(a.eDg, b.eDg);
  even_odd_to_f32(a.eDgt, b.eDgt);
  even_odd_to_f32(a.eC, b.eC);
}

// ------------------------------------------------------------------ workspace
struct Layout {
  size_t tab64, tab32, K64, K32, G64, G32, R64, R32, vert64, vert32, dinv64, dinv32, bjQ64, bjL64, bjQ32, bjL32, r64,
      p64, q64, r32, d32, p32, q32, z32, p16, z64, s64, w64, fb, partials, st, flags, total;
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int check_desc(const dg_mesh_desc* m, dg_ctx* c) {
  if (!m) return fail(c, DG_ERR_ARG, "mesh descriptor is NULL");
  if (m->nx < 1 || m->ny < 1 || m->nz < 1) return fail(c, DG_ERR_ARG, "element counts must be >= 1");
  if (m->degree < 1 || m->degree > kMaxN - 1)
    return fail(c, DG_ERR_UNSUPPORTED, "degree must be in 1..7");
  if (m->bc != DG_BC_DIRICHLET0 && m->bc != DG_BC_PERIODIC) return fail(c, DG_ERR_ARG, "unknown bc");
  if (m->reserved != 0) return fail(c, DG_ERR_ARG, "reserved field must be 0");
  const double E = (double)m->nx * m->ny * m->nz;
  const double n3 = std::pow(m->degree + 1.0, 3);
  if (E * n3 >= 2147483648.0) return fail(c, DG_ERR_ARG, "mesh too large (N_dof must be below 2^31)");
  if ((double)m->nx * m->ny * m->nz > 2.0e9) return fail(c, DG_ERR_ARG, "too many elements");
  return DG_OK;
}

Layout layout(const dg_mesh_desc* m) {
  const int n = m->degree + 1;
  const int64_t E = (int64_t)m->nx * m->ny * m->nz;
  const int64_t nd = E * n * n * n;
  const int64_t nv = (int64_t)(m->nx + 1) * (m->ny + 1) * (m->nz + 1);
  const bool tri = m->vertices != nullptr;
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.tab64 = take(sizeof(Tables<double>));
  L.tab32 = take(sizeof(Tables<float>));
  L.K64 = take(E * sizeof(double));
  L.K32 = take(E * sizeof(float));
  L.G64 = take(6 * E * sizeof(double));
  L.G32 = take(6 * E * sizeof(float));
  L.R64 = take(E * sizeof(double));
  L.R32 = take(E * sizeof(float));
  L.vert64 = take(tri ? nv * 3 * sizeof(double) : 0);
  L.vert32 = take(tri ? nv * 3 * sizeof(float) : 0);
  L.dinv64 = take(nd * sizeof(double));
  L.dinv32 = take(nd * sizeof(float));
  L.bjQ64 = take(tri ? 0 : (size_t)E * 3 * n * n * sizeof(double));
  L.bjL64 = take(tri ? 0 : (size_t)E * 3 * n * sizeof(double));
  L.bjQ32 = take(tri ? 0 : (size_t)E * 3 * n * n * sizeof(float));
  L.bjL32 = take(tri ? 0 : (size_t)E * 3 * n * sizeof(float));
  L.r64 = take(nd * sizeof(double));
  L.p64 = take(nd * sizeof(double));
  L.q64 = take(nd * sizeof(double));
  L.r32 = take(nd * sizeof(float));
  L.d32 = take(nd * sizeof(float));
  L.p32 = take(nd * sizeof(float));
  L.q32 = take(nd * sizeof(float));
  L.z32 = take(tri ? 0 : nd * sizeof(float));  // block-Jacobi z of the inner solves
  L.p16 = take(nd * sizeof(uint16_t));
  L.z64 = take(nd * sizeof(double));
  L.s64 = take(nd * sizeof(double));
  L.w64 = take(nd * sizeof(double));
  L.fb = take(tri ? (size_t)E * 3 * 2 * n * n * sizeof(double) : 0);  // FP64 size, shared by the FP32 applies
  const int64_t nb = std::max<int64_t>(std::max<int64_t>(element_blocks(n, E), vec_blocks(nd)),
                                       affine_tiles(n, m->nx, m->ny, m->nz));
  L.partials = take((size_t)nb * 3 * sizeof(double));
  L.st = take(2 * sizeof(CgState));
  L.flags = take(64);
  L.total = o;
  return L;
}

// 1/h_d, sigma_e = sig_hat / h_d, face area and At / h_d, computed in FP64
template <typename T>
void fill_scales(MeshArgs<T>& m) {
  const double h[3] = {1.0 / m.nx, 1.0 / m.ny, 1.0 / m.nz};
  const double sh = (double)m.sig_hat;
  for (int d = 0; d < 3; ++d) {
    const double at = h[(d + 1) % 3] * h[(d + 2) % 3];
    m.ih[d] = (T)(1.0 / h[d]);
    m.sg[d] = (T)(sh / h[d]);
    m.At[d] = (T)at;
    m.vs[d] = (T)(at / h[d]);
  }
}

MeshArgs<double> args64(const dg_ctx* c) {
  MeshArgs<double> m;
  m.nx = c->desc.nx;
  m.ny = c->desc.ny;
  m.nz = c->desc.nz;
  m.periodic = c->desc.bc == DG_BC_PERIODIC;
  m.E = c->E;
  m.hx = 1.0 / c->desc.nx;
  m.hy = 1.0 / c->desc.ny;
  m.hz = 1.0 / c->desc.nz;
  m.sig_hat = c->desc.penalty_hat > 0 ? c->desc.penalty_hat : 2.0 * c->n * c->n;
  m.K = c->K64;
  m.G = c->G64;
  m.vert = c->vert64;
  m.tab = c->tab64;
  m.R = c->reaction ? c->R64 : nullptr;
  m.vol = (1.0 / c->desc.nx) * (1.0 / c->desc.ny) * (1.0 / c->desc.nz);
  m.affg = c->affine_geom ? 1 : 0;
  m.fb = (double*)c->fb;
  m.go[0] = m.go[1] = m.go[2] = 0.0;
  fill_scales(m);
  return m;
}
MeshArgs<float> args32(const dg_ctx* c) {
  MeshArgs<float> m;
  m.nx = c->desc.nx;
  m.ny = c->desc.ny;
  m.nz = c->desc.nz;
  m.periodic = c->desc.bc == DG_BC_PERIODIC;
  m.E = c->E;
  m.hx = (float)(1.0 / c->desc.nx);
  m.hy = (float)(1.0 / c->desc.ny);
  m.hz = (float)(1.0 / c->desc.nz);
  m.sig_hat = (float)(c->desc.penalty_hat > 0 ? c->desc.penalty_hat : 2.0 * c->n * c->n);
  m.K = c->K32;
  m.G = c->G32;
  m.vert = c->vert32;
  m.tab = c->tab32;
  m.R = c->reaction ? c->R32 : nullptr;
  m.vol = (float)((1.0 / c->desc.nx) * (1.0 / c->desc.ny) * (1.0 / c->desc.nz));
  m.affg = c->affine_geom ? 1 : 0;
  m.fb = (float*)c->fb;
  m.go[0] = m.go[1] = m.go[2] = 0.0f;
  fill_scales(m);
  return m;
}

// The scalars of the constant-metric apply on a mesh of equal
// parallelepipeds: the line operators take the diagonal metric entries (volume
// and normal-flux scale G_dd) and the face areas, the off-diagonal entries
// couple the axes; computed in FP64 from the mesh's J.
template <typename T>
MeshArgs<T> ppd_args(const dg_ctx* c, MeshArgs<T> m) {
  for (int d = 0; d < 3; ++d) {
    m.vs[d] = (T)c->pG[d];
    m.At[d] = (T)c->parea[d];
    m.ih[d] = (T)(c->pG[d] / c->parea[d]);
  }
  m.go[0] = (T)c->pG[3];
  m.go[1] = (T)c->pG[4];
  m.go[2] = (T)c->pG[5];
  m.vol = (T)c->pdet;
  return m;
}

// dot != 0: <x, A x> into st->pq (st must then be given; par selects rho for the
// breakdown check)
// block partials of the fused <x, A x> of an apply: one per brick of the
// affine and parallelepiped kernels, one per element block of the trilinear one
int64_t apply_partials(const dg_ctx* c) {
  if (c->trilinear && !c->ppd) return element_blocks(c->n, c->E);
  return affine_tiles(c->n, c->desc.nx, c->desc.ny, c->desc.nz);
}

hipError_t apply_any(dg_ctx* c, int prec, int trans, int dot, const void* x, void* y, CgState* st, int par,
                     const int* skip, hipStream_t s, double* partials = nullptr) {
  const MeshArgs<double> m64 = args64(c);
  const MeshArgs<float> m32 = args32(c);
  double* part = partials ? partials : c->partials;
  if (c->ppd)  // the form is symmetric: the transpose is the same operator
    return launch_apply_ppd(c->n, prec, dot, ppd_args(c, m64), ppd_args(c, m32), x, y, part, st, par, skip, s);
  if (c->trilinear)
    return launch_apply_trilinear(c->n, prec, trans, dot, m64, m32, x, y, part, st, par, skip, s);
  return launch_apply_affine(c->n, prec, trans, dot, m64, m32, x, y, part, st, par, skip, s);
}

// K = exp(theta) and the face coefficients; changed != nullptr: the exp kernel
// records in *changed whether any K_T differs from the current one
hipError_t coef_setup(dg_ctx* c, const double* theta, int* changed, hipStream_t s) {
  hipError_t e = launch_exp(c->E, theta, c->K64, c->K32, changed, s);
  if (e != hipSuccess) return e;
  MeshArgs<double> m = args64(c);
  return launch_face_coef(m, c->G64, c->G32, s);
}

// Jacobi diagonal and its inverse; run != nullptr: the kernels do nothing when
// *run == 0 on the device (the coefficients did not change)
hipError_t compute_dinv(dg_ctx* c, hipStream_t s, const int* run = nullptr) {
  const MeshArgs<double> m64 = args64(c);
  hipError_t e = c->trilinear ? launch_diag_trilinear(c->n, m64, c->r64, run, s)
                              : launch_diag_affine(c->n, m64, c->r64, run, s);
  if (e != hipSuccess) return e;
  e = launch_inv_diag(c->ndof, c->r64, c->dinv64, c->dinv32, run, s);
  if (e != hipSuccess || c->trilinear) return e;
  // element block-Jacobi factors (cheap: one small eigenproblem per element and axis)
  return launch_bj_setup(c->n, m64, c->bjQ64, c->bjL64, c->bjQ32, c->bjL32, s);
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

}  // namespace

// ====================================================================== C ABI
extern "C" {

int dg_query_workspace(const dg_mesh_desc* mesh, size_t* bytes) {
  int rc = check_desc(mesh, nullptr);
  if (rc != DG_OK) return rc;
  if (!bytes) return fail(nullptr, DG_ERR_ARG, "bytes is NULL");
  *bytes = layout(mesh).total;
  return DG_OK;
}

// True when the trilinear map of every element is affine: the coefficients of
// xi1 xi2, xi1 xi3, xi2 xi3 and xi1 xi2 xi3 vanish (to a few ulps of the
// element size), i.e. every element is a parallelepiped.
static bool all_parallelepipeds(int nx, int ny, int nz, const std::vector<double>& v) {
  const double h = 1.0 / std::max(nx, std::max(ny, nz));
  const double tol = 64.0 * 2.220446049250313e-16 * std::max(1.0, h);
  auto X = [&](int ix, int iy, int iz, int a) { return v[3 * (ix + (size_t)(nx + 1) * (iy + (size_t)(ny + 1) * iz)) + a]; };
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x)
        for (int a = 0; a < 3; ++a) {
          const double c000 = X(x, y, z, a), c100 = X(x + 1, y, z, a), c010 = X(x, y + 1, z, a),
                       c110 = X(x + 1, y + 1, z, a), c001 = X(x, y, z + 1, a), c101 = X(x + 1, y, z + 1, a),
                       c011 = X(x, y + 1, z + 1, a), c111 = X(x + 1, y + 1, z + 1, a);
          const double b12 = c110 - c100 - c010 + c000, b13 = c101 - c100 - c001 + c000,
                       b23 = c011 - c010 - c001 + c000,
                       b123 = c111 - c110 - c101 - c011 + c100 + c010 + c001 - c000;
          if (std::fabs(b12) > tol || std::fabs(b13) > tol || std::fabs(b23) > tol || std::fabs(b123) > tol)
            return false;
        }
  return true;
}

// Every element is the same parallelepiped: J from the extent of the whole
// mesh (the grid's affine image), each element's edge vectors equal to its
// columns within 8 ulps of the largest coordinate, det J > 0.  Fills the
// metric, face areas and determinant of c.  Call only when every element is
// a parallelepiped.
static bool uniform_parallelepipeds(int nx, int ny, int nz, const std::vector<double>& v, dg_ctx* c) {
  auto X = [&](int ix, int iy, int iz, int a) { return v[3 * (ix + (size_t)(nx + 1) * (iy + (size_t)(ny + 1) * iz)) + a]; };
  double J[3][3], xmax = 0.0;
  for (int a = 0; a < 3; ++a) {
    J[a][0] = (X(nx, 0, 0, a) - X(0, 0, 0, a)) / nx;
    J[a][1] = (X(0, ny, 0, a) - X(0, 0, 0, a)) / ny;
    J[a][2] = (X(0, 0, nz, a) - X(0, 0, 0, a)) / nz;
  }
  for (double q : v) xmax = std::max(xmax, std::fabs(q));
  const double tol = 8.0 * 2.220446049250313e-16 * std::max(1.0, xmax);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x)
        for (int a = 0; a < 3; ++a) {
          const double o = X(x, y, z, a);
          if (std::fabs(X(x + 1, y, z, a) - o - J[a][0]) > tol || std::fabs(X(x, y + 1, z, a) - o - J[a][1]) > tol ||
              std::fabs(X(x, y, z + 1, a) - o - J[a][2]) > tol)
            return false;
        }
  // cofactors: adj[r][a] = (J e_{a+1} x J e_{a+2})_r = det J (J^-T)_{ra}
  double adj[3][3];
  for (int a = 0; a < 3; ++a) {
    const int p = (a + 1) % 3, q = (a + 2) % 3;
    adj[0][a] = J[1][p] * J[2][q] - J[2][p] * J[1][q];
    adj[1][a] = J[2][p] * J[0][q] - J[0][p] * J[2][q];
    adj[2][a] = J[0][p] * J[1][q] - J[1][p] * J[0][q];
  }
  const double det = J[0][0] * adj[0][0] + J[1][0] * adj[1][0] + J[2][0] * adj[2][0];
  if (!(det > 0.0)) return false;
  // G = det J^-1 J^-T = adj^T adj / det
  auto G = [&](int a, int b) { return (adj[0][a] * adj[0][b] + adj[1][a] * adj[1][b] + adj[2][a] * adj[2][b]) / det; };
  c->pG[0] = G(0, 0);
  c->pG[1] = G(1, 1);
  c->pG[2] = G(2, 2);
  c->pG[3] = G(0, 1);
  c->pG[4] = G(0, 2);
  c->pG[5] = G(1, 2);
  for (int d = 0; d < 3; ++d)
    c->parea[d] = std::sqrt(adj[0][d] * adj[0][d] + adj[1][d] * adj[1][d] + adj[2][d] * adj[2][d]);
  c->pdet = det;
  return true;
}

int dg_setup(const dg_mesh_desc* mesh, dg_ctx** out, void* stream) {
  if (!out) return fail(nullptr, DG_ERR_ARG, "out is NULL");
  *out = nullptr;
  int rc = check_desc(mesh, nullptr);
  if (rc != DG_OK) return rc;
  const Layout L = layout(mesh);
  if (!mesh->workspace) return fail(nullptr, DG_ERR_ARG, "workspace is NULL");
  if (!aligned(mesh->workspace, 256)) return fail(nullptr, DG_ERR_ARG, "workspace must be 256-byte aligned");
  if (mesh->workspace_bytes < L.total)
    return fail(nullptr, DG_ERR_ARG, "workspace too small: need " + std::to_string(L.total) + " bytes");
  dg_ctx* c = new (std::nothrow) dg_ctx();
  if (!c) return fail(nullptr, DG_ERR_ARG, "out of host memory");
  c->desc = *mesh;
  c->n = mesh->degree + 1;
  c->E = (int64_t)mesh->nx * mesh->ny * mesh->nz;
  c->ndof = c->E * c->n * c->n * c->n;
  c->trilinear = mesh->vertices != nullptr;
  char* w = (char*)mesh->workspace;
  c->tab64 = (Tables<double>*)(w + L.tab64);
  c->tab32 = (Tables<float>*)(w + L.tab32);
  c->K64 = (double*)(w + L.K64);
  c->K32 = (float*)(w + L.K32);
  c->G64 = (double*)(w + L.G64);
  c->G32 = (float*)(w + L.G32);
  c->R64 = (double*)(w + L.R64);
  c->R32 = (float*)(w + L.R32);
  c->reaction = false;
  c->affine_geom = false;
  c->ppd = false;
  c->vert64 = c->trilinear ? (double*)(w + L.vert64) : nullptr;
  c->vert32 = c->trilinear ? (float*)(w + L.vert32) : nullptr;
  c->dinv64 = (double*)(w + L.dinv64);
  c->dinv32 = (float*)(w + L.dinv32);
  c->bjQ64 = c->trilinear ? nullptr : (double*)(w + L.bjQ64);
  c->bjL64 = c->trilinear ? nullptr : (double*)(w + L.bjL64);
  c->bjQ32 = c->trilinear ? nullptr : (float*)(w + L.bjQ32);
  c->bjL32 = c->trilinear ? nullptr : (float*)(w + L.bjL32);
  c->r64 = (double*)(w + L.r64);
  c->p64 = (double*)(w + L.p64);
  c->q64 = (double*)(w + L.q64);
  c->r32 = (float*)(w + L.r32);
  c->d32 = (float*)(w + L.d32);
  c->p32 = (float*)(w + L.p32);
  c->q32 = (float*)(w + L.q32);
  c->z32 = c->trilinear ? nullptr : (float*)(w + L.z32);
  c->p16 = (uint16_t*)(w + L.p16);
  c->z64 = (double*)(w + L.z64);
  c->s64 = (double*)(w + L.s64);
  c->w64 = (double*)(w + L.w64);
  c->fb = c->trilinear ? (void*)(w + L.fb) : nullptr;
  c->partials = (double*)(w + L.partials);
  c->st = (CgState*)(w + L.st);
  c->coef_changed = (int*)(w + L.flags);
  hipStream_t s = (hipStream_t)stream;
  auto bail = [&](int code, const std::string& msg) {
    g_err = msg;
    delete c;
    return code;
  };
  Tables<double> t64;
  Tables<float> t32;
  if (!build_tables(c->n, t64)) return bail(DG_ERR_ARG, "1D table construction failed");
  tables_to_f32(t64, t32);
  hipError_t e;
#define SETUP_TRY(expr)                                                                   \
  do {                                                                                    \
    e = (expr);                                                                           \
    if (e != hipSuccess) return bail(DG_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e)); \
  } while (0)
  SETUP_TRY(scratch_address(&c->scratch));
  SETUP_TRY(hipMemcpyAsync(c->tab64, &t64, sizeof(t64), hipMemcpyHostToDevice, s));
  SETUP_TRY(hipMemcpyAsync(c->tab32, &t32, sizeof(t32), hipMemcpyHostToDevice, s));
  SETUP_TRY(hipMemsetAsync(c->st, 0, 2 * sizeof(CgState), s));
  SETUP_TRY(coef_setup(c, mesh->theta, nullptr, s));
  if (c->trilinear) {
    const int64_t nv3 = (int64_t)(mesh->nx + 1) * (mesh->ny + 1) * (mesh->nz + 1) * 3;
    SETUP_TRY(hipMemcpyAsync(c->vert64, mesh->vertices, nv3 * sizeof(double), hipMemcpyDeviceToDevice, s));
    SETUP_TRY(launch_to_f32(nv3, c->vert64, c->vert32, s));
    std::vector<double> hv((size_t)nv3);
    SETUP_TRY(hipMemcpyAsync(hv.data(), mesh->vertices, nv3 * sizeof(double), hipMemcpyDeviceToHost, s));
    SETUP_TRY(hipStreamSynchronize(s));
    c->affine_geom = all_parallelepipeds(mesh->nx, mesh->ny, mesh->nz, hv);
    c->ppd = c->affine_geom && uniform_parallelepipeds(mesh->nx, mesh->ny, mesh->nz, hv, c);
  }
  SETUP_TRY(compute_dinv(c, s));
  SETUP_TRY(hipStreamSynchronize(s));
#undef SETUP_TRY
  c->desc.vertices = nullptr;  // copied
  c->desc.theta = nullptr;
  *out = c;
  return DG_OK;
}

int dg_set_theta(dg_ctx* c, const double* theta, void* stream) {
  if (!c) return fail(nullptr, DG_ERR_ARG, "ctx is NULL");
  if (!theta) return fail(c, DG_ERR_ARG, "theta is NULL");
  hipStream_t s = (hipStream_t)stream;
  // the diagonal kernels skip their work on the device when no K_T changed
  // (an autograd backward sets the same theta as its forward)
  HIP_TRY(c, coef_setup(c, theta, c->coef_changed, s));
  HIP_TRY(c, compute_dinv(c, s, c->coef_changed));
  return DG_OK;
}

int dg_set_reaction(dg_ctx* c, const double* r, void* stream) {
  if (!c) return fail(nullptr, DG_ERR_ARG, "ctx is NULL");
  if (r && !aligned(r, 8)) return fail(c, DG_ERR_ARG, "misaligned reaction coefficients");
  hipStream_t s = (hipStream_t)stream;
  if (r) {
    HIP_TRY(c, hipMemcpyAsync(c->R64, r, c->E * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(c, launch_to_f32(c->E, c->R64, c->R32, s));
  }
  c->reaction = r != nullptr;
  HIP_TRY(c, compute_dinv(c, s));
  return DG_OK;
}

static int apply_common(dg_ctx* c, int prec, int trans, const void* x, void* y, void* stream) {
  if (!c) return fail(nullptr, DG_ERR_ARG, "ctx is NULL");
  if (!x || !y) return fail(c, DG_ERR_ARG, "x or y is NULL");
  if (x == y) return fail(c, DG_ERR_ARG, "x and y must not alias");
  if (prec != DG_F64 && prec != DG_F32 && prec != DG_BF16 && prec != DG_BF16_MFMA)
    return fail(c, DG_ERR_UNSUPPORTED, "unknown precision");
  if (prec == DG_BF16_MFMA && (c->trilinear || !mfma_apply_supported(c->n)))
    return fail(c, DG_ERR_UNSUPPORTED, "DG_BF16_MFMA needs an affine mesh and degree <= 4");
  const size_t ein = prec == DG_F64 ? 8 : (prec == DG_F32 ? 4 : 2);
  const size_t eout = prec == DG_F64 ? 8 : 4;
  if (!aligned(x, ein) || !aligned(y, eout)) return fail(c, DG_ERR_ARG, "misaligned x or y");
  // overlap of the two ranges is aliasing too
  const char* xb = (const char*)x;
  const char* yb = (const char*)y;
  if (xb < yb + c->ndof * eout && yb < xb + c->ndof * ein) return fail(c, DG_ERR_ARG, "x and y overlap");
  HIP_TRY(c, apply_any(c, prec, trans, 0, x, y, nullptr, 0, nullptr, (hipStream_t)stream));
  return DG_OK;
}

int dg_apply(dg_ctx* c, int prec, const void* x, void* y, void* stream) {
  return apply_common(c, prec, 0, x, y, stream);
}
int dg_apply_transpose(dg_ctx* c, int prec, const void* x, void* y, void* stream) {
  return apply_common(c, prec, 1, x, y, stream);
}

int dg_apply_multi(dg_ctx* c, int prec, int transpose, int nrhs, const void* X, void* Y, void* stream) {
  if (!c) return fail(nullptr, DG_ERR_ARG, "ctx is NULL");
  if (!X || !Y) return fail(c, DG_ERR_ARG, "X or Y is NULL");
  if (nrhs < 1 || nrhs > 65535) return fail(c, DG_ERR_ARG, "nrhs must be in 1..65535");
  if (transpose != 0 && transpose != 1) return fail(c, DG_ERR_ARG, "transpose must be 0 or 1");
  if (prec != DG_F64 && prec != DG_F32 && prec != DG_BF16 && prec != DG_BF16_MFMA)
    return fail(c, DG_ERR_UNSUPPORTED, "unknown precision");
  if (prec == DG_BF16_MFMA && (c->trilinear || !mfma_apply_supported(c->n)))
    return fail(c, DG_ERR_UNSUPPORTED, "DG_BF16_MFMA needs an affine mesh and degree <= 4");
  const size_t ein = prec == DG_F64 ? 8 : (prec == DG_F32 ? 4 : 2);
  const size_t eout = prec == DG_F64 ? 8 : 4;
  if (!aligned(X, ein) || !aligned(Y, eout)) return fail(c, DG_ERR_ARG, "misaligned X or Y");
  const char* xb = (const char*)X;
  const char* yb = (const char*)Y;
  const size_t tot = (size_t)nrhs * (size_t)c->ndof;
  if (xb < yb + tot * eout && yb < xb + tot * ein) return fail(c, DG_ERR_ARG, "X and Y overlap");
  hipStream_t s = (hipStream_t)stream;
  if (c->ppd) {  // the form is symmetric: the transpose is the same operator
    HIP_TRY(c, launch_apply_ppd_multi(c->n, prec, nrhs, ppd_args(c, args64(c)), ppd_args(c, args32(c)), X, Y, s));
    return DG_OK;
  }
  if (c->trilinear) {  // the two-pass apply shares its face buffer: one vector after the other
    for (int j = 0; j < nrhs; ++j)
      HIP_TRY(c, apply_any(c, prec, transpose, 0, xb + (size_t)j * c->ndof * ein, (char*)Y + (size_t)j * c->ndof * eout,
                           nullptr, 0, nullptr, s));
    return DG_OK;
  }
  HIP_TRY(c, launch_apply_affine_multi(c->n, prec, transpose, nrhs, args64(c), args32(c), X, Y, s));
  return DG_OK;
}

int dg_dA_dtheta(dg_ctx* c, const double* u, const double* v, double* g, void* stream) {
  if (!c) return fail(nullptr, DG_ERR_ARG, "ctx is NULL");
  if (!u || !v || !g) return fail(c, DG_ERR_ARG, "u, v or g is NULL");
  if (c->trilinear)  // the 7 per-element parts go to the FP64 CG work vector r (7 E <= N_dof)
    HIP_TRY(c, launch_dA_trilinear(c->n, args64(c), u, v, c->r64, g, (hipStream_t)stream));
  else
    HIP_TRY(c, launch_dA_affine(c->n, args64(c), u, v, g, (hipStream_t)stream));
  return DG_OK;
}

int dg_dA_dtheta_noalloc(dg_ctx* c, const double* u, const double* v, double* g, void* stream) {
  if (!c) return fail(nullptr, DG_ERR_ARG, "ctx is NULL");
  if (!u || !v || !g) return fail(c, DG_ERR_ARG, "u, v or g is NULL");
  if (c->trilinear) {  // the 7 per-element parts go to this device's static scratch array
    if ((size_t)c->E * 7 * sizeof(double) > kScratchBytes)
      return fail(c, DG_ERR_ARG, "mesh too large for dg_dA_dtheta_noalloc: at most " +
                                     std::to_string(kScratchBytes / (7 * sizeof(double))) + " elements");
    HIP_TRY(c, launch_dA_trilinear(c->n, args64(c), u, v, c->scratch, g, (hipStream_t)stream));
  } else {
    HIP_TRY(c, launch_dA_affine(c->n, args64(c), u, v, g, (hipStream_t)stream));
  }
  return DG_OK;
}

int dg_diagonal(dg_ctx* c, double* d, void* stream) {
  if (!c) return fail(nullptr, DG_ERR_ARG, "ctx is NULL");
  if (!d) return fail(c, DG_ERR_ARG, "d is NULL");
  const MeshArgs<double> m64 = args64(c);
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(c, c->trilinear ? launch_diag_trilinear(c->n, m64, d, nullptr, s)
                          : launch_diag_affine(c->n, m64, d, nullptr, s));
  return DG_OK;
}

int dg_quadrature_points(dg_ctx* c, double* xq, void* stream) {
  if (!c) return fail(nullptr, DG_ERR_ARG, "ctx is NULL");
  if (!xq) return fail(c, DG_ERR_ARG, "xq is NULL");
  HIP_TRY(c, launch_quad_points(c->n, args64(c), xq, (hipStream_t)stream));
  return DG_OK;
}

int dg_load_vector(dg_ctx* c, const double* fq, double* b, void* stream) {
  if (!c) return fail(nullptr, DG_ERR_ARG, "ctx is NULL");
  if (!fq || !b) return fail(c, DG_ERR_ARG, "fq or b is NULL");
  if (fq == b) return fail(c, DG_ERR_ARG, "fq and b must not alias");
  HIP_TRY(c, launch_load_vector(c->n, args64(c), fq, b, (hipStream_t)stream));
  return DG_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ solvers
namespace {

struct HostState {
  int done, breakdown, iters;
  double rr, bb;
};

int read_state(dg_ctx* c, int which, CgState& hs, hipStream_t s) {
  HIP_TRY(c, hipMemcpyAsync(&hs, &c->st[which], sizeof(CgState), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  return DG_OK;
}

// FP64 PCG (Alg. PCG) on x; returns iterations and sets breakdown.
int pcg64(dg_ctx* c, const dg_cg_opts* o, const double* b, double* x, int maxit, int& iters, bool& broke,
          hipStream_t s) {
  const int64_t n = c->ndof;
  const double* dinv = o->precond == DG_PC_JACOBI ? c->dinv64 : nullptr;
  CgState* st = &c->st[0];
  const int check = o->check_every > 0 ? o->check_every : 32;
  HIP_TRY(c, apply_any(c, DG_F64, o->transpose, 0, x, c->q64, nullptr, 0, nullptr, s));
  HIP_TRY(c, (launch_cg_init<double, double, double, double>(n, b, c->q64, c->r64, c->p64, dinv, o->rtol, st,
                                                            c->partials, s)));
  CgState hs;
  int rc = read_state(c, 0, hs, s);
  if (rc != DG_OK) return rc;
  // few block partials: the update kernels sum them themselves (no finish kernels)
  const int64_t nbA = apply_partials(c);
  const bool fused = nbA <= 4096 && 2 * vec_blocks(n) <= 8192;
  double* partA = c->partials;
  double* partB = c->partials + nbA;
  int it = 0;
  while (!hs.done && it < maxit) {
    const int chunk = std::min(check, maxit - it);
    for (int j = 0; j < chunk; ++j, ++it) {
      const int par = it & 1;
      if (fused) {
        HIP_TRY(c, apply_any(c, DG_F64, o->transpose, 1, c->p64, c->q64, nullptr, 0, &st->done, s, partA));
        HIP_TRY(c, (launch_cg_update_fused<double, double>(n, c->r64, c->q64, dinv, par, st, partA, nbA, partB, s)));
        HIP_TRY(c, (launch_cg_pupdate_fused<double, double, double, double>(n, x, c->r64, c->p64, dinv, par, st, partB,
                                                                            s)));
        continue;
      }
      HIP_TRY(c, apply_any(c, DG_F64, o->transpose, 1, c->p64, c->q64, st, par, &st->done, s));
      HIP_TRY(c, (launch_cg_update<double, double>(n, c->r64, c->q64, dinv, par, st, c->partials, s)));
      HIP_TRY(c, (launch_cg_pupdate<double, double, double, double>(n, x, c->r64, c->p64, dinv, par, st, 0, s)));
    }
    rc = read_state(c, 0, hs, s);
    if (rc != DG_OK) return rc;
  }
  iters = hs.iters;
  broke = hs.breakdown != 0;
  return DG_OK;
}

// FP64 PCG (Alg. PCG) with the element block-Jacobi preconditioner: z = P r
// is an element-local kernel of its own (fast diagonalisation), so each
// iteration runs the apply (with <p, q>), r -= lambda q (with <r, r>), z = P r
// (with <z, r>) and x += lambda p, p = z + beta p, where the last kernel reads
// z in place of the Jacobi-scaled residual.
int pcg64_block(dg_ctx* c, const dg_cg_opts* o, const double* b, double* x, int maxit, int& iters, bool& broke,
                hipStream_t s) {
  const int64_t n = c->ndof;
  CgState* st = &c->st[0];
  const int check = o->check_every > 0 ? o->check_every : 32;
  const int64_t nbj = element_blocks(c->n, c->E);
  HIP_TRY(c, apply_any(c, DG_F64, o->transpose, 0, x, c->q64, nullptr, 0, nullptr, s));
  // r = b - A x, <r, r>, <b, b> (z64 receives r and is overwritten below)
  HIP_TRY(c, (launch_cg_init<double, double, double, double>(n, b, c->q64, c->r64, c->z64, nullptr, o->rtol, st,
                                                            c->partials, s)));
  HIP_TRY(c, (launch_bj_apply<double, double>(c->n, c->E, c->bjQ64, c->bjL64, c->r64, c->z64, c->partials,
                                              &st->done, s)));
  HIP_TRY(c, launch_bj_finish(c->partials, nbj, st, 0, s));
  HIP_TRY(c, hipMemcpyAsync(c->p64, c->z64, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  CgState hs;
  int rc = read_state(c, 0, hs, s);
  if (rc != DG_OK) return rc;
  // few block partials: the block apply and the direction update sum them
  // themselves (no finish kernels)
  const int64_t nbA = apply_partials(c);
  const bool fused = nbA <= 4096 && nbj <= 4096;
  double* partA = c->partials;
  double* partB = c->partials + nbA;
  int it = 0;
  while (!hs.done && it < maxit) {
    const int chunk = std::min(check, maxit - it);
    for (int j = 0; j < chunk; ++j, ++it) {
      const int par = it & 1;
      if (fused) {
        HIP_TRY(c, apply_any(c, DG_F64, o->transpose, 1, c->p64, c->q64, nullptr, 0, &st->done, s, partA));
        HIP_TRY(c, (launch_bj_apply<double, double>(c->n, c->E, c->bjQ64, c->bjL64, c->r64, c->z64, partB, nullptr, s,
                                                    c->q64, st, par, partA, nbA)));
        HIP_TRY(c, (launch_cg_pupdate_fused<double, double, double, double>(n, x, c->z64, c->p64, nullptr, par, st,
                                                                            partB, s, nbj)));
        continue;
      }
      HIP_TRY(c, apply_any(c, DG_F64, o->transpose, 1, c->p64, c->q64, st, par, &st->done, s));
      // r -= lambda q and z = P r in one element pass, then FIN_UPDATE on {<z, r>, <r, r>}
      HIP_TRY(c, (launch_bj_apply<double, double>(c->n, c->E, c->bjQ64, c->bjL64, c->r64, c->z64, c->partials,
                                                  &st->done, s, c->q64, st, par)));
      HIP_TRY(c, launch_update_finish(c->partials, nbj, st, par, s));
      HIP_TRY(c, (launch_cg_pupdate<double, double, double, double>(n, x, c->z64, c->p64, nullptr, par, st, 0, s)));
    }
    rc = read_state(c, 0, hs, s);
    if (rc != DG_OK) return rc;
  }
  iters = hs.iters;
  broke = hs.breakdown != 0;
  return DG_OK;
}

// Single-reduction PCG in FP64 (Chronopoulos-Gear recurrences): per iteration
// one fused vector kernel, the apply w = A z with <z, w>, and one finish over
// both partial sets (the other sums of Alg. PCG are carried by recurrences).
int pcg64_single(dg_ctx* c, const dg_cg_opts* o, const double* b, double* x, int maxit, int& iters, bool& broke,
                 hipStream_t s) {
  const int64_t n = c->ndof;
  const double* dinv = o->precond == DG_PC_JACOBI ? c->dinv64 : nullptr;
  CgState* st = &c->st[0];
  const int check = o->check_every > 0 ? o->check_every : 32;
  const int64_t nvb = vec_blocks(n);
  double* partA = c->partials;             // <r, z>, <r, r> of the update (2 per vector block)
  double* partB = c->partials + 2 * nvb;   // <z, w> of the apply
  const int64_t nbB = apply_partials(c);
  HIP_TRY(c, apply_any(c, DG_F64, o->transpose, 0, x, c->q64, nullptr, 0, nullptr, s));
  // r = b - A x0, z = Dinv r (into z), gamma = <r, z>, <r, r>, <b, b>
  HIP_TRY(c, (launch_cg_init<double, double, double, double>(n, b, c->q64, c->r64, c->z64, dinv, o->rtol, st,
                                                            c->partials, s)));
  HIP_TRY(c, hipMemsetAsync(c->p64, 0, n * sizeof(double), s));
  HIP_TRY(c, hipMemsetAsync(c->s64, 0, n * sizeof(double), s));
  HIP_TRY(c, apply_any(c, DG_F64, o->transpose, 1, c->z64, c->w64, nullptr, 0, &st->done, s, partB));
  HIP_TRY(c, launch_cg2_finish(partA, nvb, partB, nbB, st, 0, s));
  CgState hs;
  int rc = read_state(c, 0, hs, s);
  if (rc != DG_OK) return rc;
  int it = 0;
  while (!hs.done && it < maxit) {
    const int chunk = std::min(check, maxit - it);
    for (int j = 0; j < chunk; ++j, ++it) {
      HIP_TRY(c, launch_cg2_update(n, x, c->r64, c->z64, c->p64, c->s64, c->w64, dinv, st, partA, s));
      HIP_TRY(c, apply_any(c, DG_F64, o->transpose, 1, c->z64, c->w64, nullptr, 0, &st->done, s, partB));
      HIP_TRY(c, launch_cg2_finish(partA, nvb, partB, nbB, st, 1, s));
    }
    rc = read_state(c, 0, hs, s);
    if (rc != DG_OK) return rc;
  }
  iters = hs.iters;
  broke = hs.breakdown != 0;
  return DG_OK;
}

int true_residual(dg_ctx* c, int transpose, const double* b, const double* x, double& rel, hipStream_t s) {
  HIP_TRY(c, apply_any(c, DG_F64, transpose, 0, x, c->q64, nullptr, 0, nullptr, s));
  HIP_TRY(c, launch_resid_norm(c->ndof, b, c->q64, &c->st[0], c->partials, s));
  CgState hs;
  int rc = read_state(c, 0, hs, s);
  if (rc != DG_OK) return rc;
  rel = hs.true_bb > 0 ? std::sqrt(hs.true_rr / hs.true_bb) : std::sqrt(hs.true_rr);
  return DG_OK;
}

// Inner PCG on FP32 vectors for A_lo d = r32 (TP = float or bf16 direction).
// fresh: start from d = 0, p = z (init kernel, stop at inner_rtol ||r||);
// otherwise continue from the state left by a residual replacement, whose
// iteration parity is par0.  Returns iterations and the parity of the last
// completed iteration.
template <typename TP>
int pcg_inner(dg_ctx* c, const dg_cg_opts* o, int prec, bool fresh, double inner_rtol, int par0, int maxit,
              int& iters, int& last_par, bool& broke, hipStream_t s) {
  const int64_t n = c->ndof;
  const float* dinv = o->precond == DG_PC_JACOBI ? c->dinv32 : nullptr;
  const bool blk = o->precond == DG_PC_BLOCK_JACOBI;
  CgState* st = &c->st[1];
  TP* p = prec != DG_F32 ? (TP*)c->p16 : (TP*)c->p32;
  const int check = o->check_every > 0 ? o->check_every : 32;
  const int64_t nbj = element_blocks(c->n, c->E);
  if (fresh) {
    par0 = 0;
    if (blk) {  // z = P r with {<z, r>, <r, r>}, then p = z, d = 0
      HIP_TRY(c, (launch_bj_apply<float, float>(c->n, c->E, c->bjQ32, c->bjL32, c->r32, c->z32, c->partials, nullptr,
                                                s)));
      HIP_TRY(c, launch_init_inner_finish(c->partials, nbj, st, inner_rtol, s));
      HIP_TRY(c, launch_inner_start<TP>(n, c->z32, c->d32, p, st, s));
    } else {
      HIP_TRY(c, (launch_cg_init_inner<float, TP, float>(n, c->r32, c->d32, p, dinv, inner_rtol, st, c->partials,
                                                         s)));
    }
  }
  CgState hs;
  int rc = read_state(c, 1, hs, s);
  if (rc != DG_OK) return rc;
  // few block partials: the update kernels sum them themselves (no finish kernels)
  const int64_t nbA = apply_partials(c);
  const bool fused = !blk && nbA <= 4096 && 2 * vec_blocks(n) <= 8192;
  const bool fused_blk = blk && nbA <= 4096 && nbj <= 4096;
  double* partA = c->partials;
  double* partB = c->partials + nbA;
  int it = 0;
  while (!hs.done && it < maxit) {
    const int chunk = std::min(check, maxit - it);
    for (int j = 0; j < chunk; ++j, ++it) {
      const int par = (par0 + it) & 1;
      if (fused_blk) {  // as pcg64_block, on the FP32 inner vectors
        HIP_TRY(c, apply_any(c, prec, o->transpose, 1, p, c->q32, nullptr, 0, &st->done, s, partA));
        HIP_TRY(c, (launch_bj_apply<float, float>(c->n, c->E, c->bjQ32, c->bjL32, c->r32, c->z32, partB, nullptr, s,
                                                  c->q32, st, par, partA, nbA)));
        HIP_TRY(c, (launch_cg_pupdate_fused<float, float, TP, float>(n, c->d32, c->z32, p, nullptr, par, st, partB, s,
                                                                     nbj)));
        continue;
      }
      if (blk) {  // as pcg64_block, on the FP32 inner vectors
        HIP_TRY(c, apply_any(c, prec, o->transpose, 1, p, c->q32, st, par, &st->done, s));
        HIP_TRY(c, (launch_bj_apply<float, float>(c->n, c->E, c->bjQ32, c->bjL32, c->r32, c->z32, c->partials,
                                                  &st->done, s, c->q32, st, par)));
        HIP_TRY(c, launch_update_finish(c->partials, nbj, st, par, s));
        HIP_TRY(c, (launch_cg_pupdate<float, float, TP, float>(n, c->d32, c->z32, p, nullptr, par, st, 0, s)));
        continue;
      }
      if (fused) {
        HIP_TRY(c, apply_any(c, prec, o->transpose, 1, p, c->q32, nullptr, 0, &st->done, s, partA));
        HIP_TRY(c, (launch_cg_update_fused<float, float>(n, c->r32, c->q32, dinv, par, st, partA, nbA, partB, s)));
        HIP_TRY(c, (launch_cg_pupdate_fused<float, float, TP, float>(n, c->d32, c->r32, p, dinv, par, st, partB, s)));
        continue;
      }
      HIP_TRY(c, apply_any(c, prec, o->transpose, 1, p, c->q32, st, par, &st->done, s));
      HIP_TRY(c, (launch_cg_update<float, float>(n, c->r32, c->q32, dinv, par, st, c->partials, s)));
      HIP_TRY(c, (launch_cg_pupdate<float, float, TP, float>(n, c->d32, c->r32, p, dinv, par, st, 0, s)));
    }
    rc = read_state(c, 1, hs, s);
    if (rc != DG_OK) return rc;
  }
  iters = hs.iters;
  last_par = (par0 + hs.iters - 1) & 1;
  broke = hs.breakdown != 0;
  return DG_OK;
}

// FP64 defect correction around the FP32-vector inner PCG.
// DG_DC_RESTART: every correction is a fresh inner solve to inner_rtol.
// DG_DC_KEEP: an inner segment stops at an inner_rtol reduction of its
// residual; x += d, the FP64 residual replaces the inner one, and CG goes on
// along the old direction p (p = z + beta p with the replaced residual).
template <typename TP>
int dc_solve(dg_ctx* c, const dg_cg_opts* o, int prec, const double* b, double* x, int& total, int& outer,
             bool& broke, double& rel, hipStream_t s) {
  const bool keep = o->dc_mode == DG_DC_KEEP;
  const double tin = o->inner_rtol > 0 ? o->inner_rtol
                                       : (keep ? 0.1 : (prec == DG_F32 ? 1e-5 : 1e-2));
  const int max_outer = o->max_outer > 0 ? o->max_outer : (keep ? 200 : 30);
  const float* dinv = o->precond == DG_PC_JACOBI ? c->dinv32 : nullptr;
  TP* p = prec != DG_F32 ? (TP*)c->p16 : (TP*)c->p32;
  bool fresh = true;
  int last_par = 0;
  int rc;
  // first residual
  HIP_TRY(c, apply_any(c, DG_F64, o->transpose, 0, x, c->q64, nullptr, 0, nullptr, s));
  HIP_TRY(c, launch_dc_residual(c->ndof, b, c->q64, c->r32, &c->st[0], c->partials, s));
  CgState hs;
  rc = read_state(c, 0, hs, s);
  if (rc != DG_OK) return rc;
  rel = hs.bb > 0 ? std::sqrt(hs.rr / hs.bb) : std::sqrt(hs.rr);
  for (;;) {
    if (!(rel == rel)) {
      broke = true;
      break;
    }
    if (rel <= o->rtol || outer >= max_outer || total >= o->maxit) break;
    int its = 0;
    bool ib = false;
    rc = pcg_inner<TP>(c, o, prec, fresh, tin, (last_par + 1) & 1, o->maxit - total, its, last_par, ib, s);
    if (rc != DG_OK) return rc;
    total += its;
    HIP_TRY(c, launch_dc_update(c->ndof, x, c->d32, s));
    ++outer;
    if (ib && its == 0) {
      broke = true;
      break;
    }
    HIP_TRY(c, apply_any(c, DG_F64, o->transpose, 0, x, c->q64, nullptr, 0, nullptr, s));
    if (keep && !ib && its > 0) {
      // replace the residual, keep the direction
      HIP_TRY(c, launch_dc_replace(c->ndof, b, c->q64, dinv, c->r32, &c->st[1], last_par, o->rtol, tin,
                                   c->partials, s));
      if (o->precond == DG_PC_BLOCK_JACOBI) {  // rho of the kept direction from z = P r
        HIP_TRY(c, (launch_bj_apply<float, float>(c->n, c->E, c->bjQ32, c->bjL32, c->r32, c->z32, c->partials,
                                                  &c->st[1].done, s)));
        HIP_TRY(c, launch_bj_finish(c->partials, element_blocks(c->n, c->E), &c->st[1], last_par ^ 1, s));
      }
      rc = read_state(c, 1, hs, s);
      if (rc != DG_OK) return rc;
      rel = hs.true_bb > 0 ? std::sqrt(hs.true_rr / hs.true_bb) : std::sqrt(hs.true_rr);
      if (hs.breakdown) {
        fresh = true;  // r32 holds the new residual; fall back to a fresh direction
        continue;
      }
      if (rel <= o->rtol) break;
      HIP_TRY(c, (launch_cg_pupdate<float, float, TP, float>(
                     c->ndof, c->d32, o->precond == DG_PC_BLOCK_JACOBI ? c->z32 : c->r32, p, dinv, last_par,
                     &c->st[1], 1, s)));
      fresh = false;
    } else {
      HIP_TRY(c, launch_dc_residual(c->ndof, b, c->q64, c->r32, &c->st[0], c->partials, s));
      rc = read_state(c, 0, hs, s);
      if (rc != DG_OK) return rc;
      rel = hs.bb > 0 ? std::sqrt(hs.rr / hs.bb) : std::sqrt(hs.rr);
      fresh = true;
    }
  }
  return DG_OK;
}

}  // namespace

extern "C" {

int dg_cg_solve(dg_ctx* c, const dg_cg_opts* o, const double* b, double* x, dg_cg_info* info, void* stream) {
  if (!c) return fail(nullptr, DG_ERR_ARG, "ctx is NULL");
  if (!o || !b || !x || !info) return fail(c, DG_ERR_ARG, "opts, b, x or info is NULL");
  if (b == x) return fail(c, DG_ERR_ARG, "b and x must not alias");
  if (o->prec_inner != DG_F64 && o->prec_inner != DG_F32 && o->prec_inner != DG_BF16 &&
      o->prec_inner != DG_BF16_MFMA)
    return fail(c, DG_ERR_UNSUPPORTED, "unknown inner precision");
  if (o->prec_inner == DG_BF16_MFMA && (c->trilinear || !mfma_apply_supported(c->n)))
    return fail(c, DG_ERR_UNSUPPORTED, "DG_BF16_MFMA needs an affine mesh and degree <= 4");
  if (o->precond != DG_PC_NONE && o->precond != DG_PC_JACOBI && o->precond != DG_PC_BLOCK_JACOBI)
    return fail(c, DG_ERR_ARG, "unknown preconditioner");
  if (o->precond == DG_PC_BLOCK_JACOBI && (c->trilinear || o->cg_variant != DG_CG_STANDARD))
    return fail(c, DG_ERR_UNSUPPORTED, "block-Jacobi is built for the standard CG variant on affine meshes");
  if (o->dc_mode != DG_DC_RESTART && o->dc_mode != DG_DC_KEEP) return fail(c, DG_ERR_ARG, "unknown dc_mode");
  if (o->cg_variant != DG_CG_STANDARD && o->cg_variant != DG_CG_SINGLE_REDUCTION)
    return fail(c, DG_ERR_ARG, "unknown cg_variant");
  if (o->cg_variant == DG_CG_SINGLE_REDUCTION && o->prec_inner != DG_F64)
    return fail(c, DG_ERR_UNSUPPORTED, "the single-reduction variant is built for FP64 solves only");
  if (!(o->rtol > 0) || o->maxit < 1) return fail(c, DG_ERR_ARG, "rtol must be > 0 and maxit >= 1");
  if (!aligned(b, 8) || !aligned(x, 8)) return fail(c, DG_ERR_ARG, "misaligned b or x");
  hipStream_t s = (hipStream_t)stream;
  const auto t0 = std::chrono::steady_clock::now();
  std::memset(info, 0, sizeof(*info));
  int total = 0;
  bool broke = false;
  double rel = 0.0;
  int rc;
  if (o->prec_inner == DG_F64) {
    // PCG to the recursive criterion, confirmed by the true FP64 residual;
    // restarted from the current iterate if the check fails
    for (int attempt = 0;; ++attempt) {
      int its = 0;
      rc = o->cg_variant == DG_CG_SINGLE_REDUCTION ? pcg64_single(c, o, b, x, o->maxit - total, its, broke, s)
           : o->precond == DG_PC_BLOCK_JACOBI    ? pcg64_block(c, o, b, x, o->maxit - total, its, broke, s)
                                                 : pcg64(c, o, b, x, o->maxit - total, its, broke, s);
      if (rc != DG_OK) return rc;
      total += its;
      rc = true_residual(c, o->transpose, b, x, rel, s);
      if (rc != DG_OK) return rc;
      if (rel <= o->rtol || broke || total >= o->maxit || attempt >= 10) break;
      info->restarts++;
    }
  } else {
    int outer = 0;
    rc = o->prec_inner == DG_F32 ? dc_solve<float>(c, o, DG_F32, b, x, total, outer, broke, rel, s)
                                 : dc_solve<uint16_t>(c, o, o->prec_inner, b, x, total, outer, broke, rel, s);
    if (rc != DG_OK) return rc;
    info->outer_iters = outer;
  }
  HIP_TRY(c, hipStreamSynchronize(s));
  info->iters = total;
  info->rel_true_residual = rel;
  info->status = rel <= o->rtol ? DG_OK : (broke ? DG_BREAKDOWN : DG_NOT_CONVERGED);
  info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return info->status;
}

int64_t dg_num_dofs(const dg_ctx* c) { return c ? c->ndof : -1; }
int64_t dg_num_elements(const dg_ctx* c) { return c ? c->E : -1; }
int dg_nodes_per_dir(const dg_ctx* c) { return c ? c->n : -1; }
int dg_apply_kernel(const dg_ctx* c) {
  if (!c) return -1;
  return c->ppd ? DG_KERNEL_PARALLELEPIPED : (c->trilinear ? DG_KERNEL_TRILINEAR : DG_KERNEL_AFFINE);
}

void dg_destroy(dg_ctx* c) { delete c; }

const char* dg_last_error(const dg_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

}  // extern "C"
