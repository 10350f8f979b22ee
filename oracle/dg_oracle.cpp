/*
 * dg_oracle.cpp -- plain CPU oracle for the SWIPDG diffusion operator.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg load this library.  It shares no
 * code, header, table or constant generator with the GPU library; both sides
 * only receive the same seeded input arrays.
 *
 * What it computes, by brute force and in FP64 throughout:
 *
 *   A_ij = b_h(phi_j, phi_i)
 *
 * the symmetric weighted interior-penalty bilinear form of Sec. 4.1
 * ("Continuous problem and discretization": b_h = sum of element integrals of
 * A grad v . grad w plus the face coupling forms b_h^e) for -div(K grad u) = f,
 * on an nx*ny*nz hexahedral mesh of the unit cube with trilinear element maps,
 * a tensor-product Q_k Lagrange basis on Gauss-Lobatto nodes and a scalar
 * coefficient K_T = exp(theta_T) per element, optionally plus a reaction term
 * int c_T u v with a coefficient c_T per element (the diffusion-reaction
 * problems whose operator throughput Sec. 3.3 reports).  The operator
 * application of Sec. 3.3 computes exactly this matrix-vector product without
 * the matrix.
 *
 * Readings taken where the printed form is silent or garbled (each is listed
 * with its justification in the design notes of the repository):
 *   - consistency terms carry a minus sign, [w] = w^- - w^+, n_e points from
 *     T^- (lower index along the face normal) to T^+;
 *   - weighted average / penalty of SWIPDG: (gamma/2)(grad u^- + grad u^+).n
 *     with gamma = 2 K^- K^+ / (K^- + K^+), penalty sigma_e * gamma;
 *   - sigma_e = sigma_hat / h_d, h_d = 1/n_d (nominal spacing normal to the
 *     face), sigma_hat = 2 (k+1)^2 unless given;
 *   - boundary faces (weak Dirichlet u = g): -K grad u.n v - K grad v.n u
 *     + sigma K u v, outward n; periodic meshes wrap in all three directions;
 *   - quadrature: (k+1+quad_extra)-point Gauss-Legendre per direction on
 *     volumes and faces.
 *
 * Every routine below evaluates the definition directly: basis functions by
 * the Lagrange product formula, the element map and its Jacobian from the 8
 * vertices, local matrices by summing over quadrature points, then scatter.
 * There is no sum factorisation, no blocking and no reuse beyond that.
 */
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

extern "C" {
typedef struct {
  int32_t nx, ny, nz;      /* elements per direction                             */
  int32_t degree;          /* polynomial degree k >= 1                           */
  int32_t bc;              /* 0: weak Dirichlet on all boundary faces, 1: periodic */
  int32_t quad_extra;      /* Gauss points per direction = k + 1 + quad_extra     */
  int32_t mutation;        /* 0; >0 plants a known mistake (pin-sensitivity tests) */
  int32_t pad_;
  double penalty_hat;      /* sigma * h_d; <= 0 selects 2 (k+1)^2                */
  const double* vertices;  /* (nx+1)(ny+1)(nz+1) x 3, x-index fastest; NULL: uniform */
  const double* theta;     /* nx*ny*nz, K = exp(theta); NULL: K = 1              */
  const double* reaction;  /* nx*ny*nz reaction coefficients c_T; NULL: none     */
} oracle_mesh;
}

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

/* Planted mistakes.  They exist only so that tests can show that each pin
 * catches a plausible error in this file; production of expected values never
 * sets them. */
enum {
  MUT_NONE = 0,
  MUT_PLUS_CONSISTENCY = 1,   /* '+' in front of both consistency terms      */
  MUT_NO_SYMMETRY = 2,        /* drop -(gamma/2) grad v.n [u]                 */
  MUT_NO_PENALTY = 3,         /* sigma = 0                                    */
  MUT_NO_BOUNDARY = 4,        /* skip the boundary faces                      */
  MUT_JINV_NOT_TRANSPOSED = 5,/* grad phi = J^{-1} ghat instead of J^{-T} ghat */
  MUT_ARITH_GAMMA = 6,        /* gamma = (K^- + K^+)/2                        */
  MUT_PENALTY_NO_AREA = 7,    /* penalty integrand without the area element   */
  MUT_PLUS_SIDE_AT_ONE = 8,   /* T^+ evaluated at xi_d = 1 instead of 0        */
};

/* ------------------------------------------------------------------------ */
/* 1D tables                                                                 */
/* ------------------------------------------------------------------------ */

/* Legendre P_m and its derivative on (-1,1) by the three-term recurrence. */
void legendre(int m, double x, double& p, double& dp) {
  double pm1 = 1.0, pc = x;
  if (m == 0) { p = 1.0; dp = 0.0; return; }
  for (int j = 2; j <= m; ++j) {
    double pn = ((2.0 * j - 1.0) * x * pc - (j - 1.0) * pm1) / j;
    pm1 = pc;
    pc = pn;
  }
  p = pc;
  dp = m * (pm1 - x * pc) / (1.0 - x * x);  /* (1-x^2) P_m' = m (P_{m-1} - x P_m) */
}

/* q-point Gauss-Legendre rule mapped to [0,1]: Newton on the roots of P_q. */
void gauss_rule(int q, std::vector<double>& x01, std::vector<double>& w01) {
  x01.assign(q, 0.0);
  w01.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    double x = std::cos(kPi * (i + 0.75) / (q + 0.5)), p, dp;
    for (int it = 0; it < 100; ++it) {
      legendre(q, x, p, dp);
      double dx = p / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    legendre(q, x, p, dp);
    double w = 2.0 / ((1.0 - x * x) * dp * dp);
    x01[i] = 0.5 * (1.0 - x);  /* cos(...) decreases with i, so this increases */
    w01[i] = 0.5 * w;
  }
}

/* n Gauss-Lobatto nodes on [0,1]: the endpoints and the roots of P_k', k = n-1.
 * Newton on P_k' with P_k'' from Legendre's equation
 * (1-x^2) P'' = 2 x P' - k (k+1) P. */
void gll_nodes(int n, std::vector<double>& xi) {
  const int k = n - 1;
  xi.assign(n, 0.0);
  xi[0] = 0.0;
  xi[n - 1] = 1.0;
  for (int i = 1; i < k; ++i) {
    double x = -std::cos(kPi * i / k), p, dp;
    for (int it = 0; it < 100; ++it) {
      legendre(k, x, p, dp);
      double d2p = (2.0 * x * dp - k * (k + 1.0) * p) / (1.0 - x * x);
      double dx = dp / d2p;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    xi[i] = 0.5 * (1.0 + x);
  }
}

/* Lagrange basis on the nodes xi: value and derivative by the product formula. */
double lagrange(const std::vector<double>& xi, int i, double x) {
  double v = 1.0;
  for (size_t j = 0; j < xi.size(); ++j)
    if ((int)j != i) v *= (x - xi[j]) / (xi[i] - xi[j]);
  return v;
}
double lagrange_d(const std::vector<double>& xi, int i, double x) {
  double s = 0.0;
  for (size_t m = 0; m < xi.size(); ++m) {
    if ((int)m == i) continue;
    double t = 1.0 / (xi[i] - xi[m]);
    for (size_t j = 0; j < xi.size(); ++j)
      if ((int)j != i && j != m) t *= (x - xi[j]) / (xi[i] - xi[j]);
    s += t;
  }
  return s;
}

/* ------------------------------------------------------------------------ */
/* Mesh, geometry, basis                                                     */
/* ------------------------------------------------------------------------ */

struct Mesh {
  int N[3];
  int k, n, n3, nq;
  int bc, mutation;
  double sig_hat;
  const double* vert;
  const double* theta;
  const double* reaction;
  std::vector<double> gll, gx, gw;
  int64_t E;
};

Mesh make_mesh(const oracle_mesh* m) {
  Mesh M;
  M.N[0] = m->nx; M.N[1] = m->ny; M.N[2] = m->nz;
  M.k = m->degree;
  M.n = M.k + 1;
  M.n3 = M.n * M.n * M.n;
  M.nq = M.n + std::max(0, (int)m->quad_extra);
  M.bc = m->bc;
  M.mutation = m->mutation;
  M.sig_hat = m->penalty_hat > 0 ? m->penalty_hat : 2.0 * (M.k + 1) * (M.k + 1);
  M.vert = m->vertices;
  M.theta = m->theta;
  M.reaction = m->reaction;
  gll_nodes(M.n, M.gll);
  gauss_rule(M.nq, M.gx, M.gw);
  M.E = (int64_t)M.N[0] * M.N[1] * M.N[2];
  return M;
}

bool valid(const oracle_mesh* m) {
  return m && m->nx >= 1 && m->ny >= 1 && m->nz >= 1 && m->degree >= 1 && m->degree <= 12 &&
         (m->bc == 0 || m->bc == 1) && m->quad_extra >= 0;
}

inline int64_t elem_id(const Mesh& M, const int e[3]) {
  return e[0] + (int64_t)M.N[0] * (e[1] + (int64_t)M.N[1] * e[2]);
}
inline void elem_coords(const Mesh& M, int64_t id, int e[3]) {
  e[0] = (int)(id % M.N[0]);
  e[1] = (int)((id / M.N[0]) % M.N[1]);
  e[2] = (int)(id / ((int64_t)M.N[0] * M.N[1]));
}

/* Neighbour across face (d, s) (s = 0: lower face, s = 1: upper face),
 * -1 on a Dirichlet boundary.  Periodic meshes wrap. */
int64_t neighbour(const Mesh& M, const int e[3], int d, int s) {
  int f[3] = {e[0], e[1], e[2]};
  f[d] += s ? 1 : -1;
  if (f[d] < 0 || f[d] >= M.N[d]) {
    if (M.bc != 1) return -1;
    f[d] = (f[d] + M.N[d]) % M.N[d];
  }
  return elem_id(M, f);
}

struct Geo { double X[8][3]; };  /* corner c = c0 + 2 c1 + 4 c2 */

void element_geo(const Mesh& M, const int e[3], Geo& g) {
  for (int c = 0; c < 8; ++c) {
    int v[3] = {e[0] + (c & 1), e[1] + ((c >> 1) & 1), e[2] + ((c >> 2) & 1)};
    if (M.vert) {
      int64_t vid = v[0] + (int64_t)(M.N[0] + 1) * (v[1] + (int64_t)(M.N[1] + 1) * v[2]);
      for (int a = 0; a < 3; ++a) g.X[c][a] = M.vert[3 * vid + a];
    } else {
      for (int a = 0; a < 3; ++a) g.X[c][a] = (double)v[a] / M.N[a];
    }
  }
}

/* Trilinear map F(xi) and its Jacobian J[a][d] = dF_a / dxi_d. */
void map_point(const Geo& g, const double xi[3], double x[3]) {
  x[0] = x[1] = x[2] = 0.0;
  for (int c = 0; c < 8; ++c) {
    double w = 1.0;
    for (int d = 0; d < 3; ++d) w *= ((c >> d) & 1) ? xi[d] : 1.0 - xi[d];
    for (int a = 0; a < 3; ++a) x[a] += w * g.X[c][a];
  }
}
void jacobian(const Geo& g, const double xi[3], double J[3][3]) {
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) J[a][d] = 0.0;
  for (int c = 0; c < 8; ++c) {
    double f[3], df[3];
    for (int d = 0; d < 3; ++d) {
      bool hi = (c >> d) & 1;
      f[d] = hi ? xi[d] : 1.0 - xi[d];
      df[d] = hi ? 1.0 : -1.0;
    }
    double dN[3] = {df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]};
    for (int a = 0; a < 3; ++a)
      for (int d = 0; d < 3; ++d) J[a][d] += g.X[c][a] * dN[d];
  }
}
double det3(const double J[3][3]) {
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
         J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}
void inverse3(const double J[3][3], double Ji[3][3]) {
  double det = det3(J);
  Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
}

/* Values and physical gradients of all n^3 basis functions at reference point
 * xi of an element with Jacobian J:  grad phi = J^{-T} grad_ref phi. */
void basis_at(const Mesh& M, const double xi[3], const double J[3][3], double* val, double* grad) {
  const int n = M.n;
  double l[3][16], dl[3][16];
  for (int d = 0; d < 3; ++d)
    for (int i = 0; i < n; ++i) {
      l[d][i] = lagrange(M.gll, i, xi[d]);
      dl[d][i] = lagrange_d(M.gll, i, xi[d]);
    }
  double Ji[3][3];
  inverse3(J, Ji);
  for (int i3 = 0; i3 < n; ++i3)
    for (int i2 = 0; i2 < n; ++i2)
      for (int i1 = 0; i1 < n; ++i1) {
        int i = i1 + n * (i2 + n * i3);
        val[i] = l[0][i1] * l[1][i2] * l[2][i3];
        double gr[3] = {dl[0][i1] * l[1][i2] * l[2][i3], l[0][i1] * dl[1][i2] * l[2][i3],
                        l[0][i1] * l[1][i2] * dl[2][i3]};
        for (int a = 0; a < 3; ++a) {
          double s = 0.0;
          for (int d = 0; d < 3; ++d)
            s += (M.mutation == MUT_JINV_NOT_TRANSPOSED ? Ji[a][d] : Ji[d][a]) * gr[d];
          grad[3 * i + a] = s;
        }
      }
}

inline void cross(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Area-weighted normal of the face xi_d = const of an element: dF/dxi_a x
 * dF/dxi_b with (d, a, b) cyclic; it points towards increasing xi_d. */
void face_normal(const double J[3][3], int d, double nv[3]) {
  int a = (d + 1) % 3, b = (d + 2) % 3;
  double ta[3] = {J[0][a], J[1][a], J[2][a]};
  double tb[3] = {J[0][b], J[1][b], J[2][b]};
  cross(ta, tb, nv);
}

/* ------------------------------------------------------------------------ */
/* Local matrices (rows = test functions, columns = trial functions)          */
/* ------------------------------------------------------------------------ */

/* Volume: A[i][j] = sum_q w_q |det J_q| K (grad phi_i . grad phi_j). */
template <class S>
void volume_matrix(const Mesh& M, const Geo& g, S K, std::vector<S>& A) {
  const int n3 = M.n3, q = M.nq;
  A.assign((size_t)n3 * n3, S(0));
  std::vector<double> val(n3), grad(3 * n3);
  for (int q3 = 0; q3 < q; ++q3)
    for (int q2 = 0; q2 < q; ++q2)
      for (int q1 = 0; q1 < q; ++q1) {
        double xi[3] = {M.gx[q1], M.gx[q2], M.gx[q3]};
        double J[3][3];
        jacobian(g, xi, J);
        double c = M.gw[q1] * M.gw[q2] * M.gw[q3] * std::fabs(det3(J));
        basis_at(M, xi, J, val.data(), grad.data());
        for (int i = 0; i < n3; ++i)
          for (int j = 0; j < n3; ++j) {
            double gg = grad[3 * i] * grad[3 * j] + grad[3 * i + 1] * grad[3 * j + 1] +
                        grad[3 * i + 2] * grad[3 * j + 2];
            A[(size_t)i * n3 + j] += K * (c * gg);
          }
      }
}

/* Reaction (diffusion-reaction problems of Sec. 3.3):
 * A[i][j] = sum_q w_q |det J_q| c phi_i phi_j. */
void mass_matrix(const Mesh& M, const Geo& g, double c, std::vector<double>& A) {
  const int n3 = M.n3, q = M.nq;
  A.assign((size_t)n3 * n3, 0.0);
  std::vector<double> val(n3), grad(3 * n3);
  for (int q3 = 0; q3 < q; ++q3)
    for (int q2 = 0; q2 < q; ++q2)
      for (int q1 = 0; q1 < q; ++q1) {
        double xi[3] = {M.gx[q1], M.gx[q2], M.gx[q3]};
        double J[3][3];
        jacobian(g, xi, J);
        double w = M.gw[q1] * M.gw[q2] * M.gw[q3] * std::fabs(det3(J));
        basis_at(M, xi, J, val.data(), grad.data());
        for (int i = 0; i < n3; ++i)
          for (int j = 0; j < n3; ++j) A[(size_t)i * n3 + j] += c * (w * val[i] * val[j]);
      }
}

/* Interior face normal to axis d between T^- (geometry gm, face xi_d = 1) and
 * T^+ (geometry gp, face xi_d = 0), on the combined index set
 * beta = side * n3 + local (side 0 = T^-, side 1 = T^+).  Only rows in
 * [r0, r1) are formed; A has (r1-r0) x 2 n3 entries.
 *   a_e(u, v) = int_e -(gamma/2)(grad u^- + grad u^+).n [v]
 *                     -(gamma/2)(grad v^- + grad v^+).n [u] + sigma gamma [u][v]  */
template <class S>
void face_matrix(const Mesh& M, const Geo& gm, const Geo& gp, int d, S gamma, double sigma,
                 int r0, int r1, std::vector<S>& A) {
  const int n3 = M.n3, q = M.nq, a = (d + 1) % 3, b = (d + 2) % 3;
  const int nc = 2 * n3;
  A.assign((size_t)(r1 - r0) * nc, S(0));
  std::vector<double> vm(n3), gradm(3 * n3), vp(n3), gradp(3 * n3), jump(nc), flux(nc);
  const double cons = (M.mutation == MUT_PLUS_CONSISTENCY) ? 1.0 : -1.0;
  const double sym = (M.mutation == MUT_NO_SYMMETRY) ? 0.0 : 1.0;
  const double pen = (M.mutation == MUT_NO_PENALTY) ? 0.0 : sigma;
  for (int qb = 0; qb < q; ++qb)
    for (int qa = 0; qa < q; ++qa) {
      double xim[3], xip[3];
      xim[d] = 1.0;
      xip[d] = (M.mutation == MUT_PLUS_SIDE_AT_ONE) ? 1.0 : 0.0;
      xim[a] = xip[a] = M.gx[qa];
      xim[b] = xip[b] = M.gx[qb];
      double Jm[3][3], Jp[3][3], nv[3];
      jacobian(gm, xim, Jm);
      jacobian(gp, xip, Jp);
      face_normal(Jm, d, nv);
      double area = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
      double w = M.gw[qa] * M.gw[qb];
      basis_at(M, xim, Jm, vm.data(), gradm.data());
      basis_at(M, xip, Jp, vp.data(), gradp.data());
      for (int i = 0; i < n3; ++i) {
        jump[i] = vm[i];
        jump[n3 + i] = -vp[i];
        flux[i] = gradm[3 * i] * nv[0] + gradm[3 * i + 1] * nv[1] + gradm[3 * i + 2] * nv[2];
        flux[n3 + i] = gradp[3 * i] * nv[0] + gradp[3 * i + 1] * nv[1] + gradp[3 * i + 2] * nv[2];
      }
      double pa = (M.mutation == MUT_PENALTY_NO_AREA) ? 1.0 : area;
      for (int al = r0; al < r1; ++al)
        for (int be = 0; be < nc; ++be) {
          S v = gamma * (0.5 * cons * flux[be] * jump[al] + 0.5 * cons * sym * flux[al] * jump[be] +
                         pen * pa * jump[be] * jump[al]);
          A[(size_t)(al - r0) * nc + be] += w * v;
        }
    }
}

/* Boundary face (d, s) of an element, outward normal, weak Dirichlet:
 *   a_e(u, v) = int_e -K grad u.n v - K grad v.n u + sigma K u v. */
template <class S>
void boundary_matrix(const Mesh& M, const Geo& g, int d, int s, S K, double sigma,
                     std::vector<S>& A) {
  const int n3 = M.n3, q = M.nq, a = (d + 1) % 3, b = (d + 2) % 3;
  A.assign((size_t)n3 * n3, S(0));
  std::vector<double> v(n3), grad(3 * n3), flux(n3);
  const double cons = (M.mutation == MUT_PLUS_CONSISTENCY) ? 1.0 : -1.0;
  const double sym = (M.mutation == MUT_NO_SYMMETRY) ? 0.0 : 1.0;
  const double pen = (M.mutation == MUT_NO_PENALTY) ? 0.0 : sigma;
  for (int qb = 0; qb < q; ++qb)
    for (int qa = 0; qa < q; ++qa) {
      double xi[3];
      xi[d] = (double)s;
      xi[a] = M.gx[qa];
      xi[b] = M.gx[qb];
      double J[3][3], nv[3];
      jacobian(g, xi, J);
      face_normal(J, d, nv);
      if (s == 0)
        for (int c = 0; c < 3; ++c) nv[c] = -nv[c];
      double area = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
      double w = M.gw[qa] * M.gw[qb];
      basis_at(M, xi, J, v.data(), grad.data());
      for (int i = 0; i < n3; ++i)
        flux[i] = grad[3 * i] * nv[0] + grad[3 * i + 1] * nv[1] + grad[3 * i + 2] * nv[2];
      double pa = (M.mutation == MUT_PENALTY_NO_AREA) ? 1.0 : area;
      for (int al = 0; al < n3; ++al)
        for (int be = 0; be < n3; ++be) {
          S val = K * (cons * flux[be] * v[al] + cons * sym * flux[al] * v[be] +
                       pen * pa * v[be] * v[al]);
          A[(size_t)al * n3 + be] += w * val;
        }
    }
}

template <class S>
S coef_K(const Mesh& M, int64_t e) {
  using std::exp;
  return M.theta ? S(exp(M.theta[e])) : S(1.0);
}
template <class S>
S face_gamma(const Mesh& M, S Km, S Kp) {
  if (M.mutation == MUT_ARITH_GAMMA) return 0.5 * (Km + Kp);
  return 2.0 * Km * Kp / (Km + Kp);
}
inline double face_sigma(const Mesh& M, int d) { return M.sig_hat * M.N[d]; }

/* Sorted list of the distinct elements coupled to element e (itself plus
 * its interior-face neighbours). */
std::vector<int64_t> coupled(const Mesh& M, int64_t id) {
  int e[3];
  elem_coords(M, id, e);
  std::vector<int64_t> c{id};
  for (int d = 0; d < 3; ++d)
    for (int s = 0; s < 2; ++s) {
      int64_t nb = neighbour(M, e, d, s);
      if (nb >= 0) c.push_back(nb);
    }
  std::sort(c.begin(), c.end());
  c.erase(std::unique(c.begin(), c.end()), c.end());
  return c;
}

/* Block row of element `id`: the n3 rows of A belonging to it, stored densely
 * over the coupled elements (rows x (ncoupled * n3)). */
void element_block_row(const Mesh& M, int64_t id, const std::vector<int64_t>& cpl,
                       std::vector<double>& R) {
  const int n3 = M.n3;
  const int ncol = (int)cpl.size() * n3;
  R.assign((size_t)n3 * ncol, 0.0);
  auto slot = [&](int64_t el) {
    return (int)(std::lower_bound(cpl.begin(), cpl.end(), el) - cpl.begin());
  };
  int e[3];
  elem_coords(M, id, e);
  Geo g;
  element_geo(M, e, g);
  const double K = coef_K<double>(M, id);
  std::vector<double> L;
  volume_matrix<double>(M, g, K, L);
  int so = slot(id);
  for (int i = 0; i < n3; ++i)
    for (int j = 0; j < n3; ++j) R[(size_t)i * ncol + so * n3 + j] += L[(size_t)i * n3 + j];
  if (M.reaction) {
    mass_matrix(M, g, M.reaction[id], L);
    for (int i = 0; i < n3; ++i)
      for (int j = 0; j < n3; ++j) R[(size_t)i * ncol + so * n3 + j] += L[(size_t)i * n3 + j];
  }
  for (int d = 0; d < 3; ++d)
    for (int s = 0; s < 2; ++s) {
      int64_t nb = neighbour(M, e, d, s);
      if (nb < 0) {
        if (M.mutation == MUT_NO_BOUNDARY) continue;
        boundary_matrix<double>(M, g, d, s, K, face_sigma(M, d), L);
        for (int i = 0; i < n3; ++i)
          for (int j = 0; j < n3; ++j) R[(size_t)i * ncol + so * n3 + j] += L[(size_t)i * n3 + j];
        continue;
      }
      int en[3];
      elem_coords(M, nb, en);
      Geo gn;
      element_geo(M, en, gn);
      const double Kn = coef_K<double>(M, nb);
      /* upper face: this element is T^-; lower face: it is T^+ */
      const Geo& gm = s ? g : gn;
      const Geo& gp = s ? gn : g;
      const double Km = s ? K : Kn, Kp = s ? Kn : K;
      const int64_t em = s ? id : nb, ep = s ? nb : id;
      int r0 = s ? 0 : n3;
      face_matrix<double>(M, gm, gp, d, face_gamma<double>(M, Km, Kp), face_sigma(M, d), r0,
                          r0 + n3, L);
      int sm = slot(em), sp = slot(ep);
      for (int i = 0; i < n3; ++i)
        for (int j = 0; j < n3; ++j) {
          R[(size_t)i * ncol + sm * n3 + j] += L[(size_t)i * 2 * n3 + j];
          R[(size_t)i * ncol + sp * n3 + j] += L[(size_t)i * 2 * n3 + n3 + j];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Right-hand sides and errors for analytic data                             */
/* ------------------------------------------------------------------------ */

struct Exact {
  int kind;           /* 1: u = sin(pi x) sin(pi y) sin(pi z), f = 3 pi^2 u; 2: polynomial */
  int k;
  const double* c;    /* kind 2: u = sum c[a + (k+1)(b + (k+1) e)] x^a y^b z^e */
  double u(const double x[3]) const {
    if (kind == 1) return std::sin(kPi * x[0]) * std::sin(kPi * x[1]) * std::sin(kPi * x[2]);
    if (kind == 2) {
      double s = 0.0;
      const int m = k + 1;
      for (int e = 0; e < m; ++e)
        for (int b = 0; b < m; ++b)
          for (int a = 0; a < m; ++a)
            s += c[a + m * (b + m * e)] * std::pow(x[0], a) * std::pow(x[1], b) * std::pow(x[2], e);
      return s;
    }
    return 0.0;
  }
  /* f = -K lap u (K constant on the element) */
  double f(const double x[3], double K) const {
    if (kind == 1) return 3.0 * kPi * kPi * u(x);
    if (kind == 2) {
      double s = 0.0;
      const int m = k + 1;
      auto mono = [](double t, int p) { return p < 0 ? 0.0 : std::pow(t, p); };
      for (int e = 0; e < m; ++e)
        for (int b = 0; b < m; ++b)
          for (int a = 0; a < m; ++a) {
            double cc = c[a + m * (b + m * e)];
            if (cc == 0.0) continue;
            s += cc * (a * (a - 1) * mono(x[0], a - 2) * mono(x[1], b) * mono(x[2], e) +
                       b * (b - 1) * mono(x[0], a) * mono(x[1], b - 2) * mono(x[2], e) +
                       e * (e - 1) * mono(x[0], a) * mono(x[1], b) * mono(x[2], e - 2));
          }
      return -K * s;
    }
    return 0.0;
  }
  /* Dirichlet data on the boundary */
  double g(const double x[3]) const { return kind == 2 ? u(x) : 0.0; }
};

}  // namespace

/* ------------------------------------------------------------------------ */
/* C ABI                                                                     */
/* ------------------------------------------------------------------------ */
extern "C" {

int oracle_num_threads(void) { return omp_get_max_threads(); }

/* 1D tables: n GLL nodes, nq Gauss points and weights, all on [0,1]. */
int oracle_tables(int n, int nq, double* gll, double* gx, double* gw) {
  if (n < 2 || nq < 1) return -1;
  std::vector<double> a, b, c;
  gll_nodes(n, a);
  gauss_rule(nq, b, c);
  std::copy(a.begin(), a.end(), gll);
  std::copy(b.begin(), b.end(), gx);
  std::copy(c.begin(), c.end(), gw);
  return 0;
}

/* Number of stored entries of the CSR matrix (dense n^3 blocks per coupled
 * element pair). */
int64_t oracle_csr_nnz(const oracle_mesh* m) {
  if (!valid(m)) return -1;
  Mesh M = make_mesh(m);
  int64_t nnz = 0;
  for (int64_t id = 0; id < M.E; ++id) nnz += (int64_t)coupled(M, id).size() * M.n3 * M.n3;
  return nnz;
}

/* Assemble A (rows = test DOFs) into caller-allocated CSR arrays: rowptr
 * (N_dof+1), cols and vals (oracle_csr_nnz entries); columns sorted. */
int oracle_csr_assemble(const oracle_mesh* m, int64_t* rowptr, int64_t* cols, double* vals) {
  if (!valid(m)) return -1;
  Mesh M = make_mesh(m);
  const int n3 = M.n3;
  std::vector<int64_t> rowlen(M.E);
  for (int64_t id = 0; id < M.E; ++id) rowlen[id] = (int64_t)coupled(M, id).size() * n3;
  rowptr[0] = 0;
  for (int64_t id = 0; id < M.E; ++id)
    for (int i = 0; i < n3; ++i) rowptr[id * n3 + i + 1] = rowptr[id * n3 + i] + rowlen[id];
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t id = 0; id < M.E; ++id) {
    std::vector<int64_t> cpl = coupled(M, id);
    std::vector<double> R;
    element_block_row(M, id, cpl, R);
    const int ncol = (int)cpl.size() * n3;
    for (int i = 0; i < n3; ++i) {
      int64_t p = rowptr[id * n3 + i];
      for (size_t c = 0; c < cpl.size(); ++c)
        for (int j = 0; j < n3; ++j) {
          cols[p] = cpl[c] * n3 + j;
          vals[p] = R[(size_t)i * ncol + c * n3 + j];
          ++p;
        }
    }
  }
  return 0;
}

/* y = A x for CSR A (OpenMP over rows). */
int oracle_spmv(int64_t nrows, const int64_t* rowptr, const int64_t* cols, const double* vals,
                const double* x, double* y) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < nrows; ++r) {
    double s = 0.0;
    for (int64_t p = rowptr[r]; p < rowptr[r + 1]; ++p) s += vals[p] * x[cols[p]];
    y[r] = s;
  }
  return 0;
}

/* Rows of y = A x belonging to the listed elements, from local matrices,
 * without global storage.  y has nsel * n^3 entries (element order of elems). */
int oracle_apply_rows(const oracle_mesh* m, const double* x, int64_t nsel, const int64_t* elems,
                      double* y) {
  if (!valid(m)) return -1;
  Mesh M = make_mesh(m);
  const int n3 = M.n3;
  for (int64_t s = 0; s < nsel; ++s)
    if (elems[s] < 0 || elems[s] >= M.E) return -1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t s = 0; s < nsel; ++s) {
    int64_t id = elems[s];
    std::vector<int64_t> cpl = coupled(M, id);
    std::vector<double> R;
    element_block_row(M, id, cpl, R);
    const int ncol = (int)cpl.size() * n3;
    for (int i = 0; i < n3; ++i) {
      double acc = 0.0;
      for (size_t c = 0; c < cpl.size(); ++c)
        for (int j = 0; j < n3; ++j) acc += R[(size_t)i * ncol + c * n3 + j] * x[cpl[c] * n3 + j];
      y[s * n3 + i] = acc;
    }
  }
  return 0;
}

/* Alg. "PCG" of Sec. 2.4 on a CSR matrix with M = diag(A)^{-1} (jacobi != 0)
 * or M = I; the convergence test ||r|| <= rtol ||b|| is evaluated together
 * with <z, r>.  x holds x0 on entry and the iterate on exit. */
int oracle_pcg(int64_t n, const int64_t* rowptr, const int64_t* cols, const double* vals,
               const double* b, double* x, double rtol, int maxit, int jacobi, int* iters,
               double* relres) {
  std::vector<double> r(n), p(n), q(n), z(n), dinv(n, 1.0);
  if (jacobi)
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
        if (cols[k] == i) dinv[i] = 1.0 / vals[k];
  auto dot = [&](const std::vector<double>& a, const std::vector<double>& c) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * c[i];
    return s;
  };
  double bnorm = 0.0;
  for (int64_t i = 0; i < n; ++i) bnorm += b[i] * b[i];
  bnorm = std::sqrt(bnorm);
  oracle_spmv(n, rowptr, cols, vals, x, q.data());
  for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
  for (int64_t i = 0; i < n; ++i) p[i] = dinv[i] * r[i];
  double rho = dot(p, r);
  int it = 0;
  bool done = std::sqrt(dot(r, r)) <= rtol * bnorm;
  while (!done && it < maxit) {
    ++it;
    oracle_spmv(n, rowptr, cols, vals, p.data(), q.data());
    double alpha = dot(p, q);
    double lam = rho / alpha;
    for (int64_t i = 0; i < n; ++i) {
      x[i] += lam * p[i];
      r[i] -= lam * q[i];
    }
    for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
    double rr = dot(r, r), rho_new = dot(z, r);
    if (std::sqrt(rr) <= rtol * bnorm) break;
    double beta = rho_new / rho;
    for (int64_t i = 0; i < n; ++i) p[i] = beta * p[i] + z[i];
    rho = rho_new;
  }
  oracle_spmv(n, rowptr, cols, vals, x, q.data());
  double rn = 0.0;
  for (int64_t i = 0; i < n; ++i) rn += (b[i] - q[i]) * (b[i] - q[i]);
  *iters = it;
  *relres = bnorm > 0 ? std::sqrt(rn) / bnorm : std::sqrt(rn);
  return 0;
}

/* Load vector b_i = int f phi_i (+ Dirichlet lifting terms
 * int_{boundary} -K grad phi_i.n g + sigma K g phi_i for fkind 2). */
int oracle_rhs(const oracle_mesh* m, int fkind, const double* coef, double* bvec) {
  if (!valid(m) || fkind < 1 || fkind > 2) return -1;
  Mesh M = make_mesh(m);
  Exact ex{fkind, M.k, coef};
  const int n3 = M.n3, q = M.nq;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t id = 0; id < M.E; ++id) {
    int e[3];
    elem_coords(M, id, e);
    Geo g;
    element_geo(M, e, g);
    double K = coef_K<double>(M, id);
    std::vector<double> v(n3), grad(3 * n3), acc(n3, 0.0);
    for (int q3 = 0; q3 < q; ++q3)
      for (int q2 = 0; q2 < q; ++q2)
        for (int q1 = 0; q1 < q; ++q1) {
          double xi[3] = {M.gx[q1], M.gx[q2], M.gx[q3]}, J[3][3], x[3];
          jacobian(g, xi, J);
          map_point(g, xi, x);
          double c = M.gw[q1] * M.gw[q2] * M.gw[q3] * std::fabs(det3(J)) * ex.f(x, K);
          basis_at(M, xi, J, v.data(), grad.data());
          for (int i = 0; i < n3; ++i) acc[i] += c * v[i];
        }
    if (fkind == 2) {
      for (int d = 0; d < 3; ++d)
        for (int s = 0; s < 2; ++s) {
          if (neighbour(M, e, d, s) >= 0) continue;
          const int a = (d + 1) % 3, b = (d + 2) % 3;
          for (int qb = 0; qb < q; ++qb)
            for (int qa = 0; qa < q; ++qa) {
              double xi[3], J[3][3], nv[3], x[3];
              xi[d] = (double)s;
              xi[a] = M.gx[qa];
              xi[b] = M.gx[qb];
              jacobian(g, xi, J);
              map_point(g, xi, x);
              face_normal(J, d, nv);
              if (s == 0)
                for (int c = 0; c < 3; ++c) nv[c] = -nv[c];
              double area = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
              double w = M.gw[qa] * M.gw[qb], gval = ex.g(x);
              basis_at(M, xi, J, v.data(), grad.data());
              for (int i = 0; i < n3; ++i) {
                double fl = grad[3 * i] * nv[0] + grad[3 * i + 1] * nv[1] + grad[3 * i + 2] * nv[2];
                acc[i] += w * K * (-fl * gval + face_sigma(M, d) * area * gval * v[i]);
              }
            }
        }
    }
    for (int i = 0; i < n3; ++i) bvec[id * n3 + i] = acc[i];
  }
  return 0;
}

/* ||u_h - u||_{L2} with (k+3)-point Gauss per direction. */
double oracle_l2_error(const oracle_mesh* m, const double* uh, int fkind, const double* coef) {
  if (!valid(m)) return -1.0;
  oracle_mesh mm = *m;
  mm.quad_extra = 2;
  Mesh M = make_mesh(&mm);
  Exact ex{fkind, M.k, coef};
  const int n3 = M.n3, q = M.nq;
  double total = 0.0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
  for (int64_t id = 0; id < M.E; ++id) {
    int e[3];
    elem_coords(M, id, e);
    Geo g;
    element_geo(M, e, g);
    std::vector<double> v(n3), grad(3 * n3);
    for (int q3 = 0; q3 < q; ++q3)
      for (int q2 = 0; q2 < q; ++q2)
        for (int q1 = 0; q1 < q; ++q1) {
          double xi[3] = {M.gx[q1], M.gx[q2], M.gx[q3]}, J[3][3], x[3];
          jacobian(g, xi, J);
          map_point(g, xi, x);
          basis_at(M, xi, J, v.data(), grad.data());
          double s = 0.0;
          for (int i = 0; i < n3; ++i) s += uh[id * n3 + i] * v[i];
          double diff = s - ex.u(x);
          total += M.gw[q1] * M.gw[q2] * M.gw[q3] * std::fabs(det3(J)) * diff * diff;
        }
  }
  return std::sqrt(total);
}

/* g_T = u^T (dA/dtheta_T) v, K_T = exp(theta_T): the volume matrix with K_T
 * replaced by dK_T/dtheta_T = K_T, each face matrix of T with gamma_e replaced
 * by d gamma_e / d theta_T = gamma_e K_other / (K^- + K^+) (interior) or
 * d K_T / d theta_T = K_T (boundary). */
int oracle_dA_dtheta_elems(const oracle_mesh* m, const double* u, const double* vv, int64_t nsel,
                           const int64_t* elems, double* gout);

int oracle_dA_dtheta(const oracle_mesh* m, const double* u, const double* vv, double* gout) {
  if (!valid(m)) return -1;
  const int64_t E = (int64_t)m->nx * m->ny * m->nz;
  std::vector<int64_t> all(E);
  for (int64_t i = 0; i < E; ++i) all[i] = i;
  return oracle_dA_dtheta_elems(m, u, vv, E, all.data(), gout);
}

/* The same for the listed elements only: gout[s] = g_{elems[s]}. */
int oracle_dA_dtheta_elems(const oracle_mesh* m, const double* u, const double* vv, int64_t nsel,
                           const int64_t* elems, double* gout) {
  if (!valid(m)) return -1;
  Mesh M = make_mesh(m);
  const int n3 = M.n3;
  for (int64_t s = 0; s < nsel; ++s)
    if (elems[s] < 0 || elems[s] >= M.E) return -1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t sel = 0; sel < nsel; ++sel) {
    const int64_t id = elems[sel];

    int e[3];
    elem_coords(M, id, e);
    Geo g;
    element_geo(M, e, g);
    const double K = coef_K<double>(M, id);
    std::vector<double> L;
    double acc = 0.0;
    volume_matrix<double>(M, g, K, L);  /* dK/dtheta = K */
    for (int i = 0; i < n3; ++i)
      for (int j = 0; j < n3; ++j) acc += u[id * n3 + i] * L[(size_t)i * n3 + j] * vv[id * n3 + j];
    for (int d = 0; d < 3; ++d)
      for (int s = 0; s < 2; ++s) {
        int64_t nb = neighbour(M, e, d, s);
        if (nb < 0) {
          if (M.mutation == MUT_NO_BOUNDARY) continue;
          boundary_matrix<double>(M, g, d, s, K, face_sigma(M, d), L);
          for (int i = 0; i < n3; ++i)
            for (int j = 0; j < n3; ++j)
              acc += u[id * n3 + i] * L[(size_t)i * n3 + j] * vv[id * n3 + j];
          continue;
        }
        int en[3];
        elem_coords(M, nb, en);
        Geo gn;
        element_geo(M, en, gn);
        const double Kn = coef_K<double>(M, nb);
        const Geo& gm = s ? g : gn;
        const Geo& gp = s ? gn : g;
        const double Km = s ? K : Kn, Kp = s ? Kn : K;
        const int64_t em = s ? id : nb, ep = s ? nb : id;
        double gam = face_gamma<double>(M, Km, Kp);
        double dgam = (M.mutation == MUT_ARITH_GAMMA) ? 0.5 * K : gam * Kn / (Km + Kp);
        face_matrix<double>(M, gm, gp, d, dgam, face_sigma(M, d), 0, 2 * n3, L);
        const int nc = 2 * n3;
        for (int al = 0; al < nc; ++al) {
          double ua = al < n3 ? u[em * n3 + al] : u[ep * n3 + al - n3];
          for (int be = 0; be < nc; ++be) {
            double vb = be < n3 ? vv[em * n3 + be] : vv[ep * n3 + be - n3];
            acc += ua * L[(size_t)al * nc + be] * vb;
          }
        }
      }
    gout[sel] = acc;
  }
  return 0;
}


/* The same gradient by the complex-step derivative: theta_T -> theta_T + i h,
 * h = 1e-30, and g_T = Im(u^T A(theta + i h e_T) v) / h over the local
 * matrices that depend on theta_T (the volume of T and each distinct face of
 * T).  Exact to rounding; checks the closed forms used above. */
int oracle_dA_dtheta_cs(const oracle_mesh* m, const double* u, const double* vv, double* gout) {
  if (!valid(m)) return -1;
  typedef std::complex<double> C;
  Mesh M = make_mesh(m);
  const int n3 = M.n3;
  const double h = 1e-30;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t id = 0; id < M.E; ++id) {
    int e[3];
    elem_coords(M, id, e);
    Geo g;
    element_geo(M, e, g);
    const double th = M.theta ? M.theta[id] : 0.0;
    const C K = std::exp(C(th, h));
    std::vector<C> L;
    C acc(0.0, 0.0);
    volume_matrix<C>(M, g, K, L);
    for (int i = 0; i < n3; ++i)
      for (int j = 0; j < n3; ++j) acc += u[id * n3 + i] * L[(size_t)i * n3 + j] * vv[id * n3 + j];
    for (int d = 0; d < 3; ++d)
      for (int s = 0; s < 2; ++s) {
        /* with one element along d and periodic wrap, the lower and upper
         * faces are the same face: count it once */
        if (M.bc == 1 && M.N[d] == 1 && s == 0) continue;
        int64_t nb = neighbour(M, e, d, s);
        if (nb < 0) {
          if (M.mutation == MUT_NO_BOUNDARY) continue;
          boundary_matrix<C>(M, g, d, s, K, face_sigma(M, d), L);
          for (int i = 0; i < n3; ++i)
            for (int j = 0; j < n3; ++j)
              acc += u[id * n3 + i] * L[(size_t)i * n3 + j] * vv[id * n3 + j];
          continue;
        }
        int en[3];
        elem_coords(M, nb, en);
        Geo gn;
        element_geo(M, en, gn);
        const C Kn = (nb == id) ? K : coef_K<C>(M, nb);
        const Geo& gm = s ? g : gn;
        const Geo& gp = s ? gn : g;
        const C Km = s ? K : Kn, Kp = s ? Kn : K;
        const int64_t em = s ? id : nb, ep = s ? nb : id;
        face_matrix<C>(M, gm, gp, d, face_gamma<C>(M, Km, Kp), face_sigma(M, d), 0, 2 * n3, L);
        const int nc = 2 * n3;
        for (int al = 0; al < nc; ++al) {
          double ua = al < n3 ? u[em * n3 + al] : u[ep * n3 + al - n3];
          for (int be = 0; be < nc; ++be) {
            double vb = be < n3 ? vv[em * n3 + be] : vv[ep * n3 + be - n3];
            acc += ua * L[(size_t)al * nc + be] * vb;
          }
        }
      }
    gout[id] = acc.imag() / h;
  }
  return 0;
}

}  // extern "C"
