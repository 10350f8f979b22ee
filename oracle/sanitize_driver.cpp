/*
 * sanitize_driver.cpp -- TEST INFRASTRUCTURE.  Calls every entry point of the
 * oracle on small meshes (affine and trilinear, Dirichlet and periodic with
 * a self-neighbouring element, lognormal-like K, reaction term) so that the
 * test-suite can run the oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer on the CPU.  Exit status 0 when every call
 * succeeded; the sanitizers abort on the first finding.
 */
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

extern "C" {
typedef struct {
  int32_t nx, ny, nz, degree, bc, quad_extra, mutation, pad_;
  double penalty_hat;
  const double* vertices;
  const double* theta;
  const double* reaction;
} oracle_mesh;
int oracle_tables(int n, int nq, double* gll, double* gx, double* gw);
int64_t oracle_csr_nnz(const oracle_mesh* m);
int oracle_csr_assemble(const oracle_mesh* m, int64_t* rowptr, int64_t* cols, double* vals);
int oracle_spmv(int64_t nrows, const int64_t* rowptr, const int64_t* cols, const double* vals, const double* x,
                double* y);
int oracle_apply_rows(const oracle_mesh* m, const double* x, int64_t nsel, const int64_t* elems, double* y);
int oracle_pcg(int64_t n, const int64_t* rowptr, const int64_t* cols, const double* vals, const double* b, double* x,
               double rtol, int maxit, int jacobi, int* iters, double* relres);
int oracle_rhs(const oracle_mesh* m, int fkind, const double* coef, double* bvec);
double oracle_l2_error(const oracle_mesh* m, const double* uh, int fkind, const double* coef);
int oracle_dA_dtheta(const oracle_mesh* m, const double* u, const double* vv, double* gout);
int oracle_dA_dtheta_elems(const oracle_mesh* m, const double* u, const double* vv, int64_t nsel,
                           const int64_t* elems, double* gout);
int oracle_dA_dtheta_cs(const oracle_mesh* m, const double* u, const double* vv, double* gout);
}

static int fails = 0;
#define CHECK(c)                                              \
  do {                                                        \
    if (!(c)) {                                               \
      std::printf("FAILED: %s (line %d)\n", #c, __LINE__);    \
      ++fails;                                                \
    }                                                         \
  } while (0)

static void run(int nx, int ny, int nz, int k, int bc, bool trilinear, bool reaction) {
  const int n = k + 1, n3 = n * n * n;
  const int64_t E = (int64_t)nx * ny * nz, N = E * n3;
  std::vector<double> theta(E), c(E), V;
  for (int64_t e = 0; e < E; ++e) {
    theta[e] = 0.5 * std::sin(1.3 * (double)e + 0.2);
    c[e] = 1.0 + 0.25 * (double)(e % 3);
  }
  if (trilinear) {
    for (int z = 0; z <= nz; ++z)
      for (int y = 0; y <= ny; ++y)
        for (int x = 0; x <= nx; ++x) {
          const bool in = x > 0 && x < nx && y > 0 && y < ny && z > 0 && z < nz;
          const double d = in ? 0.05 * std::sin(3.0 * x + 5.0 * y + 7.0 * z) : 0.0;
          V.push_back((double)x / nx + d / nx);
          V.push_back((double)y / ny - d / ny);
          V.push_back((double)z / nz + d / nz);
        }
  }
  oracle_mesh m{nx, ny, nz, k, bc, 0, 0, 0, 0.0, trilinear ? V.data() : nullptr, theta.data(),
                reaction ? c.data() : nullptr};
  const int64_t nnz = oracle_csr_nnz(&m);
  CHECK(nnz > 0);
  std::vector<int64_t> rp(N + 1), ci(nnz);
  std::vector<double> va(nnz);
  CHECK(oracle_csr_assemble(&m, rp.data(), ci.data(), va.data()) == 0);
  std::vector<double> x(N), y(N), b(N), u(N, 0.0), g(E), g2(E);
  for (int64_t i = 0; i < N; ++i) x[i] = std::cos(0.7 * (double)i);
  CHECK(oracle_spmv(N, rp.data(), ci.data(), va.data(), x.data(), y.data()) == 0);
  std::vector<int64_t> el = {0, E - 1};
  std::vector<double> rows(2 * n3);
  CHECK(oracle_apply_rows(&m, x.data(), 2, el.data(), rows.data()) == 0);
  for (int i = 0; i < n3; ++i) CHECK(std::fabs(rows[i] - y[i]) <= 1e-12 * (1.0 + std::fabs(y[i])));
  CHECK(oracle_rhs(&m, 1, nullptr, b.data()) == 0);
  if (bc == 1 && !reaction) b.assign(N, 0.0), b[0] = 1.0, b[N - 1] = -1.0;  // periodic A is singular: b in the range
  int it = 0;
  double rr = 0.0;
  CHECK(oracle_pcg(N, rp.data(), ci.data(), va.data(), b.data(), u.data(), 1e-10, 5000, 1, &it, &rr) >= 0);
  const double l2 = oracle_l2_error(&m, u.data(), 1, nullptr);
  CHECK(l2 >= 0.0);
  CHECK(oracle_dA_dtheta(&m, x.data(), y.data(), g.data()) == 0);
  CHECK(oracle_dA_dtheta_cs(&m, x.data(), y.data(), g2.data()) == 0);
  for (int64_t e = 0; e < E; ++e) CHECK(std::fabs(g[e] - g2[e]) <= 1e-9 * (1.0 + std::fabs(g[e])));
  std::vector<double> g3(2);
  CHECK(oracle_dA_dtheta_elems(&m, x.data(), y.data(), 2, el.data(), g3.data()) == 0);
  CHECK(std::fabs(g3[0] - g[0]) <= 1e-12 * (1.0 + std::fabs(g[0])));
}

int main() {
  std::vector<double> a(8), b(8), w(8);
  CHECK(oracle_tables(5, 5, a.data(), b.data(), w.data()) == 0);
  CHECK(oracle_tables(1, 1, a.data(), b.data(), w.data()) != 0);  // rejected
  oracle_mesh bad{0, 1, 1, 1, 0, 0, 0, 0, 0.0, nullptr, nullptr, nullptr};
  CHECK(oracle_csr_nnz(&bad) < 0);
  run(2, 2, 2, 2, 0, false, false);
  run(2, 1, 3, 1, 1, false, false);  // periodic, one element along y couples with itself
  run(2, 2, 2, 3, 0, true, true);    // trilinear with reaction
  run(1, 1, 1, 4, 1, true, true);    // self-neighbour in every direction
  std::printf(fails ? "sanitize driver: %d failures\n" : "sanitize driver: ok\n", fails);
  return fails ? 1 : 0;
}
