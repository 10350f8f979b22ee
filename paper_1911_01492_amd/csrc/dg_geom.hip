// dg_geom.hip -- element geometry helpers: trilinear element maps, volume
// quadrature points and the load vector b_i = int f phi_i (Sec. 4.1, right
// hand side l_h), for affine and trilinear meshes.
#include "dg_internal.hpp"
#include "dg_kernels.hpp"
#include "dg_geom.hpp"

namespace dg {

// one block per element, one thread per quadrature point
template <int N>
__global__ __launch_bounds__(512) void k_quad_points(MeshArgs<double> m, double* __restrict__ xq) {
  constexpr int N3 = N * N * N;
  const int64_t e = blockIdx.x;
  const int q = threadIdx.x;
  if (q >= N3) return;
  const Tables<double>& T = *m.tab;
  double X[8][3];
  element_corners(m, e, X);
  const double xi[3] = {T.gx[q % N], T.gx[(q / N) % N], T.gx[q / (N * N)]};
  double x[3];
  trilinear_map(X, xi, x);
  for (int a = 0; a < 3; ++a) xq[(e * N3 + q) * 3 + a] = x[a];
}

// b_i = sum_q w_q |det J_q| f_q B_{q1 i1} B_{q2 i2} B_{q3 i3}
template <int N>
__global__ __launch_bounds__(512) void k_load_vector(MeshArgs<double> m, const double* __restrict__ fq,
                                                     double* __restrict__ b) {
  constexpr int N3 = N * N * N;
  __shared__ double W[N3];
  const int64_t e = blockIdx.x;
  const int t = threadIdx.x;
  const Tables<double>& T = *m.tab;
  if (t < N3) {
    double X[8][3];
    element_corners(m, e, X);
    const int q1 = t % N, q2 = (t / N) % N, q3 = t / (N * N);
    const double xi[3] = {T.gx[q1], T.gx[q2], T.gx[q3]};
    double J[3][3];
    trilinear_jacobian(X, xi, J);
    W[t] = T.gw[q1] * T.gw[q2] * T.gw[q3] * fabs(det3(J)) * fq[e * N3 + t];
  }
  __syncthreads();
  if (t < N3) {
    const int i1 = t % N, i2 = (t / N) % N, i3 = t / (N * N);
    double s = 0.0;
    for (int q3 = 0; q3 < N; ++q3)
      for (int q2 = 0; q2 < N; ++q2) {
        const double c = T.B[q3 * kMaxN + i3] * T.B[q2 * kMaxN + i2];
        for (int q1 = 0; q1 < N; ++q1) s += c * T.B[q1 * kMaxN + i1] * W[(q3 * N + q2) * N + q1];
      }
    b[e * N3 + t] = s;
  }
}

template <int N>
static hipError_t run_qp(const MeshArgs<double>& m, double* xq, hipStream_t s) {
  const int th = ((N * N * N + 63) / 64) * 64;
  hipLaunchKernelGGL((k_quad_points<N>), dim3((unsigned)m.E), dim3(th), 0, s, m, xq);
  return hipGetLastError();
}
template <int N>
static hipError_t run_lv(const MeshArgs<double>& m, const double* fq, double* b, hipStream_t s) {
  const int th = ((N * N * N + 63) / 64) * 64;
  hipLaunchKernelGGL((k_load_vector<N>), dim3((unsigned)m.E), dim3(th), 0, s, m, fq, b);
  return hipGetLastError();
}

hipError_t launch_quad_points(int n, const MeshArgs<double>& m, double* xq, hipStream_t s) {
  switch (n) {
    case 2: return run_qp<2>(m, xq, s);
    case 3: return run_qp<3>(m, xq, s);
    case 4: return run_qp<4>(m, xq, s);
    case 5: return run_qp<5>(m, xq, s);
    case 6: return run_qp<6>(m, xq, s);
    case 7: return run_qp<7>(m, xq, s);
    case 8: return run_qp<8>(m, xq, s);
  }
  return hipErrorInvalidValue;
}
hipError_t launch_load_vector(int n, const MeshArgs<double>& m, const double* fq, double* b,
                              hipStream_t s) {
  switch (n) {
    case 2: return run_lv<2>(m, fq, b, s);
    case 3: return run_lv<3>(m, fq, b, s);
    case 4: return run_lv<4>(m, fq, b, s);
    case 5: return run_lv<5>(m, fq, b, s);
    case 6: return run_lv<6>(m, fq, b, s);
    case 7: return run_lv<7>(m, fq, b, s);
    case 8: return run_lv<8>(m, fq, b, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace dg
