// Setup kernels: geometric factors of the element maps and the operator diagonal.
//
// Geometry (chain rule, Sec. 2.2): J = dx/dr by applying D along i, j, k to
// the nodal coordinates; with C the adjugate of J (C = detJ J^{-1}, rows =
// detJ grad r, grad s, grad t),
//   G_ab = w_q (C_a . C_b) / detJ,   B = w_q detJ,   w_q = rho_i rho_j rho_k.
#include "common.hpp"

namespace sem {
namespace {

constexpr int kGeoThreads = 256;
constexpr int kMaxP = (kMaxOrder + 1) * (kMaxOrder + 1) * (kMaxOrder + 1);

__global__ __launch_bounds__(kGeoThreads) void geometry_kernel(
    const double* __restrict__ xyz, const double* __restrict__ Dg, const double* __restrict__ rho,
    int n1, int64_t E, double* __restrict__ G, double* __restrict__ B, float* __restrict__ G32,
    float* __restrict__ B32, int* __restrict__ bad) {
  __shared__ double X[3][kMaxP];
  __shared__ double D[(kMaxOrder + 1) * (kMaxOrder + 1)];
  __shared__ double w1[kMaxOrder + 1];
  const int64_t e = blockIdx.x;  // one workgroup per element: the grid is E
  (void)E;
  const int P2 = n1 * n1, P = P2 * n1;
  for (int a = threadIdx.x; a < n1 * n1; a += blockDim.x) D[a] = Dg[a];
  for (int a = threadIdx.x; a < n1; a += blockDim.x) w1[a] = rho[a];
  for (int a = threadIdx.x; a < 3 * P; a += blockDim.x) {
    const int q = a / 3, d = a - 3 * q;
    X[d][q] = xyz[e * 3 * P + a];
  }
  __syncthreads();
  int nbad = 0;
  for (int q = threadIdx.x; q < P; q += blockDim.x) {
    const int i = q % n1, j = (q / n1) % n1, k = q / P2;
    double J[3][3];
    for (int d = 0; d < 3; ++d) {
      double dr = 0, ds = 0, dt = 0;
      for (int l = 0; l < n1; ++l) {
        dr += D[i * n1 + l] * X[d][k * P2 + j * n1 + l];
        ds += D[j * n1 + l] * X[d][k * P2 + l * n1 + i];
        dt += D[k * n1 + l] * X[d][l * P2 + j * n1 + i];
      }
      J[d][0] = dr;
      J[d][1] = ds;
      J[d][2] = dt;
    }
    // adjugate rows: C[a][c] = detJ * (d r_a / d x_c)
    double C[3][3];
    C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    C[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    C[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    C[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    C[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    C[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    C[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * C[0][0] + J[0][1] * C[1][0] + J[0][2] * C[2][0];
    if (!(det > 0.0)) ++nbad;
    const double wq = w1[i] * w1[j] * w1[k];
    const double s = wq / det;
    const int pairs[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    for (int c = 0; c < 6; ++c) {
      const int a = pairs[c][0], b = pairs[c][1];
      const double g = s * (C[a][0] * C[b][0] + C[a][1] * C[b][1] + C[a][2] * C[b][2]);
      G[(e * 6 + c) * P + q] = g;
      G32[(e * 6 + c) * P + q] = (float)g;
    }
    B[e * P + q] = wq * det;
    B32[e * P + q] = (float)(wq * det);
  }
  if (nbad) atomicAdd(bad, nbad);
}

// Diagonal of A_L(k) at every local point (i, j, k):
//   sum_l D_li^2 (kG_rr)(l,j,k) + sum_l D_lj^2 (kG_ss)(i,l,k) + sum_l D_lk^2 (kG_tt)(i,j,l)
//   + 2 (D_ii D_jj kG_rs + D_ii D_kk kG_rt + D_jj D_kk kG_st)(i,j,k) + h2 B.
__global__ void local_diag_kernel(const double* __restrict__ G, const double* __restrict__ B,
                                  const double* __restrict__ kf, const double* __restrict__ D,
                                  double h2, int n1, int64_t nL, double* __restrict__ dL) {
  const int P2 = n1 * n1, P = P2 * n1;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < nL;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = idx / P;
    const int q = (int)(idx - e * P);
    const int i = q % n1, j = (q / n1) % n1, k = q / P2;
    const double* g = G + e * 6 * P;
    const double* kk = kf ? kf + e * P : nullptr;
    double s = 0.0;
    for (int l = 0; l < n1; ++l) {
      const int qr = k * P2 + j * n1 + l, qs = k * P2 + l * n1 + i, qt = l * P2 + j * n1 + i;
      const double dli = D[l * n1 + i], dlj = D[l * n1 + j], dlk = D[l * n1 + k];
      s += dli * dli * g[0 * P + qr] * (kk ? kk[qr] : 1.0);
      s += dlj * dlj * g[3 * P + qs] * (kk ? kk[qs] : 1.0);
      s += dlk * dlk * g[5 * P + qt] * (kk ? kk[qt] : 1.0);
    }
    const double dii = D[i * n1 + i], djj = D[j * n1 + j], dkk = D[k * n1 + k];
    s += 2.0 * (dii * djj * g[1 * P + q] + dii * dkk * g[2 * P + q] + djj * dkk * g[4 * P + q]) *
         (kk ? kk[q] : 1.0);
    if (h2 != 0.0) s += h2 * B[idx];
    dL[idx] = s;
  }
}

}  // namespace

hipError_t launch_geometry(const sem_mesh* m, const double* xyz, double* G, double* B, float* G32,
                           float* B32, int* bad_count, hipStream_t s) {
  // rho lives right after D in the D64 buffer (see api setup)
  const double* D = m->D64.as<double>();
  const double* rho = D + m->n1 * m->n1;
  hipLaunchKernelGGL(geometry_kernel, dim3((unsigned)m->E), dim3(kGeoThreads), 0, s, xyz, D, rho,
                     m->n1, m->E, G, B, G32, B32, bad_count);
  return hipGetLastError();
}

hipError_t launch_local_diag(const sem_mesh* m, const double* k, double h2, double* dL,
                             hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((m->nL + kVecBlock - 1) / kVecBlock, 16384);
  hipLaunchKernelGGL(local_diag_kernel, dim3((unsigned)blocks), dim3(kVecBlock), 0, s,
                     m->G64.as<double>(), m->B64.as<double>(), k, m->D64.as<double>(), h2, m->n1,
                     m->nL, dL);
  return hipGetLastError();
}

}  // namespace sem
