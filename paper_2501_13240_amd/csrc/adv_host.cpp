// Host side of the convective term: the 1-D quadrature rules and the
// interpolation from the GLL nodes to them.
#include <cmath>

#include "advection.hpp"

namespace sem {

int adv_points(int N, int rule) { return rule == 0 ? N + 1 : (3 * (N + 1)) / 2; }

namespace {

// P_M(x) and P_M'(x) by the three-term recurrence
void legendre_pd(int M, double x, double& p, double& dp) {
  double pm1 = 1.0, pc = x;
  for (int k = 1; k < M; ++k) {
    const double pn = ((2.0 * k + 1.0) * x * pc - k * pm1) / (k + 1.0);
    pm1 = pc;
    pc = pn;
  }
  p = M == 0 ? 1.0 : pc;
  dp = M == 0 ? 0.0 : M * (x * pc - pm1) / (x * x - 1.0);
}

// Gauss-Legendre points (ascending) and weights: Newton's method on P_M from
// the Chebyshev-like first guesses cos(pi (i + 3/4) / (M + 1/2)), weights
// 2 / ((1 - x^2) P_M'(x)^2)
void gauss_legendre(int M, double* x, double* w) {
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < M; ++i) {
    double z = std::cos(pi * (i + 0.75) / (M + 0.5)), p, dp;
    for (int it = 0; it < 100; ++it) {
      legendre_pd(M, z, p, dp);
      const double step = p / dp;
      z -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    legendre_pd(M, z, p, dp);
    x[M - 1 - i] = z;
    w[M - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  // exact mirror symmetry
  for (int i = 0; i < M / 2; ++i) {
    const double a = 0.5 * (x[M - 1 - i] - x[i]), b = 0.5 * (w[i] + w[M - 1 - i]);
    x[i] = -a;
    x[M - 1 - i] = a;
    w[i] = w[M - 1 - i] = b;
  }
  if (M % 2) x[M / 2] = 0.0;
}

}  // namespace

sem_status host_adv_rule(int N, int rule, double* x, double* w, double* J) {
  if (N < 1 || N > kMaxOrder) return fail(SEM_EINVAL, "N must be in [1, 10]");
  if (rule != 0 && rule != 1) return fail(SEM_EINVAL, "rule must be 0 (collocation) or 1 (3/2 rule)");
  const int n = N + 1, q1 = adv_points(N, rule);
  double xg[kMaxOrder + 1], wg[kMaxOrder + 1];
  if (sem_status st = host_gll(N, xg, wg, nullptr)) return st;
  double xq[16], wq[16];
  if (rule == 0) {
    for (int i = 0; i < n; ++i) xq[i] = xg[i], wq[i] = wg[i];
  } else {
    gauss_legendre(q1, xq, wq);
  }
  if (x)
    for (int i = 0; i < q1; ++i) x[i] = xq[i];
  if (w)
    for (int i = 0; i < q1; ++i) w[i] = wq[i];
  if (J) {
    // barycentric form of the Lagrange basis of the GLL nodes
    double bw[kMaxOrder + 1];
    for (int j = 0; j < n; ++j) {
      double p = 1.0;
      for (int k = 0; k < n; ++k)
        if (k != j) p *= xg[j] - xg[k];
      bw[j] = 1.0 / p;
    }
    for (int i = 0; i < q1; ++i) {
      double* row = J + (size_t)i * n;
      int hit = -1;
      for (int j = 0; j < n; ++j)
        if (rule == 0 ? i == j : xq[i] == xg[j]) hit = j;
      if (hit >= 0) {
        for (int j = 0; j < n; ++j) row[j] = j == hit ? 1.0 : 0.0;
        continue;
      }
      double sum = 0.0;
      for (int j = 0; j < n; ++j) sum += (row[j] = bw[j] / (xq[i] - xg[j]));
      for (int j = 0; j < n; ++j) row[j] /= sum;
    }
  }
  return SEM_OK;
}

}  // namespace sem
