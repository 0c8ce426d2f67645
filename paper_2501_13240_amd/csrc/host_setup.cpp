// Host-side setup: GLL quadrature and the gather-scatter numbering.
//
// GLL (the nodal basis and quadrature of Sec. 2.2): interior nodes are the
// roots of P_N', found here by Newton's method on P_N' itself with P_N'' from
// Legendre's equation (1 - x^2) P'' = 2 x P' - N (N+1) P, started at the
// Chebyshev-Gauss-Lobatto points; weights 2 / (N (N+1) P_N(x)^2); derivative
// matrix D_ij = l_j'(x_i) = P_N(x_i) / (P_N(x_j) (x_i - x_j)) off the diagonal,
// -N(N+1)/4 and +N(N+1)/4 in the corners and 0 elsewhere on the diagonal.
//
// Numbering: local points are visited in ascending local index; each global
// id gets a dense index at its first visit ("first-touch" order).  Free
// indices put the nodes with a single local copy (element interiors) first
// and the shared ones after them, each class in first-touch order, so the
// unique vectors of the solver follow the element order of the mesh, the
// operator's gathers and direct stores run over contiguous stretches, and
// the segmented sum covers one contiguous range.  Segments list the local
// copies of each node in ascending order (counting sort, O(n_L)).
#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>

#include "common.hpp"

namespace sem {

static void legendre_all(int N, double x, double& p, double& dp) {
  double pm1 = 1.0, pc = x;
  if (N == 0) {
    p = 1.0;
    dp = 0.0;
    return;
  }
  for (int m = 1; m < N; ++m) {
    const double pn = ((2.0 * m + 1.0) * x * pc - m * pm1) / (m + 1.0);
    pm1 = pc;
    pc = pn;
  }
  p = pc;
  // (1 - x^2) P_N' = N (P_{N-1} - x P_N), valid for |x| < 1
  dp = N * (pm1 - x * pc) / (1.0 - x * x);
}

sem_status host_gll(int N, double* xi_out, double* rho_out, double* D_out) {
  if (N < 1 || N > kMaxOrder) return fail(SEM_EINVAL, "N must be in [1, 10]");
  const int n1 = N + 1;
  double xi[kMaxOrder + 1], pn[kMaxOrder + 1];
  xi[0] = -1.0;
  xi[N] = 1.0;
  const double pi = 3.14159265358979323846;
  for (int j = 1; j < N; ++j) {
    double x = -std::cos(pi * j / N);
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre_all(N, x, p, dp);
      const double d2p = (2.0 * x * dp - N * (N + 1.0) * p) / (1.0 - x * x);
      const double step = dp / d2p;
      x -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    xi[j] = x;
  }
  // exact mirror symmetry
  for (int j = 0; j <= N / 2; ++j) {
    const double a = 0.5 * (xi[N - j] - xi[j]);
    xi[j] = -a;
    xi[N - j] = a;
  }
  if (N % 2 == 0) xi[N / 2] = 0.0;
  for (int j = 0; j < n1; ++j) {
    double p, dp;
    if (j == 0 || j == N) {
      p = (j == 0 && (N % 2)) ? -1.0 : 1.0;  // P_N(+-1) = (+-1)^N
    } else {
      legendre_all(N, xi[j], p, dp);
    }
    pn[j] = p;
  }
  if (xi_out)
    for (int j = 0; j < n1; ++j) xi_out[j] = xi[j];
  if (rho_out)
    for (int j = 0; j < n1; ++j) rho_out[j] = 2.0 / (N * (N + 1.0) * pn[j] * pn[j]);
  if (D_out) {
    for (int i = 0; i < n1; ++i)
      for (int j = 0; j < n1; ++j)
        D_out[i * n1 + j] = (i == j) ? 0.0 : pn[i] / (pn[j] * (xi[i] - xi[j]));
    D_out[0] = -N * (N + 1.0) / 4.0;
    D_out[N * n1 + N] = N * (N + 1.0) / 4.0;
  }
  return SEM_OK;
}

sem_status build_numbering(int N, int64_t E, const int64_t* gid, const uint8_t* dirichlet,
                           HostNumbering& out) {
  if (N < 1 || N > kMaxOrder) return fail(SEM_EINVAL, "N must be in [1, 10]");
  if (E < 1) return fail(SEM_EINVAL, "E must be >= 1");
  if (!gid) return fail(SEM_EINVAL, "gid is NULL");
  const int64_t P = (int64_t)(N + 1) * (N + 1) * (N + 1);
  if (E > (int64_t)0x7fffffff / P) return fail(SEM_EINVAL, "E*(N+1)^3 must be < 2^31");
  const int64_t nL = E * P;

  int64_t gmin = gid[0], gmax = gid[0];
  for (int64_t q = 0; q < nL; ++q) {
    gmin = std::min(gmin, gid[q]);
    gmax = std::max(gmax, gid[q]);
  }
  if (gmin < 0) return fail(SEM_EINVAL, "gid must be >= 0");

  // dense unique index in first-touch order
  std::vector<int32_t> uidx(nL);
  int64_t nu = 0;
  if (gmax < std::max<int64_t>(4 * nL, 1 << 20)) {
    std::vector<int32_t> tab((size_t)gmax + 1, -1);
    for (int64_t q = 0; q < nL; ++q) {
      int32_t& t = tab[(size_t)gid[q]];
      if (t < 0) t = (int32_t)nu++;
      uidx[q] = t;
    }
  } else {
    std::vector<int32_t> order(nL);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return gid[a] < gid[b]; });
    // groups of equal gid; first element of each group = its first touch
    std::vector<int32_t> first;  // first-touch local index per group
    std::vector<int64_t> gstart;
    for (int64_t a = 0; a < nL; ++a)
      if (a == 0 || gid[order[a]] != gid[order[a - 1]]) {
        gstart.push_back(a);
        first.push_back(order[a]);
      }
    const int64_t ng = (int64_t)first.size();
    std::vector<int32_t> gorder(ng);
    std::iota(gorder.begin(), gorder.end(), 0);
    std::sort(gorder.begin(), gorder.end(), [&](int32_t a, int32_t b) { return first[a] < first[b]; });
    std::vector<int32_t> rank(ng);
    for (int64_t r = 0; r < ng; ++r) rank[gorder[r]] = (int32_t)r;
    for (int64_t gI = 0; gI < ng; ++gI) {
      const int64_t end = gI + 1 < ng ? gstart[gI + 1] : nL;
      for (int64_t a = gstart[gI]; a < end; ++a) uidx[order[a]] = rank[gI];
    }
    nu = ng;
  }

  std::vector<int32_t> mult(nu, 0), dcount(nu, 0);
  for (int64_t q = 0; q < nL; ++q) {
    mult[uidx[q]]++;
    if (dirichlet && dirichlet[q]) dcount[uidx[q]]++;
  }
  // free indices: nodes with one local copy first, then the shared ones,
  // each class in first-touch order (an element's own nodes are then one
  // contiguous run, and the shared ones a contiguous range)
  int64_t nfree = 0, nshared = 0, nsingle = 0;
  for (int64_t u = 0; u < nu; ++u) {
    if (dcount[u] != 0 && dcount[u] != mult[u])
      return fail(SEM_EINVAL, "Dirichlet flag differs between copies of global node " +
                                  std::to_string(u));
    if (dcount[u] == 0 && mult[u] == 1) ++nsingle;
  }
  std::vector<int32_t> fidx(nu, -1), sidx(nu, -1);
  int64_t next_single = 0, next_shared = nsingle;
  for (int64_t u = 0; u < nu; ++u) {
    if (dcount[u] == 0) {
      fidx[u] = (int32_t)(mult[u] == 1 ? next_single++ : next_shared++);
      ++nfree;
    }
    if (mult[u] > 1) sidx[u] = (int32_t)nshared++;
  }

  out.n_unique = nu;
  out.n_free = nfree;
  out.n_single = nsingle;
  out.n_shared = nshared;
  out.lmap.assign(nL, -1);
  out.fseg.assign(nfree + 1, 0);
  out.gseg.assign(nshared + 1, 0);
  out.dlist.clear();
  for (int64_t q = 0; q < nL; ++q) {
    const int32_t u = uidx[q];
    out.lmap[q] = fidx[u];
    if (fidx[u] >= 0) out.fseg[fidx[u] + 1]++;
    else out.dlist.push_back((int32_t)q);
    if (sidx[u] >= 0) out.gseg[sidx[u] + 1]++;
  }
  for (int64_t f = 0; f < nfree; ++f) out.fseg[f + 1] += out.fseg[f];
  for (int64_t s = 0; s < nshared; ++s) out.gseg[s + 1] += out.gseg[s];
  out.fperm.assign(out.fseg[nfree], 0);
  out.gperm.assign(out.gseg[nshared], 0);
  std::vector<int32_t> fcur(out.fseg.begin(), out.fseg.end() - 1);
  std::vector<int32_t> gcur(out.gseg.begin(), out.gseg.end() - 1);
  for (int64_t q = 0; q < nL; ++q) {
    const int32_t u = uidx[q];
    if (fidx[u] >= 0) out.fperm[fcur[fidx[u]]++] = (int32_t)q;
    if (sidx[u] >= 0) out.gperm[gcur[sidx[u]]++] = (int32_t)q;
  }
  return SEM_OK;
}

}  // namespace sem
