// Host side of the overlapping Schwarz smoother: subdomain maps and
// fast-diagonalisation factors.
//
// The subdomain of an element is its (N+1)^3 nodes plus, across each face,
// the neighbouring element's node layer one GLL step inside (the box of
// (N+3)^3 points, whose edge and corner points stay empty).  The local
// operator is separable on the box; along each direction its 1-D factors are
// the stiffness and mass of three 1-D GLL elements [left | element | right]
// with the mean lengths of the three elements, assembled and restricted to
// the N+3 central points (homogeneous Dirichlet beyond).  A side without a
// neighbour gets a decoupled ghost point, a Dirichlet face also decouples
// the element's own boundary point.  With A S = B S L and S^T B S = I the
// local inverse is (S x S x S) diag(1 / (l_i + l_j + l_k)) (S x S x S)^T.
#include <algorithm>
#include <array>
#include <cmath>
#include <unordered_map>

#include "schwarz.hpp"

namespace sem {
namespace {

struct FaceKey {
  std::array<int64_t, 4> c;  // sorted corner ids
  bool operator==(const FaceKey& o) const { return c == o.c; }
};
struct FaceKeyHash {
  size_t operator()(const FaceKey& k) const {
    uint64_t h = 0x9e3779b97f4a7c15ull;
    for (int64_t v : k.c) h ^= (uint64_t)v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};
struct FaceRef {
  int64_t e;
  int d, side;
};

// local index (i, j, k) -> offset, and the face point (a, b) of face (d, side)
inline int64_t lidx(int n, int i, int j, int k) { return i + (int64_t)n * (j + (int64_t)n * k); }
inline void face_point(int d, int side, int N, int a, int b, int q[3]) {
  const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
  q[d] = side ? N : 0;
  q[t0] = a;
  q[t1] = b;
}

// cyclic Jacobi eigenvalue iteration for a small symmetric matrix (row-major,
// overwritten): eigenvalues in w, eigenvectors in the columns of V
void sym_eigen(int n, double* a, double* w, double* V) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += a[i * n + j] * a[i * n + j];
        if (i != j) off += a[i * n + j] * a[i * n + j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[p * n + q];
        if (apq == 0.0) continue;
        const double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - s * akq;
          a[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - s * aqk;
          a[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < n; ++i) w[i] = a[i * n + i];
}

}  // namespace

sem_status extended_operator_1d(int N, double l_left, double l, double l_right, bool dir_lo,
                                bool dir_hi, double* A, double* B) {
  const int n = N + 1, nx = N + 3;
  double xi[kMaxOrder + 1], rho[kMaxOrder + 1], D[(kMaxOrder + 1) * (kMaxOrder + 1)];
  sem_status st = host_gll(N, xi, rho, D);
  if (st) return st;
  std::vector<double> K((size_t)n * n, 0.0);  // D^T diag(rho) D
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      double s = 0.0;
      for (int q = 0; q < n; ++q) s += D[q * n + a] * rho[q] * D[q * n + b];
      K[a * n + b] = s;
    }
  const bool has_l = l_left > 0.0, has_r = l_right > 0.0;
  const double len[3] = {has_l ? l_left : l, l, has_r ? l_right : l};
  std::fill(A, A + nx * nx, 0.0);
  std::fill(B, B + nx * nx, 0.0);
  // global 1-D node g in [0, 3N] of element el and local node a: g = el N + a;
  // the box keeps g = N-1 .. 2N+1 (box index g - (N-1))
  for (int el = 0; el < 3; ++el) {
    if ((el == 0 && !has_l) || (el == 2 && !has_r)) continue;  // no neighbour, no contribution
    for (int a = 0; a < n; ++a) {
      const int ga = el * N + a - (N - 1);
      if (ga < 0 || ga >= nx) continue;
      B[ga * nx + ga] += 0.5 * len[el] * rho[a];
      for (int b = 0; b < n; ++b) {
        const int gb = el * N + b - (N - 1);
        if (gb < 0 || gb >= nx) continue;
        A[ga * nx + gb] += (2.0 / len[el]) * K[a * n + b];
      }
    }
  }
  int dec[4], nd = 0;
  if (!has_l) dec[nd++] = 0;
  if (!has_r) dec[nd++] = N + 2;
  if (dir_lo) dec[nd++] = 1;
  if (dir_hi) dec[nd++] = N + 1;
  for (int t = 0; t < nd; ++t) {
    const int p = dec[t];
    for (int q = 0; q < nx; ++q) {
      A[p * nx + q] = A[q * nx + p] = 0.0;
      B[p * nx + q] = B[q * nx + p] = 0.0;
    }
    A[p * nx + p] = B[p * nx + p] = 1.0;
  }
  return SEM_OK;
}

sem_status build_schwarz(int N, int64_t E, const int64_t* gid, const uint8_t* dir,
                         const double* xyz, const int32_t* lmap, int64_t n_free,
                         SchwarzHost& out) {
  if (N < 1 || N > kMaxOrder || E < 1) return fail(SEM_EINVAL, "bad Schwarz mesh");
  const int n = N + 1, nx = N + 3;
  const int64_t P = (int64_t)n * n * n, PX = (int64_t)nx * nx * nx;

  // mean lengths along r, s, t from the corner vertices
  std::vector<double> len((size_t)E * 3, 0.0);
  for (int64_t e = 0; e < E; ++e) {
    const double* X = xyz + e * P * 3;
    auto dist = [&](int64_t p, int64_t q) {
      const double dx = X[q * 3] - X[p * 3], dy = X[q * 3 + 1] - X[p * 3 + 1],
                   dz = X[q * 3 + 2] - X[p * 3 + 2];
      return std::sqrt(dx * dx + dy * dy + dz * dz);
    };
    for (int a : {0, N})
      for (int b : {0, N}) {
        len[e * 3 + 0] += 0.25 * dist(lidx(n, 0, b, a), lidx(n, N, b, a));
        len[e * 3 + 1] += 0.25 * dist(lidx(n, b, 0, a), lidx(n, b, N, a));
        len[e * 3 + 2] += 0.25 * dist(lidx(n, b, a, 0), lidx(n, b, a, N));
      }
  }

  // faces named by their sorted corner ids
  auto face_key = [&](int64_t e, int d, int side, FaceKey& key) -> bool {
    int c = 0;
    for (int a : {0, N})
      for (int b : {0, N}) {
        int q[3];
        face_point(d, side, N, a, b, q);
        key.c[c++] = gid[e * P + lidx(n, q[0], q[1], q[2])];
      }
    std::sort(key.c.begin(), key.c.end());
    return key.c[0] != key.c[1] && key.c[1] != key.c[2] && key.c[2] != key.c[3];
  };
  std::unordered_map<FaceKey, std::vector<FaceRef>, FaceKeyHash> faces;
  faces.reserve((size_t)(E * 4));
  for (int64_t e = 0; e < E; ++e)
    for (int d = 0; d < 3; ++d)
      for (int side = 0; side < 2; ++side) {
        FaceKey k;
        if (!face_key(e, d, side, k))
          return fail(SEM_EINVAL, "Schwarz: a face whose corners share a global id");
        faces[k].push_back(FaceRef{e, d, side});
      }

  out.N = N;
  out.xmap.assign((size_t)(E * PX), -1);
  out.S.assign((size_t)(E * 3 * nx * nx), 0.0);
  out.lam.assign((size_t)(E * 3 * nx), 0.0);
  std::vector<std::pair<int64_t, int>> fpts((size_t)n * n);  // (gid, index) of a neighbour face
  std::vector<double> A((size_t)nx * nx), Bm((size_t)nx * nx), C((size_t)nx * nx),
      V((size_t)nx * nx), w(nx);
  for (int64_t e = 0; e < E; ++e) {
    int32_t* xm = out.xmap.data() + e * PX;
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
          xm[lidx(nx, i + 1, j + 1, k + 1)] = lmap[e * P + lidx(n, i, j, k)];
    double nlen[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    bool dface[3][2] = {{false, false}, {false, false}, {false, false}};
    for (int d = 0; d < 3; ++d)
      for (int side = 0; side < 2; ++side) {
        if (dir) {
          bool all = true;
          for (int a = 0; a < n && all; ++a)
            for (int b = 0; b < n && all; ++b) {
              int q[3];
              face_point(d, side, N, a, b, q);
              all = dir[e * P + lidx(n, q[0], q[1], q[2])] != 0;
            }
          dface[d][side] = all;
        }
        FaceKey key;
        face_key(e, d, side, key);
        const auto& refs = faces[key];
        const FaceRef* nb = nullptr;
        for (const auto& f : refs)
          if (!(f.e == e && f.d == d && f.side == side)) {
            if (nb) return fail(SEM_EINVAL, "Schwarz: a face shared by more than two elements");
            nb = &f;
          }
        if (!nb) continue;
        nlen[d][side] = len[nb->e * 3 + nb->d];
        // neighbour face points by global id
        for (int a = 0; a < n; ++a)
          for (int b = 0; b < n; ++b) {
            int q[3];
            face_point(nb->d, nb->side, N, a, b, q);
            fpts[a * n + b] = {gid[nb->e * P + lidx(n, q[0], q[1], q[2])], a * n + b};
          }
        std::sort(fpts.begin(), fpts.end());
        for (int a = 0; a < n; ++a)
          for (int b = 0; b < n; ++b) {
            int q[3];
            face_point(d, side, N, a, b, q);
            const int64_t g = gid[e * P + lidx(n, q[0], q[1], q[2])];
            auto it = std::lower_bound(fpts.begin(), fpts.end(), std::make_pair(g, -1));
            if (it == fpts.end() || it->first != g)
              return fail(SEM_EINVAL, "Schwarz: neighbouring faces do not share their nodes");
            int qn[3];
            face_point(nb->d, nb->side, N, it->second / n, it->second % n, qn);
            qn[nb->d] += nb->side ? -1 : 1;  // one step into the neighbour
            int qe[3] = {q[0] + 1, q[1] + 1, q[2] + 1};
            qe[d] = side ? N + 2 : 0;
            xm[lidx(nx, qe[0], qe[1], qe[2])] = lmap[nb->e * P + lidx(n, qn[0], qn[1], qn[2])];
          }
      }
    for (int d = 0; d < 3; ++d) {
      sem_status st = extended_operator_1d(N, nlen[d][0], len[e * 3 + d], nlen[d][1], dface[d][0],
                                           dface[d][1], A.data(), Bm.data());
      if (st) return st;
      // B diagonal: C = B^-1/2 A B^-1/2, C V = V L, S = B^-1/2 V
      for (int p = 0; p < nx; ++p)
        for (int q = 0; q < nx; ++q)
          C[p * nx + q] = A[p * nx + q] / std::sqrt(Bm[p * nx + p] * Bm[q * nx + q]);
      sym_eigen(nx, C.data(), w.data(), V.data());
      double* S = out.S.data() + (e * 3 + d) * nx * nx;
      double* L = out.lam.data() + (e * 3 + d) * nx;
      for (int p = 0; p < nx; ++p) {
        L[p] = w[p];
        for (int q = 0; q < nx; ++q) S[p * nx + q] = V[p * nx + q] / std::sqrt(Bm[p * nx + p]);
      }
    }
  }

  // copies of each free node among the box points, ascending (deterministic sums)
  out.xseg.assign((size_t)n_free + 1, 0);
  for (int64_t a = 0; a < E * PX; ++a)
    if (out.xmap[a] >= 0) out.xseg[out.xmap[a] + 1]++;
  for (int64_t f = 0; f < n_free; ++f) out.xseg[f + 1] += out.xseg[f];
  out.xperm.assign((size_t)out.xseg[n_free], 0);
  std::vector<int32_t> cur(out.xseg.begin(), out.xseg.end() - 1);
  for (int64_t a = 0; a < E * PX; ++a)
    if (out.xmap[a] >= 0) out.xperm[cur[out.xmap[a]]++] = (int32_t)a;
  return SEM_OK;
}

}  // namespace sem
