// Host side of the p-multigrid hierarchy: GLL-to-GLL interpolation and the
// coarse-order mesh on the same hexahedra.
//
// A coarse node is identified across elements by the mesh entity it lies on
// and its position there, with the entity named by fine global ids (so
// periodicity, expressed by equal ids, carries over):
//   vertex       the fine id of the corner;
//   edge         the ids of its two ends, smaller first, and the position
//                counted from that end;
//   face         three of its corners taken in a canonical order (the
//                smallest id, then its adjacent corner with the smaller id,
//                then the other adjacent corner) and the position measured
//                from the first along the two face axes in that order;
//   interior     new per element.
// Two elements that share an entity see the same corner ids at the same
// physical corners, so they derive the same key whatever their orientation.
#include <cstring>
#include <unordered_map>

#include "pmg.hpp"

namespace sem {

sem_status host_interp_matrix(int n_from, int n_to, double* M) {
  if (n_from < 1 || n_from > kMaxOrder || n_to < 1 || n_to > kMaxOrder)
    return fail(SEM_EINVAL, "interpolation orders must be in [1, 10]");
  double xf[kMaxOrder + 1], xt[kMaxOrder + 1], wb[kMaxOrder + 1];
  sem_status st;
  if ((st = host_gll(n_from, xf, nullptr, nullptr)) || (st = host_gll(n_to, xt, nullptr, nullptr)))
    return st;
  const int nf = n_from + 1, nt = n_to + 1;
  // barycentric weights of the source nodes
  for (int j = 0; j < nf; ++j) {
    double p = 1.0;
    for (int k = 0; k < nf; ++k)
      if (k != j) p *= xf[j] - xf[k];
    wb[j] = 1.0 / p;
  }
  for (int i = 0; i < nt; ++i) {
    double* row = M + (size_t)i * nf;
    int hit = -1;
    for (int j = 0; j < nf; ++j)
      if (xt[i] == xf[j]) hit = j;
    if (hit >= 0) {
      for (int j = 0; j < nf; ++j) row[j] = (j == hit) ? 1.0 : 0.0;
      continue;
    }
    double sum = 0.0;
    for (int j = 0; j < nf; ++j) {
      row[j] = wb[j] / (xt[i] - xf[j]);
      sum += row[j];
    }
    for (int j = 0; j < nf; ++j) row[j] /= sum;
  }
  return SEM_OK;
}

namespace {

struct EntityKey {
  int64_t a, b, c;
  int32_t kind, p, q;
  bool operator==(const EntityKey& o) const {
    return a == o.a && b == o.b && c == o.c && kind == o.kind && p == o.p && q == o.q;
  }
};
struct EntityKeyHash {
  size_t operator()(const EntityKey& k) const {
    uint64_t h = 0x9e3779b97f4a7c15ull;
    auto mix = [&](uint64_t v) {
      h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    };
    mix((uint64_t)k.a);
    mix((uint64_t)k.b);
    mix((uint64_t)k.c);
    mix(((uint64_t)(uint32_t)k.kind << 40) ^ ((uint64_t)(uint32_t)k.p << 20) ^ (uint32_t)k.q);
    return (size_t)h;
  }
};

// (M x M x M) on one element block: in n_in^3 -> out n_out^3, ijk order
void tensor3(const double* M, int n_in, int n_out, const double* in, double* out,
             std::vector<double>& t1, std::vector<double>& t2) {
  t1.assign((size_t)n_in * n_in * n_out, 0.0);
  t2.assign((size_t)n_in * n_out * n_out, 0.0);
  for (int k = 0; k < n_in; ++k)
    for (int j = 0; j < n_in; ++j)
      for (int a = 0; a < n_out; ++a) {
        double s = 0.0;
        for (int i = 0; i < n_in; ++i) s += M[a * n_in + i] * in[(k * n_in + j) * n_in + i];
        t1[(k * n_in + j) * n_out + a] = s;
      }
  for (int k = 0; k < n_in; ++k)
    for (int b = 0; b < n_out; ++b)
      for (int a = 0; a < n_out; ++a) {
        double s = 0.0;
        for (int j = 0; j < n_in; ++j) s += M[b * n_in + j] * t1[(k * n_in + j) * n_out + a];
        t2[(k * n_out + b) * n_out + a] = s;
      }
  for (int c = 0; c < n_out; ++c)
    for (int b = 0; b < n_out; ++b)
      for (int a = 0; a < n_out; ++a) {
        double s = 0.0;
        for (int k = 0; k < n_in; ++k) s += M[c * n_in + k] * t2[(k * n_out + b) * n_out + a];
        out[(c * n_out + b) * n_out + a] = s;
      }
}

}  // namespace

sem_status host_coarse_mesh(int N, int64_t E, const int64_t* gid, const uint8_t* dir,
                            const double* xyz, int Nc, int64_t* gid_c, uint8_t* dir_c,
                            double* xyz_c) {
  if (N < 2 || N > kMaxOrder || Nc < 1 || Nc >= N)
    return fail(SEM_EINVAL, "coarse order must satisfy 1 <= Nc < N <= 10");
  if (E < 1 || !gid || !gid_c) return fail(SEM_EINVAL, "E >= 1 and gid arrays are required");
  if ((dir == nullptr) != (dir_c == nullptr))
    return fail(SEM_EINVAL, "Dirichlet flags in and out must both be given or both be NULL");
  const int n = N + 1, nc = Nc + 1;
  const int64_t P = (int64_t)n * n * n, Pc = (int64_t)nc * nc * nc;

  if (xyz && xyz_c) {
    std::vector<double> I((size_t)nc * n), in(P), out(Pc), t1, t2;
    sem_status st = host_interp_matrix(N, Nc, I.data());
    if (st) return st;
    for (int64_t e = 0; e < E; ++e)
      for (int c = 0; c < 3; ++c) {
        for (int64_t q = 0; q < P; ++q) in[q] = xyz[(e * P + q) * 3 + c];
        tensor3(I.data(), n, nc, in.data(), out.data(), t1, t2);
        for (int64_t q = 0; q < Pc; ++q) xyz_c[(e * Pc + q) * 3 + c] = out[q];
      }
  }

  // fine index of a coarse coordinate: the ends map to the ends, interior
  // positions to the first interior fine position (same entity)
  auto fpos = [&](int c) { return c == 0 ? 0 : (c == Nc ? N : 1); };
  auto fidx = [&](int i, int j, int k) { return (int64_t)i + n * ((int64_t)j + n * k); };
  std::unordered_map<EntityKey, int64_t, EntityKeyHash> ids;
  ids.reserve((size_t)(E * (Pc - (int64_t)(nc - 2) * (nc - 2) * (nc - 2)) / 2 + 16));
  int64_t next = 0;
  for (int64_t e = 0; e < E; ++e) {
    const int64_t* g = gid + e * P;
    for (int k = 0; k < nc; ++k)
      for (int j = 0; j < nc; ++j)
        for (int i = 0; i < nc; ++i) {
          const int cc[3] = {i, j, k};
          const bool on[3] = {i == 0 || i == Nc, j == 0 || j == Nc, k == 0 || k == Nc};
          const int nb = (int)on[0] + (int)on[1] + (int)on[2];
          int fq[3] = {fpos(i), fpos(j), fpos(k)};
          int64_t id;
          if (nb == 0) {
            id = next++;
          } else {
            EntityKey key{};
            if (nb == 3) {
              key = EntityKey{g[fidx(fq[0], fq[1], fq[2])], 0, 0, 0, 0, 0};
            } else if (nb == 2) {
              const int d = on[0] ? (on[1] ? 2 : 1) : 0;  // direction along the edge
              int q0[3] = {fq[0], fq[1], fq[2]}, q1[3] = {fq[0], fq[1], fq[2]};
              q0[d] = 0;
              q1[d] = N;
              const int64_t g0 = g[fidx(q0[0], q0[1], q0[2])], g1 = g[fidx(q1[0], q1[1], q1[2])];
              if (g0 == g1) return fail(SEM_EINVAL, "a mesh edge whose two ends share a global id");
              const int t = cc[d];
              key = g0 < g1 ? EntityKey{g0, g1, 0, 1, t, 0} : EntityKey{g1, g0, 0, 1, Nc - t, 0};
            } else {
              const int d = on[0] ? 0 : (on[1] ? 1 : 2);  // face normal
              const int d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
              int64_t cs[2][2];
              for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                  int q[3] = {fq[0], fq[1], fq[2]};
                  q[d1] = a ? N : 0;
                  q[d2] = b ? N : 0;
                  cs[a][b] = g[fidx(q[0], q[1], q[2])];
                }
              if (cs[0][0] == cs[0][1] || cs[0][0] == cs[1][0] || cs[0][0] == cs[1][1] ||
                  cs[0][1] == cs[1][0] || cs[0][1] == cs[1][1] || cs[1][0] == cs[1][1])
                return fail(SEM_EINVAL, "a mesh face whose corners share a global id");
              int oa = 0, ob = 0;
              for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                  if (cs[a][b] < cs[oa][ob]) {
                    oa = a;
                    ob = b;
                  }
              const int64_t n1c = cs[1 - oa][ob];  // neighbour across the d1 axis
              const int64_t n2c = cs[oa][1 - ob];  // neighbour across the d2 axis
              const int r1 = oa == 0 ? cc[d1] : Nc - cc[d1];
              const int r2 = ob == 0 ? cc[d2] : Nc - cc[d2];
              key = n1c < n2c ? EntityKey{cs[oa][ob], n1c, n2c, 2, r1, r2}
                              : EntityKey{cs[oa][ob], n2c, n1c, 2, r2, r1};
            }
            auto it = ids.find(key);
            if (it == ids.end()) {
              id = next++;
              ids.emplace(key, id);
            } else {
              id = it->second;
            }
          }
          const int64_t qc = e * Pc + i + (int64_t)nc * (j + (int64_t)nc * k);
          gid_c[qc] = id;
          if (dir_c) dir_c[qc] = nb > 0 ? dir[e * P + fidx(fq[0], fq[1], fq[2])] : 0;
        }
  }
  return SEM_OK;
}

}  // namespace sem
