// Overlapping Schwarz smoother with fast-diagonalisation local solves
// (internal): the smoother the p-multigrid cycle of Sec. 2.2 accelerates.
#pragma once

#include <vector>

#include "common.hpp"

namespace sem {

// host factors of one mesh level
struct SchwarzHost {
  int N = 0;
  std::vector<int32_t> xmap;        // [E][(N+3)^3] free index of each box point or -1
  std::vector<double> S;            // [E][3][(N+3)^2] S_d row-major (rows: box points)
  std::vector<double> lam;          // [E][3][N+3] eigenvalues
  std::vector<int32_t> xseg, xperm; // box points of each free node, ascending
};

// 1-D extended stiffness A and mass B (row-major (N+3)^2): three GLL elements
// of lengths l_left, l, l_right (a length <= 0: no neighbour on that side)
// restricted to the N+3 central points; dir_lo / dir_hi: Dirichlet at the
// element's own end points
sem_status extended_operator_1d(int N, double l_left, double l, double l_right, bool dir_lo,
                                bool dir_hi, double* A, double* B);

// subdomain maps and factors from a mesh description and its free numbering
// (lmap: free index of each local point or -1)
sem_status build_schwarz(int N, int64_t E, const int64_t* gid, const uint8_t* dir,
                         const double* xyz, const int32_t* lmap, int64_t n_free,
                         SchwarzHost& out);

// device copy of the factors, in both precisions, with a box buffer
struct SchwarzDev {
  int nx = 0;
  DevBuf xmap, xseg, xperm, S64, S32, L64, L32, box64, box32;
};

// box_out[e] = A~_e^{-1} R_e r (one element per workgroup, matrix cores)
template <typename T>
hipError_t launch_fdm(const SchwarzDev& X, int64_t E, const T* r, T* box_out,
                      const int32_t* skip, hipStream_t s);

}  // namespace sem
