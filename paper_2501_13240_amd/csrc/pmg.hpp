// p-multigrid hierarchy (internal).
//
// Sec. 2.2 names the default preconditioner of the pressure solve: p-multigrid
// with fourth-kind Chebyshev acceleration of the smoother, most of it in FP32.
// Levels are orders N_0 = N > N_1 > ... > N_L on the same hexahedra; each
// coarse level is a mesh of its own (coordinates interpolated from the fine
// element maps, unknowns identified through the fine global ids), so every
// level runs the same operator, Jacobi and Chebyshev code as the fine one.
#pragma once

#include <vector>

#include "common.hpp"
#include "schwarz.hpp"
#include "solver.hpp"

namespace sem {

struct PmgLevel {
  sem_mesh* m = nullptr;  // level mesh (level 0: the fine mesh, not owned)
  bool owned = false;
  int N = 0;
  // interpolation from level l+1 to level l, (N_l+1) x (N_{l+1}+1) row-major,
  // and its transpose (restriction), in both precisions
  DevBuf J64, J32, JT64, JT32;
  // free vectors of this level: r (input), x (output), t, u, w (scratch),
  // d, rk, q (Chebyshev-Schwarz smoothing)
  DevBuf r64, x64, t64, u64, w64, d64, k64v, q64, r32, x32, t32, u32, w32, d32, k32v, q32;
  SchwarzDev sch;          // Schwarz factors (levels that smooth, Schwarz smoother only)
  double sch_rho = 0.0;    // cached bound of the Schwarz-preconditioned operator (k == NULL)
  double sch_rho_h2 = -1.0;
  DevBuf Ik64;  // interpolation from level 0's GLL points to this level's (levels >= 1)
  DevBuf k64;   // k interpolated to this level (levels >= 1, per solve)
  // per solve
  Op<double> op64;
  Op<float> op32;
  const double* dinv64 = nullptr;
  const float* dinv32 = nullptr;
  double rho_hat = 0.0;  // Chebyshev bound of this level
};

struct Pmg {
  std::vector<PmgLevel> lv;
  int smooth_order = 4;
  int coarse_iters = 30;
  int smoother = 1;  // 0 Jacobi, 1 overlapping Schwarz
  template <typename T>
  T* vec(PmgLevel& L, int which);  // 0 r, 1 x, 2 t, 3 u, 4 w, 5 d, 6 rk, 7 q
};

void pmg_destroy(Pmg* p);

// host: 1-D Lagrange interpolation from the order-n_from GLL nodes to the
// order-n_to GLL nodes, M is (n_to+1) x (n_from+1) row-major
sem_status host_interp_matrix(int n_from, int n_to, double* M);
// host: coordinates, global ids and Dirichlet flags of the order-Nc mesh on
// the hexahedra of an order-N mesh (dir / dir_c may be null together)
sem_status host_coarse_mesh(int N, int64_t E, const int64_t* gid, const uint8_t* dir,
                            const double* xyz, int Nc, int64_t* gid_c, uint8_t* dir_c,
                            double* xyz_c);

// device: out_L = (M x M x M) applied to each element block (M: n_out x n_in,
// element blocks of n_in^3 and n_out^3 points).  mode 0: the input is a
// local vector in_L; mode 1: gathered from the free vector in_f through
// lmap (0 at Dirichlet copies); mode 2: as 1, divided by the number of local
// copies of the free node (taken from seg).
template <typename T>
hipError_t launch_interp(int64_t E, int n_in, int n_out, const T* M, int mode, const T* in,
                         const int32_t* lmap, const int32_t* seg, T* out_L, const int32_t* skip,
                         hipStream_t s);

// One V-cycle z = V(r) on free vectors of level 0 (Tr: the caller's vector
// type, Tp: the arithmetic of the cycle).  Coupled to an enclosing flexible CG
// through `cg` exactly as the Chebyshev preconditioner is (convergence gate
// first, z.r and z.(w - mean_w) partials last); a stand-alone call passes an
// empty ChebCg.  The hierarchy must have been prepared for the solve's k, h2.
template <typename Tr, typename Tp>
sem_status pmg_precond(const sem_mesh* m, SolveWork& W, const Tr* r, Tr* z, const ChebCg& cg,
                       hipStream_t s, int* applies);

// The Schwarz smoother of one level as a flexible-CG preconditioner (for the
// Lanczos bound of the Schwarz-preconditioned operator): z = S r.
sem_status schwarz_precond(Pmg& P, int level, const double* r, double* z, const ChebCg& cg,
                           hipStream_t s);

}  // namespace sem
