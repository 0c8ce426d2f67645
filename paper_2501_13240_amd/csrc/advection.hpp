// Convective term of the Boussinesq equations (internal): the element
// contributions C_e(u) f = sum_q phi_i w_q detJ_q u(x_q) . grad f(x_q) of
// the advection of temperature and velocity (Sec. 4.1), on the GLL nodes
// (collocation) or on floor(3(N+1)/2) Gauss-Legendre points per direction
// (over-integration, the 3/2 rule).
#pragma once

#include "common.hpp"

namespace sem {

// one quadrature rule's factors on a mesh
struct AdvRule {
  int q1 = 0;             // points per direction
  DevBuf mats64, mats32;  // J [q1][n], JD = J D [q1][n], J^T [n][q1]
  DevBuf G64, G32;        // [E][9][q1^3]: w detJ dr_a/dx_d in slot 3 a + d
};

// points per direction of a rule (0: collocation, 1: 3/2 rule)
int adv_points(int N, int rule);

// the rule's points x and weights w on [-1, 1] (ascending) and the
// interpolation J [q1][N+1] from the GLL nodes to them (the identity for
// collocation)
sem_status host_adv_rule(int N, int rule, double* x, double* w, double* J);

// G <- the factors of every element from xyz (DEVICE [E][P][3]); mats as in
// AdvRule (FP64), w1 the 1-D weights (DEVICE, q1); G32 (nullable) its FP32
// copy; *bad (DEVICE, zeroed by the caller) counts points with detJ <= 0
hipError_t launch_adv_geometry(const sem_mesh* m, int q1, const double* mats, const double* w1,
                               const double* xyz, double* G, float* G32, int* bad,
                               hipStream_t s);

// out[k][e] = C_e(u) f[k] for every element and each of nf fields: u DEVICE
// [3][E][P], f and out [nf][E][P]; rule 0 reads D (DEVICE [n][n]) and G
// [E][9][P], rule 1 mats and G [E][9][q1^3]
template <typename T>
hipError_t launch_advect(const sem_mesh* m, int rule, int nf, const T* mats, const T* D,
                         const T* G, const T* u, const T* f, T* out, hipStream_t s);

}  // namespace sem
