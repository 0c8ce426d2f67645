// Element operator kernels for gfx950 (wave64).
//
// A_L(k) u = sum_ab D_a^T diag(k G_ab) D_b u + h2 B u on every element: the
// matrix-free tensor-product operator of Sec. 2.2, whose leading work is
// dense (N+1)x(N+1) contractions identical for all elements.
//
// Mapping: one thread per (i, j) column of an element, the column's N+1
// values along t held in registers.  For N = 7 an element is exactly one
// wavefront (8 x 8 columns = 64 lanes).  The r- and s-contractions read the
// current k-plane from LDS; the t-contraction runs in registers with D[k][l]
// read as a wave-uniform (scalar) value; the transposed contractions reuse the
// same plane buffers.  Per local point the kernel streams u (8 B), the six
// geometric factors (48 B, planar layout [E][6][P] so each factor of a plane
// is one contiguous 8*(N+1)^2-byte run) and w (8 B): 64 B in FP64.
#include "common.hpp"

namespace sem {
namespace {

constexpr int pick_epb(int n1) {
  // elements per workgroup: fill whole wavefronts with (N+1)^2 columns each
  return n1 == 8 ? 1 : n1 == 10 ? 5 : n1 == 11 ? 4 : (256 / (n1 * n1) > 0 ? 256 / (n1 * n1) : 1);
}

template <int N>
struct Shape {
  static constexpr int n1 = N + 1;
  static constexpr int P2 = n1 * n1;
  static constexpr int P = P2 * n1;
  static constexpr int EPB = pick_epb(n1);
  static constexpr int BT = ((EPB * P2 + 63) / 64) * 64;
  static constexpr int LD = (n1 % 2 == 0) ? n1 + 1 : n1;  // padded LDS row (bank spread)
};

template <int N, typename T, bool GATHER>
__global__ __launch_bounds__(Shape<N>::BT) void ax_kernel(
    const T* __restrict__ u, const int32_t* __restrict__ lmap, T* __restrict__ w,
    const T* __restrict__ kf, const T h2, const T* __restrict__ G, const T* __restrict__ B,
    const T* __restrict__ D, const int64_t E, const int32_t* __restrict__ skip) {
  using S = Shape<N>;
  constexpr int n1 = S::n1, P2 = S::P2, P = S::P, EPB = S::EPB, LD = S::LD;
  if (skip && *skip) return;  // uniform over the grid
  __shared__ T su[EPB][n1 * LD];
  __shared__ T svr[EPB][n1 * LD];
  __shared__ T svs[EPB][n1 * LD];

  const int t = threadIdx.x;
  const int slot = t / P2;
  const int col = t - slot * P2;
  const int i = col % n1, j = col / n1;
  const int64_t e = (int64_t)blockIdx.x * EPB + slot;
  const bool lds_ok = slot < EPB;
  const bool active = lds_ok && e < E;
  const int ss = lds_ok ? slot : 0;

  T Dri[n1], Drj[n1], Dci[n1], Dcj[n1];
#pragma unroll
  for (int l = 0; l < n1; ++l) {
    Dri[l] = D[i * n1 + l];
    Drj[l] = D[j * n1 + l];
    Dci[l] = D[l * n1 + i];
    Dcj[l] = D[l * n1 + j];
  }

  const int64_t base = e * P + col;
  T ureg[n1];
#pragma unroll
  for (int k = 0; k < n1; ++k) {
    T v = T(0);
    if (active) {
      const int64_t idx = base + k * P2;
      if constexpr (GATHER) {
        const int32_t lm = lmap[idx];
        v = lm >= 0 ? u[lm] : T(0);
      } else {
        v = u[idx];
      }
    }
    ureg[k] = v;
  }

  const T* g = G + e * 6 * P + col;
  T wreg[n1], vt[n1];
#pragma unroll
  for (int k = 0; k < n1; ++k) {
    if (lds_ok) su[ss][j * LD + i] = ureg[k];
    __syncthreads();
    T ur = T(0), us = T(0), ut = T(0);
    if (lds_ok) {
#pragma unroll
      for (int l = 0; l < n1; ++l) {
        ur += Dri[l] * su[ss][j * LD + l];
        us += Drj[l] * su[ss][l * LD + i];
      }
    }
#pragma unroll
    for (int l = 0; l < n1; ++l) ut += D[k * n1 + l] * ureg[l];
    T vr = T(0), vs = T(0), vtt = T(0);
    if (active) {
      const int o = k * P2;
      const T grr = g[o], grs = g[P + o], grt = g[2 * P + o];
      const T gss = g[3 * P + o], gst = g[4 * P + o], gtt = g[5 * P + o];
      vr = grr * ur + grs * us + grt * ut;
      vs = grs * ur + gss * us + gst * ut;
      vtt = grt * ur + gst * us + gtt * ut;
      if (kf) {
        const T kq = kf[base + o];
        vr *= kq;
        vs *= kq;
        vtt *= kq;
      }
    }
    vt[k] = vtt;
    if (lds_ok) {
      svr[ss][j * LD + i] = vr;
      svs[ss][j * LD + i] = vs;
    }
    __syncthreads();
    T acc = T(0);
    if (lds_ok) {
#pragma unroll
      for (int l = 0; l < n1; ++l) acc += Dci[l] * svr[ss][j * LD + l] + Dcj[l] * svs[ss][l * LD + i];
    }
    wreg[k] = acc;
  }

  if (active) {
#pragma unroll
    for (int k = 0; k < n1; ++k) {
      T acc = wreg[k];
#pragma unroll
      for (int l = 0; l < n1; ++l) acc += D[l * n1 + k] * vt[l];
      if (h2 != T(0)) acc += h2 * B[base + k * P2] * ureg[k];
      w[base + k * P2] = acc;
    }
  }
}

// kbar_q = sum_ab (D_a wbar)_q G_ab,q (D_b u)_q: the derivative of the
// operator in k contracted with a cotangent (same column mapping).
template <int N>
__global__ __launch_bounds__(Shape<N>::BT) void kbar_kernel(
    const double* __restrict__ u, const double* __restrict__ wb, double* __restrict__ kbar,
    const double* __restrict__ G, const double* __restrict__ D, const int64_t E) {
  using S = Shape<N>;
  constexpr int n1 = S::n1, P2 = S::P2, P = S::P, EPB = S::EPB, LD = S::LD;
  __shared__ double su[EPB][n1 * LD];
  __shared__ double sw[EPB][n1 * LD];
  const int t = threadIdx.x;
  const int slot = t / P2;
  const int col = t - slot * P2;
  const int i = col % n1, j = col / n1;
  const int64_t e = (int64_t)blockIdx.x * EPB + slot;
  const bool lds_ok = slot < EPB;
  const bool active = lds_ok && e < E;
  const int ss = lds_ok ? slot : 0;

  double Dri[n1], Drj[n1];
#pragma unroll
  for (int l = 0; l < n1; ++l) {
    Dri[l] = D[i * n1 + l];
    Drj[l] = D[j * n1 + l];
  }
  const int64_t base = e * P + col;
  double ucol[n1], wcol[n1];
#pragma unroll
  for (int k = 0; k < n1; ++k) {
    ucol[k] = active ? u[base + k * P2] : 0.0;
    wcol[k] = active ? wb[base + k * P2] : 0.0;
  }
  const double* g = G + e * 6 * P + col;
#pragma unroll
  for (int k = 0; k < n1; ++k) {
    if (lds_ok) {
      su[ss][j * LD + i] = ucol[k];
      sw[ss][j * LD + i] = wcol[k];
    }
    __syncthreads();
    double ur = 0, us = 0, ut = 0, wr = 0, ws = 0, wt = 0;
    if (lds_ok) {
#pragma unroll
      for (int l = 0; l < n1; ++l) {
        ur += Dri[l] * su[ss][j * LD + l];
        us += Drj[l] * su[ss][l * LD + i];
        wr += Dri[l] * sw[ss][j * LD + l];
        ws += Drj[l] * sw[ss][l * LD + i];
      }
    }
#pragma unroll
    for (int l = 0; l < n1; ++l) {
      ut += D[k * n1 + l] * ucol[l];
      wt += D[k * n1 + l] * wcol[l];
    }
    if (active) {
      const int o = k * P2;
      const double grr = g[o], grs = g[P + o], grt = g[2 * P + o];
      const double gss = g[3 * P + o], gst = g[4 * P + o], gtt = g[5 * P + o];
      const double vr = grr * ur + grs * us + grt * ut;
      const double vs = grs * ur + gss * us + gst * ut;
      const double vt = grt * ur + gst * us + gtt * ut;
      kbar[base + o] = wr * vr + ws * vs + wt * vt;
    }
    __syncthreads();
  }
}

template <typename T>
__global__ void mass_kernel(int64_t n, const T* __restrict__ B, const T* __restrict__ u,
                            T* __restrict__ w) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x)
    w[q] = B[q] * u[q];
}

template <int N, typename T>
hipError_t run_ax(const sem_mesh* m, const T* u, const int32_t* lmap, T* w, const T* k, T h2,
                  const T* G, const T* B, const T* D, hipStream_t s, const int32_t* skip) {
  using S = Shape<N>;
  const int64_t grid = (m->E + S::EPB - 1) / S::EPB;
  if (lmap)
    hipLaunchKernelGGL((ax_kernel<N, T, true>), dim3((unsigned)grid), dim3(S::BT), 0, s, u, lmap,
                       w, k, h2, G, B, D, m->E, skip);
  else
    hipLaunchKernelGGL((ax_kernel<N, T, false>), dim3((unsigned)grid), dim3(S::BT), 0, s, u,
                       lmap, w, k, h2, G, B, D, m->E, skip);
  return hipGetLastError();
}

template <int N>
hipError_t run_kbar(const sem_mesh* m, const double* u, const double* wb, double* kbar,
                    hipStream_t s) {
  using S = Shape<N>;
  const int64_t grid = (m->E + S::EPB - 1) / S::EPB;
  hipLaunchKernelGGL((kbar_kernel<N>), dim3((unsigned)grid), dim3(S::BT), 0, s, u, wb, kbar,
                     m->G64.as<double>(), m->D64.as<double>(), m->E);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_ax(const sem_mesh* m, const T* u, const int32_t* lmap, T* w, const T* k, T h2,
                     const T* G, const T* B, const T* D, hipStream_t s, const int32_t* skip) {
  switch (m->N) {
    case 1: return run_ax<1, T>(m, u, lmap, w, k, h2, G, B, D, s, skip);
    case 2: return run_ax<2, T>(m, u, lmap, w, k, h2, G, B, D, s, skip);
    case 3: return run_ax<3, T>(m, u, lmap, w, k, h2, G, B, D, s, skip);
    case 4: return run_ax<4, T>(m, u, lmap, w, k, h2, G, B, D, s, skip);
    case 5: return run_ax<5, T>(m, u, lmap, w, k, h2, G, B, D, s, skip);
    case 6: return run_ax<6, T>(m, u, lmap, w, k, h2, G, B, D, s, skip);
    case 7: return run_ax<7, T>(m, u, lmap, w, k, h2, G, B, D, s, skip);
    case 8: return run_ax<8, T>(m, u, lmap, w, k, h2, G, B, D, s, skip);
    case 9: return run_ax<9, T>(m, u, lmap, w, k, h2, G, B, D, s, skip);
    case 10: return run_ax<10, T>(m, u, lmap, w, k, h2, G, B, D, s, skip);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_ax<double>(const sem_mesh*, const double*, const int32_t*, double*,
                                      const double*, double, const double*, const double*,
                                      const double*, hipStream_t, const int32_t*);
template hipError_t launch_ax<float>(const sem_mesh*, const float*, const int32_t*, float*,
                                     const float*, float, const float*, const float*,
                                     const float*, hipStream_t, const int32_t*);

hipError_t launch_ax_kbar(const sem_mesh* m, const double* u, const double* wbar, double* kbar,
                          hipStream_t s) {
  switch (m->N) {
    case 1: return run_kbar<1>(m, u, wbar, kbar, s);
    case 2: return run_kbar<2>(m, u, wbar, kbar, s);
    case 3: return run_kbar<3>(m, u, wbar, kbar, s);
    case 4: return run_kbar<4>(m, u, wbar, kbar, s);
    case 5: return run_kbar<5>(m, u, wbar, kbar, s);
    case 6: return run_kbar<6>(m, u, wbar, kbar, s);
    case 7: return run_kbar<7>(m, u, wbar, kbar, s);
    case 8: return run_kbar<8>(m, u, wbar, kbar, s);
    case 9: return run_kbar<9>(m, u, wbar, kbar, s);
    case 10: return run_kbar<10>(m, u, wbar, kbar, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_mass(int64_t n, const T* B, const T* u, T* w, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((n + kVecBlock - 1) / kVecBlock, 8192);
  hipLaunchKernelGGL((mass_kernel<T>), dim3((unsigned)std::max<int64_t>(blocks, 1)),
                     dim3(kVecBlock), 0, s, n, B, u, w);
  return hipGetLastError();
}
template hipError_t launch_mass<double>(int64_t, const double*, const double*, double*,
                                        hipStream_t);
template hipError_t launch_mass<float>(int64_t, const float*, const float*, float*, hipStream_t);

}  // namespace sem
