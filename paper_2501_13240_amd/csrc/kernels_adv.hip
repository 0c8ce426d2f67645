// Convective term C_e(u) f on every element (the advection terms of the
// Boussinesq equations, Sec. 4.1).
//
// Over-integrated rule (M = floor(3(N+1)/2) Gauss points per direction), one
// element at a time per workgroup of four wavefronts:
//   1. each velocity component u_d is interpolated to the M^3 points,
//      (J x J x J) u_d, and folded into V_a = sum_d G_ad u_d (a = r, s, t);
//      the nine factors G_ad = w detJ dr_a/dx_d are streamed from HBM once;
//   2. the reference derivatives of f at the points, (J x J x JD) f,
//      (J x JD x J) f and (JD x J x J) f with JD = J D, give
//      c = sum_a V_a df/dr_a;
//   3. the test functions project back: out = (J^T x J^T x J^T) c.
// Every 1-D interpolation is a batch of 16-column tiles of a 16x16x4 MFMA
// product (the M x (N+1) matrix J fits one tile, N <= 10), staged through
// LDS; the last interpolation stage (along t) keeps its tile in registers,
// where V and c are formed, so no M^3 array of u or of the derivatives is
// ever stored.  The factors (9 M^3 values against 5 (N+1)^3 of fields) are
// most of the HBM traffic.  With one field the kernel reaches about half of
// the HBM peak: the factors of a pass can be requested only one pass ahead
// within the register budget, less than the loaded latency.  With several
// fields sharing V most of the work is MFMA products and LDS stages, at about
// a third of the matrix cores' peak (the stages' barrier and LDS latencies,
// at two workgroups per CU).
//
// Collocation (the GLL nodes themselves): one thread per node, derivative
// sums over LDS.
#include "advection.hpp"
#include "mfma_16x16x4.hpp"

namespace sem {
namespace {

// dst = A src along direction DIR of an [S2][S1][S0] array (index 0
// fastest); the extent along DIR changes from NI to NO.  A is NO x NI,
// passed as this lane's fragments a[s] = A[lane % 16][4 s + lane / 16].
// The columns of the product are the points of the other two directions,
// in storage order.
template <typename T, int S2, int S1, int S0, int NO, int DIR>
struct Ct {
  typedef typename Mm<T>::V V;
  static constexpr int NI = DIR == 0 ? S0 : DIR == 1 ? S1 : S2;
  static constexpr int NC = S2 * S1 * S0 / NI;
  static constexpr int NT = (NC + 15) / 16;
  static constexpr int KS = (NI + 3) / 4;
  static_assert(NI <= 16 && NO <= 16, "one MFMA tile per matrix");
  // address of (column c, index l along DIR) with extent L along DIR
  template <int L>
  static __device__ __forceinline__ int addr(int c, int l) {
    if constexpr (DIR == 0) return c * L + l;
    else if constexpr (DIR == 1) return (c / S0) * (L * S0) + l * S0 + c % S0;
    else return l * (S1 * S0) + c;
  }
  static __device__ __forceinline__ V tile(const T* __restrict__ src, const T* a, int t,
                                           int lane) {
    const int col = t * 16 + (lane & 15);
    const bool cv = col < NC;
    const int kk = lane >> 4;
    V acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int l = 4 * s + kk;
      const T b = (cv && l < NI) ? src[addr<NI>(cv ? col : 0, l)] : T(0);
      acc = Mm<T>::mma(a[s], b, acc);
    }
    return acc;
  }
  static __device__ __forceinline__ void store(T* __restrict__ dst, V acc, int t, int lane) {
    const int col = t * 16 + (lane & 15);
    if (col >= NC) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = Mm<T>::row(lane, r);
      if (row < NO) dst[addr<NO>(col, row)] = acc[r];
    }
  }
};

// this lane's fragments of the NO x NI row-major matrix A
template <typename T, int NO, int NI>
__device__ __forceinline__ void fragments(const T* __restrict__ A, T* a, int lane) {
  constexpr int KS = (NI + 3) / 4;
  const int row = lane & 15;
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int l = 4 * s + (lane >> 4);
    a[s] = (row < NO && l < NI) ? A[row * NI + l] : T(0);
  }
}

constexpr int kAdvWaves = 4;
constexpr int kAdvThreads = 64 * kAdvWaves;

// The interpolation stages of an order-N element to M points per direction.
template <int N, int M, typename T, int W = kAdvWaves>
struct Stages {
  static constexpr int n = N + 1, P = n * n * n, Q = M * M * M;
  typedef Ct<T, n, n, n, M, 0> I0;  // (n,n,n) -> (n,n,M)
  typedef Ct<T, n, n, M, M, 1> I1;  // (n,n,M) -> (n,M,M)
  typedef Ct<T, n, M, M, M, 2> I2;  // (n,M,M) -> (M,M,M)
  typedef Ct<T, M, M, M, n, 2> B2;  // (M,M,M) -> (n,M,M)
  typedef Ct<T, n, M, M, n, 1> B1;  // (n,M,M) -> (n,n,M)
  typedef Ct<T, n, n, M, n, 0> B0;  // (n,n,M) -> (n,n,n)
  static constexpr int KN = I0::KS, KM = B2::KS;
  static constexpr int TPW = (I2::NT + W - 1) / W;  // last-stage tiles per wave
  // LDS: the input block and the two first-stage outputs (later the M^3
  // array c and the (n,n,M) back-projection stage), and one (n,M,M) array
  static constexpr int IX = P + 2 * n * n * M;
  static constexpr int YS = n * M * M;
  static_assert(Q <= IX && P <= YS, "LDS regions");
};

// Tiles of a stage handled by this wavefront (t = wv, wv + kW, ...), unrolled.
#define FOR_TILES(C, ...)                                                               \
  _Pragma("unroll") for (int ti_ = 0; ti_ < (C::NT + kW - 1) / kW; ++ti_) {           \
    const int t = wv + ti_ * kW;                                                        \
    if (t < C::NT) { __VA_ARGS__; }                                                     \
  }

// Wavefronts per workgroup of the dealiased kernel: the faster of four and
// eight, measured per order and precision on meshes of 14-16 thousand
// elements.  Eight halve each wave's last-stage tiles, and with them its V
// accumulators and prefetched factors: FP64 from N = 8 on then runs two waves
// per SIMD instead of one (1.3-1.6x faster at N = 8..10), FP64 at N = 5, 6
// gains 13-20 % and FP32 at N = 6 8 %.  FP64 at N = 7 and FP32 at the other
// orders are faster with four waves, which keep two workgroups per CU; at
// N <= 4 the stages have too few tiles for eight waves.
template <int N, typename T>
constexpr int adv_waves() {
  return (sizeof(T) == 8 ? (N == 5 || N == 6 || N >= 8) : N == 6) ? 8 : kAdvWaves;
}

// Persistent: workgroup b processes elements b, b + grid, ...  The factors a
// pass consumes are requested one pass ahead (the first pass's during the
// previous element's field passes and projections), into the registers the
// previous pass has just consumed, so the factor stream stays in flight
// while the matrix cores interpolate.  V is formed once per element and
// applied to each of the nf fields f[k] (stride E P, like u).
template <int N, typename T>
__global__ __launch_bounds__((64 * adv_waves<N, T>())) void adv_dealias_kernel(
    int64_t E, int nf, const T* __restrict__ mats, const T* __restrict__ G,
    const T* __restrict__ u, int64_t ustride, const T* __restrict__ f, T* __restrict__ out) {
  constexpr int M = (3 * (N + 1)) / 2;
  constexpr int kW = adv_waves<N, T>(), kThreads = 64 * kW;
  typedef Stages<N, M, T, kW> S;
  typedef typename S::I0 I0;
  typedef typename S::I1 I1;
  typedef typename S::I2 I2;
  typedef typename S::B2 B2;
  typedef typename S::B1 B1;
  typedef typename S::B0 B0;
  typedef typename Mm<T>::V V;
  constexpr int n = S::n, P = S::P, Q = S::Q, TPW = S::TPW;
  // the four input blocks and the first-stage outputs; later c and the
  // (n,n,M) projection stage
  constexpr int R0 = 4 * P + 2 * n * n * M;
  static_assert(Q <= R0, "c fits the first region");
  // FP64: the f pass forms its three (n,M,M) arrays in one phase when they
  // fit beside the rest with two workgroups per CU (two barriers per field
  // instead of six; measured 3.5 % faster with four fields at N = 7).  FP32
  // keeps one array: the larger LDS and register footprint cost it a wave
  // per SIMD (27 % slower)
  constexpr bool kMerge = sizeof(T) == 8 && (R0 + 3 * S::YS) * sizeof(T) <= 80 * 1024;
  __shared__ T sR[R0];
  __shared__ T sY[kMerge ? 3 * S::YS : S::YS];
  T* sIn = sR;  // u_x, u_y, u_z, f
  T* sX0 = sR + 4 * P;
  T* sX1 = sX0 + n * n * M;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  T aJ[S::KN], aJD[S::KN], aJT[S::KM];
  fragments<T, M, n>(mats, aJ, lane);
  fragments<T, M, n>(mats + M * n, aJD, lane);
  fragments<T, n, M>(mats + 2 * M * n, aJT, lane);
  // this lane's point in each of its last-stage tiles (-1: none)
  int goff[TPW][4];
#pragma unroll
  for (int ti = 0; ti < TPW; ++ti) {
    const int t = wv + ti * kW;
    const int col = t * 16 + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = Mm<T>::row(lane, r);
      goff[ti][r] = (t < I2::NT && row < M && col < M * M) ? row * M * M + col : -1;
    }
  }
  T g[TPW][3][4];  // G_ad of pass d at those points
  auto fetch = [&](int64_t ee, int d) {
    const T* Gd = G + (ee * 9 + d) * Q;
#pragma unroll
    for (int ti = 0; ti < TPW; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int a = 0; a < 3; ++a)
          g[ti][a][r] = goff[ti][r] >= 0 ? Gd[3 * a * Q + goff[ti][r]] : T(0);
  };
  int64_t e = blockIdx.x;
  if (e < E) fetch(e, 0);
  for (; e < E; e += gridDim.x) {
    const int64_t en = e + gridDim.x;
    for (int q = threadIdx.x; q < 4 * P; q += kThreads) {
      const int d = q / P, p = q - d * P;
      sIn[q] = d < 3 ? u[d * ustride + e * P + p] : f[e * P + p];
    }
    __syncthreads();

    // 1. V_a = sum_d G_ad (J x J x J) u_d, held in the last stage's tiles
    V Va[TPW][3];
#pragma unroll
    for (int ti = 0; ti < TPW; ++ti)
#pragma unroll
      for (int a = 0; a < 3; ++a) Va[ti][a] = V{T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      FOR_TILES(I0, I0::store(sX0, I0::tile(sIn + d * P, aJ, t, lane), t, lane));
      __syncthreads();
      FOR_TILES(I1, I1::store(sY, I1::tile(sX0, aJ, t, lane), t, lane));
      __syncthreads();
#pragma unroll
      for (int ti = 0; ti < TPW; ++ti) {
        const int t = wv + ti * kW;
        if (t < I2::NT) {
          const V ui = I2::tile(sY, aJ, t, lane);
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int r = 0; r < 4; ++r) Va[ti][a][r] += g[ti][a][r] * ui[r];
        }
      }
      if (d < 2) fetch(e, d + 1);
      else if (en < E) fetch(en, 0);
    }

    // every field k advected by the same V
    for (int k = 0; k < nf; ++k) {
      if (k > 0) {
        for (int q = threadIdx.x; q < P; q += kThreads)
          sIn[3 * P + q] = f[k * ustride + e * P + q];
        __syncthreads();
      }
      // 2. c = sum_a V_a df/dr_a: r (J x J x JD), s (J x JD x J), t (JD x J x J)
      FOR_TILES(I0, I0::store(sX0, I0::tile(sIn + 3 * P, aJ, t, lane), t, lane);
                I0::store(sX1, I0::tile(sIn + 3 * P, aJD, t, lane), t, lane));
      __syncthreads();
      V c[TPW];
#pragma unroll
      for (int ti = 0; ti < TPW; ++ti) c[ti] = V{T(0), T(0), T(0), T(0)};
      if constexpr (kMerge) {
        FOR_TILES(I1, I1::store(sY, I1::tile(sX1, aJ, t, lane), t, lane);
                  I1::store(sY + S::YS, I1::tile(sX0, aJD, t, lane), t, lane);
                  I1::store(sY + 2 * S::YS, I1::tile(sX0, aJ, t, lane), t, lane));
        __syncthreads();
#pragma unroll
        for (int ti = 0; ti < TPW; ++ti) {
          const int t = wv + ti * kW;
          if (t < I2::NT) {
            // one derivative tile live at a time (the scheduler would
            // otherwise hoist all of them and halve the occupancy)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const V fa = I2::tile(sY + a * S::YS, a == 2 ? aJD : aJ, t, lane);
#pragma unroll
              for (int r = 0; r < 4; ++r) c[ti][r] += Va[ti][a][r] * fa[r];
              __builtin_amdgcn_sched_barrier(0);
            }
          }
        }
        // (the c stores below touch sR only, whose arrays the phase above read
        // before the barrier)
      } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const T* src = a == 0 ? sX1 : sX0;
          const T* a1 = a == 1 ? aJD : aJ;
          const T* a2 = a == 2 ? aJD : aJ;
          FOR_TILES(I1, I1::store(sY, I1::tile(src, a1, t, lane), t, lane));
          __syncthreads();
#pragma unroll
          for (int ti = 0; ti < TPW; ++ti) {
            const int t = wv + ti * kW;
            if (t < I2::NT) {
              const V fa = I2::tile(sY, a2, t, lane);
#pragma unroll
              for (int r = 0; r < 4; ++r) c[ti][r] += Va[ti][a][r] * fa[r];
            }
          }
          __syncthreads();
        }
      }
      // c into the first region (its inputs and first-stage arrays are dead)
      T* sC = sR;
#pragma unroll
      for (int ti = 0; ti < TPW; ++ti) {
        const int t = wv + ti * kW;
        if (t < I2::NT) I2::store(sC, c[ti], t, lane);
      }
      __syncthreads();

      // 3. out = (J^T x J^T x J^T) c
      FOR_TILES(B2, B2::store(sY, B2::tile(sC, aJT, t, lane), t, lane));
      __syncthreads();
      FOR_TILES(B1, B1::store(sR, B1::tile(sY, aJT, t, lane), t, lane));
      __syncthreads();
      FOR_TILES(B0, B0::store(out + k * ustride + e * P, B0::tile(sR, aJT, t, lane), t, lane));
      __syncthreads();  // sR is restaged next
    }
  }
}

template <int N, typename T>
__global__ __launch_bounds__(kAdvThreads) void adv_colloc_kernel(
    int nf, const T* __restrict__ D, const T* __restrict__ G, const T* __restrict__ u,
    int64_t ustride, const T* __restrict__ f, T* __restrict__ out) {
  constexpr int n = N + 1, P = n * n * n, PT = (P + kAdvThreads - 1) / kAdvThreads;
  __shared__ T sF[P];
  __shared__ T sD[n * n];
  const int64_t e = blockIdx.x;
  for (int q = threadIdx.x; q < n * n; q += kAdvThreads) sD[q] = D[q];
  // V_a = sum_d G_ad u_d at this thread's nodes
  const T* Ge = G + e * 9 * P;
  T V[PT][3];
#pragma unroll
  for (int j = 0; j < PT; ++j) {
    const int q = threadIdx.x + j * kAdvThreads;
#pragma unroll
    for (int a = 0; a < 3; ++a) V[j][a] = T(0);
    if (q < P)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const T ud = u[d * ustride + e * P + q];
#pragma unroll
        for (int a = 0; a < 3; ++a) V[j][a] += Ge[(3 * a + d) * P + q] * ud;
      }
  }
  for (int k = 0; k < nf; ++k) {
    if (k > 0) __syncthreads();  // the previous field's sums are done with sF
    for (int q = threadIdx.x; q < P; q += kAdvThreads) sF[q] = f[k * ustride + e * P + q];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      const int q = threadIdx.x + j * kAdvThreads;
      if (q >= P) continue;
      const int i = q % n, jj = (q / n) % n, kk = q / (n * n);
      T fr = T(0), fs = T(0), ft = T(0);
#pragma unroll
      for (int l = 0; l < n; ++l) {
        fr += sD[i * n + l] * sF[(kk * n + jj) * n + l];
        fs += sD[jj * n + l] * sF[(kk * n + l) * n + i];
        ft += sD[kk * n + l] * sF[(l * n + jj) * n + i];
      }
      out[k * ustride + e * P + q] = V[j][0] * fr + V[j][1] * fs + V[j][2] * ft;
    }
  }
}

// dX[e][3 c + a] = dx_c/dr_a at the rule's points: the reference gradient of
// each coordinate, by the same stages as f in the dealiased kernel
template <int N, int M>
__global__ __launch_bounds__(kAdvThreads) void adv_metric_kernel(const double* __restrict__ mats,
                                                                 const double* __restrict__ xyz,
                                                                 double* __restrict__ dX) {
  typedef Stages<N, M, double> S;
  constexpr int n = S::n, P = S::P, Q = S::Q;
  __shared__ double sIX[S::IX];
  __shared__ double sY[S::YS];
  double* sIn = sIX;
  double* sX0 = sIX + P;
  double* sX1 = sX0 + n * n * M;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t e = blockIdx.x;
  double aJ[S::KN], aJD[S::KN];
  fragments<double, M, n>(mats, aJ, lane);
  fragments<double, M, n>(mats + M * n, aJD, lane);
  for (int cc = 0; cc < 3; ++cc) {
    for (int q = threadIdx.x; q < P; q += kAdvThreads) sIn[q] = xyz[(e * P + q) * 3 + cc];
    __syncthreads();
    for (int t = wv; t < S::I0::NT; t += kAdvWaves) {
      S::I0::store(sX0, S::I0::tile(sIn, aJ, t, lane), t, lane);
      S::I0::store(sX1, S::I0::tile(sIn, aJD, t, lane), t, lane);
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double* src = a == 0 ? sX1 : sX0;
      const double* a1 = a == 1 ? aJD : aJ;
      const double* a2 = a == 2 ? aJD : aJ;
      for (int t = wv; t < S::I1::NT; t += kAdvWaves)
        S::I1::store(sY, S::I1::tile(src, a1, t, lane), t, lane);
      __syncthreads();
      double* dst = dX + (e * 9 + 3 * cc + a) * Q;
      for (int t = wv; t < S::I2::NT; t += kAdvWaves)
        S::I2::store(dst, S::I2::tile(sY, a2, t, lane), t, lane);
      __syncthreads();
    }
  }
}

// G_ad = w detJ dr_a/dx_d = w adj(dx/dr)_ad in place of dx_c/dr_a, per point
__global__ void adv_metric_finish(int64_t E, int q1, const double* __restrict__ w1,
                                  double* __restrict__ G, float* __restrict__ G32,
                                  int* __restrict__ bad) {
  const int64_t Q = (int64_t)q1 * q1 * q1;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= E * Q) return;
  const int64_t e = idx / Q, q = idx % Q;
  const int i = (int)(q % q1), j = (int)((q / q1) % q1), k = (int)(q / ((int64_t)q1 * q1));
  double* g = G + e * 9 * Q + q;
  double m[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < 3; ++a) m[c][a] = g[(3 * c + a) * Q];
  double adj[3][3];  // adj[a][d] = det * (dr_a/dx_d)
  adj[0][0] = m[1][1] * m[2][2] - m[1][2] * m[2][1];
  adj[0][1] = m[0][2] * m[2][1] - m[0][1] * m[2][2];
  adj[0][2] = m[0][1] * m[1][2] - m[0][2] * m[1][1];
  adj[1][0] = m[1][2] * m[2][0] - m[1][0] * m[2][2];
  adj[1][1] = m[0][0] * m[2][2] - m[0][2] * m[2][0];
  adj[1][2] = m[0][2] * m[1][0] - m[0][0] * m[1][2];
  adj[2][0] = m[1][0] * m[2][1] - m[1][1] * m[2][0];
  adj[2][1] = m[0][1] * m[2][0] - m[0][0] * m[2][1];
  adj[2][2] = m[0][0] * m[1][1] - m[0][1] * m[1][0];
  const double det = m[0][0] * adj[0][0] + m[0][1] * adj[1][0] + m[0][2] * adj[2][0];
  if (!(det > 0.0)) atomicAdd(bad, 1);
  const double W = w1[i] * w1[j] * w1[k];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double v = W * adj[a][d];
      g[(3 * a + d) * Q] = v;
      if (G32) G32[e * 9 * Q + (3 * a + d) * Q + q] = (float)v;
    }
}

template <int N, typename T>
hipError_t run_advect(const sem_mesh* m, int rule, int nf, const T* mats, const T* D, const T* G,
                      const T* u, const T* f, T* out, hipStream_t s) {
  const int64_t ustride = m->E * (int64_t)m->P;
  if (rule == 0) {
    hipLaunchKernelGGL((adv_colloc_kernel<N, T>), dim3((unsigned)m->E), dim3(kAdvThreads), 0, s,
                       nf, D, G, u, ustride, f, out);
    return hipGetLastError();
  }
  // persistent grid: twice the resident workgroups (measured best of 1x, 2x)
  static const int per_cu = [] {
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, adv_dealias_kernel<N, T>,
                                                     64 * adv_waves<N, T>(),
                                                     0) != hipSuccess || v <= 0)
      v = 1;
    return v;
  }();
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  int64_t grid = 2 * (int64_t)cus * per_cu;
  if (grid > m->E) grid = m->E;
  hipLaunchKernelGGL((adv_dealias_kernel<N, T>), dim3((unsigned)grid), dim3(64 * adv_waves<N, T>()), 0, s,
                     m->E, nf, mats, G, u, ustride, f, out);
  return hipGetLastError();
}

template <int N>
hipError_t run_metric(const sem_mesh* m, int q1, const double* mats, const double* xyz,
                      double* dX, hipStream_t s) {
  constexpr int Md = (3 * (N + 1)) / 2;
  if (q1 == N + 1)
    hipLaunchKernelGGL((adv_metric_kernel<N, N + 1>), dim3((unsigned)m->E), dim3(kAdvThreads), 0,
                       s, mats, xyz, dX);
  else if (q1 == Md)
    hipLaunchKernelGGL((adv_metric_kernel<N, Md>), dim3((unsigned)m->E), dim3(kAdvThreads), 0, s,
                       mats, xyz, dX);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

hipError_t launch_adv_geometry(const sem_mesh* m, int q1, const double* mats, const double* w1,
                               const double* xyz, double* G, float* G32, int* bad,
                               hipStream_t s) {
  hipError_t err;
  switch (m->N) {
    case 1: err = run_metric<1>(m, q1, mats, xyz, G, s); break;
    case 2: err = run_metric<2>(m, q1, mats, xyz, G, s); break;
    case 3: err = run_metric<3>(m, q1, mats, xyz, G, s); break;
    case 4: err = run_metric<4>(m, q1, mats, xyz, G, s); break;
    case 5: err = run_metric<5>(m, q1, mats, xyz, G, s); break;
    case 6: err = run_metric<6>(m, q1, mats, xyz, G, s); break;
    case 7: err = run_metric<7>(m, q1, mats, xyz, G, s); break;
    case 8: err = run_metric<8>(m, q1, mats, xyz, G, s); break;
    case 9: err = run_metric<9>(m, q1, mats, xyz, G, s); break;
    case 10: err = run_metric<10>(m, q1, mats, xyz, G, s); break;
    default: return hipErrorInvalidValue;
  }
  if (err != hipSuccess) return err;
  const int64_t total = m->E * (int64_t)q1 * q1 * q1;
  const int64_t blocks = (total + 255) / 256;
  hipLaunchKernelGGL(adv_metric_finish, dim3((unsigned)blocks), dim3(256), 0, s, m->E, q1, w1, G,
                     G32, bad);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_advect(const sem_mesh* m, int rule, int nf, const T* mats, const T* D,
                         const T* G, const T* u, const T* f, T* out, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  switch (m->N) {
    case 1: return run_advect<1, T>(m, rule, nf, mats, D, G, u, f, out, s);
    case 2: return run_advect<2, T>(m, rule, nf, mats, D, G, u, f, out, s);
    case 3: return run_advect<3, T>(m, rule, nf, mats, D, G, u, f, out, s);
    case 4: return run_advect<4, T>(m, rule, nf, mats, D, G, u, f, out, s);
    case 5: return run_advect<5, T>(m, rule, nf, mats, D, G, u, f, out, s);
    case 6: return run_advect<6, T>(m, rule, nf, mats, D, G, u, f, out, s);
    case 7: return run_advect<7, T>(m, rule, nf, mats, D, G, u, f, out, s);
    case 8: return run_advect<8, T>(m, rule, nf, mats, D, G, u, f, out, s);
    case 9: return run_advect<9, T>(m, rule, nf, mats, D, G, u, f, out, s);
    case 10: return run_advect<10, T>(m, rule, nf, mats, D, G, u, f, out, s);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_advect<double>(const sem_mesh*, int, int, const double*,
                                          const double*, const double*, const double*,
                                          const double*, double*, hipStream_t);
template hipError_t launch_advect<float>(const sem_mesh*, int, int, const float*, const float*,
                                         const float*, const float*, const float*, float*,
                                         hipStream_t);

}  // namespace sem
