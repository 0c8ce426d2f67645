// Fast-diagonalisation local solves of the overlapping Schwarz smoother.
//
// One element per workgroup: the residual is gathered into the element's
// (N+3)^3 box through its subdomain map (0 at points outside the
// subdomain), transformed by S_r^T, S_s^T, S_t^T along the three directions,
// divided by l_r,i + l_s,j + l_t,k, transformed back by S_t, S_s, S_r, and
// written to the box buffer; a segmented sum over the box points of each
// free node completes z = sum_e R_e^T A~_e^{-1} R_e r.  Each 1-D transform of
// the box is a batch of 16-column tiles C = M X on the matrix cores (16x16x4
// MFMA in FP64 or FP32) with M = S or S^T of this element, read from LDS.
#include <algorithm>

#include "mfma_16x16x4.hpp"
#include "schwarz.hpp"

namespace sem {
namespace {

// one 16-column tile of dst = M src along direction DIR of an n^3 box
// ([k][j][i]); M = S^T (TRANS) or S, S row-major n x n in LDS
template <int n, typename T, int DIR, bool TRANS>
__device__ __forceinline__ void fdm_tile(const T* __restrict__ src, T* __restrict__ dst,
                                         const T* __restrict__ S, int tile, int lane) {
  constexpr int P2 = n * n, KS = (n + 3) / 4;
  const int col = tile * 16 + (lane & 15);
  const int kk = lane >> 4, mrow = lane & 15;
  const bool cval = col < P2;
  const int c1 = cval ? col / n : 0, c0 = cval ? col % n : 0;
  typename Mm<T>::V acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int l = 4 * s + kk;
    T a = T(0), b = T(0);
    if (mrow < n && l < n) a = TRANS ? S[l * n + mrow] : S[mrow * n + l];
    if (cval && l < n) {
      const int ad = DIR == 0 ? c1 * P2 + c0 * n + l : DIR == 1 ? c1 * P2 + l * n + c0 : l * P2 + col;
      b = src[ad];
    }
    acc = Mm<T>::mma(a, b, acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = Mm<T>::row(lane, r);
    if (cval && row < n) {
      const int ad =
          DIR == 0 ? c1 * P2 + c0 * n + row : DIR == 1 ? c1 * P2 + row * n + c0 : row * P2 + col;
      dst[ad] = acc[r];
    }
  }
}

// The same tile with this lane's fragments of M (one per k-step) already in
// registers: a transform loads them once for all of its tiles.
template <int n, typename T>
__device__ __forceinline__ void fdm_frag(const T* __restrict__ S, bool trans, int lane,
                                         T (&af)[(n + 3) / 4]) {
  constexpr int KS = (n + 3) / 4;
  const int kk = lane >> 4, mrow = lane & 15;
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int l = 4 * s + kk;
    af[s] = (mrow < n && l < n) ? (trans ? S[l * n + mrow] : S[mrow * n + l]) : T(0);
  }
}

template <int n, typename T, int DIR>
__device__ __forceinline__ void fdm_tile_f(const T* __restrict__ src, T* __restrict__ dst,
                                           const T (&af)[(n + 3) / 4], int tile, int lane) {
  constexpr int P2 = n * n, KS = (n + 3) / 4;
  const int col = tile * 16 + (lane & 15);
  const int kk = lane >> 4;
  const bool cval = col < P2;
  const int c1 = cval ? col / n : 0, c0 = cval ? col % n : 0;
  typename Mm<T>::V acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int l = 4 * s + kk;
    T b = T(0);
    if (cval && l < n) {
      const int ad = DIR == 0 ? c1 * P2 + c0 * n + l : DIR == 1 ? c1 * P2 + l * n + c0 : l * P2 + col;
      b = src[ad];
    }
    acc = Mm<T>::mma(af[s], b, acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = Mm<T>::row(lane, r);
    if (cval && row < n) {
      const int ad =
          DIR == 0 ? c1 * P2 + c0 * n + row : DIR == 1 ? c1 * P2 + row * n + c0 : row * P2 + col;
      dst[ad] = acc[r];
    }
  }
}

// wavefronts per workgroup of the one-element-per-workgroup kernel (n >= 9)
#ifndef SEM_FDM_WAVES
#define SEM_FDM_WAVES 4
#endif
constexpr int fdm_waves(int n) { return n >= 9 ? SEM_FDM_WAVES : 4; }
// persistent, software-pipelined local solves for n >= 9 (see fdm_pipe_kernel)
#ifndef SEM_FDM_PIPE
#define SEM_FDM_PIPE 1
#endif

// dst[q] = r[xmap[q]] (0 where xmap < 0) for q = t, t + NTHR, ... < P3: every
// map entry of this thread first, then every gather, so that no gather waits
// behind the map load of the thread's next point (measured 3-5 % faster
// p-multigrid solves on the 32^3, N = 9 cube)
template <int P3, int NTHR, typename T>
__device__ __forceinline__ void gather_box(const int32_t* __restrict__ xmap,
                                           const T* __restrict__ r, T* __restrict__ dst, int t) {
  constexpr int PPT = (P3 + NTHR - 1) / NTHR;
  int32_t gi[PPT];
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int q = t + s * NTHR;
    gi[s] = q < P3 ? xmap[q] : -1;
  }
  T rv[PPT];
#pragma unroll
  for (int s = 0; s < PPT; ++s) rv[s] = gi[s] >= 0 ? r[gi[s]] : T(0);
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int q = t + s * NTHR;
    if (q < P3) dst[q] = rv[s];
  }
}

template <int n, typename T, int NW>
__global__ __launch_bounds__(64 * NW) void fdm_kernel(const int32_t* __restrict__ xmap,
                                                          const T* __restrict__ S,
                                                          const T* __restrict__ lam,
                                                          const T* __restrict__ r,
                                                          T* __restrict__ out,
                                                          const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int P2 = n * n, P3 = P2 * n, NT = (P2 + 15) / 16, NTHR = 64 * NW;
  __shared__ T sA[P3];
  __shared__ T sB[P3];
  __shared__ T sS[3][P2];
  __shared__ T sL[3][n];
  const int64_t e = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  for (int q = t; q < 3 * P2; q += NTHR) (&sS[0][0])[q] = S[e * 3 * P2 + q];
  for (int q = t; q < 3 * n; q += NTHR) (&sL[0][0])[q] = lam[e * 3 * n + q];
  gather_box<P3, NTHR>(xmap + e * P3, r, sA, t);
  __syncthreads();
  for (int tile = wv; tile < NT; tile += NW) fdm_tile<n, T, 0, true>(sA, sB, sS[0], tile, lane);
  __syncthreads();
  for (int tile = wv; tile < NT; tile += NW) fdm_tile<n, T, 1, true>(sB, sA, sS[1], tile, lane);
  __syncthreads();
  for (int tile = wv; tile < NT; tile += NW) fdm_tile<n, T, 2, true>(sA, sB, sS[2], tile, lane);
  __syncthreads();
  for (int q = t; q < P3; q += NTHR) {
    const int a = q % n, b = (q / n) % n, c = q / P2;
    sB[q] = sB[q] / (sL[0][a] + sL[1][b] + sL[2][c]);
  }
  __syncthreads();
  for (int tile = wv; tile < NT; tile += NW) fdm_tile<n, T, 2, false>(sB, sA, sS[2], tile, lane);
  __syncthreads();
  for (int tile = wv; tile < NT; tile += NW) fdm_tile<n, T, 1, false>(sA, sB, sS[1], tile, lane);
  __syncthreads();
  for (int tile = wv; tile < NT; tile += NW) fdm_tile<n, T, 0, false>(sB, sA, sS[0], tile, lane);
  __syncthreads();
  for (int q = t; q < P3; q += NTHR) out[e * P3 + q] = sA[q];
}

// The same with a persistent grid: each workgroup walks the elements
// e = blockIdx.x, blockIdx.x + gridDim.x, ... and keeps the next element's
// loads in flight while it transforms the current one (subdomain-map loads
// during the first transform, then the residual gathers and the S and lam
// factors during the other five), so the gather latency no longer separates
// the transform phases of one workgroup.
template <int n, typename T, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(
    sizeof(T) == 4 ? 8 : 1))) void fdm_pipe_kernel(int64_t E,
                                                           const int32_t* __restrict__ xmap,
                                                           const T* __restrict__ S,
                                                           const T* __restrict__ lam,
                                                           const T* __restrict__ r,
                                                           T* __restrict__ out,
                                                           const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int P2 = n * n, P3 = P2 * n, NT = (P2 + 15) / 16, NTHR = 64 * NW;
  constexpr int NF = 3 * P2 + 3 * n;                  // S then lam of one element
  constexpr int PPT = (P3 + NTHR - 1) / NTHR, FPT = (NF + NTHR - 1) / NTHR;
  __shared__ T sA[P3];
  __shared__ T sB[P3];
  __shared__ T sF[NF];
  const T* sS0 = sF;
  const T* sS1 = sF + P2;
  const T* sS2 = sF + 2 * P2;
  const T* sL = sF + 3 * P2;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  int32_t gi[PPT];
  T rv[PPT], fv[FPT];
  T af[(n + 3) / 4];
  auto load_map = [&](int64_t e) {
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
      const int q = t + s * NTHR;
      gi[s] = q < P3 ? xmap[e * P3 + q] : -1;
    }
  };
  auto load_vals = [&](int64_t e) {
#pragma unroll
    for (int s = 0; s < PPT; ++s) rv[s] = gi[s] >= 0 ? r[gi[s]] : T(0);
#pragma unroll
    for (int s = 0; s < FPT; ++s) {
      const int f = t + s * NTHR;
      fv[s] = f < 3 * P2 ? S[e * 3 * P2 + f] : f < NF ? lam[e * 3 * n + (f - 3 * P2)] : T(0);
    }
  };
  int64_t e = blockIdx.x;
  if (e >= E) return;  // uniform over the workgroup
  load_map(e);
  load_vals(e);
  for (; e < E; e += gridDim.x) {
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
      const int q = t + s * NTHR;
      if (q < P3) sA[q] = rv[s];
    }
#pragma unroll
    for (int s = 0; s < FPT; ++s) {
      const int f = t + s * NTHR;
      if (f < NF) sF[f] = fv[s];
    }
    __syncthreads();
    const int64_t en = e + gridDim.x;
    const bool more = en < E;
    if (more) load_map(en);
    fdm_frag<n, T>(sS0, true, lane, af);
    for (int tile = wv; tile < NT; tile += NW) fdm_tile_f<n, T, 0>(sA, sB, af, tile, lane);
    __syncthreads();
    if (more) load_vals(en);
    fdm_frag<n, T>(sS1, true, lane, af);
    for (int tile = wv; tile < NT; tile += NW) fdm_tile_f<n, T, 1>(sB, sA, af, tile, lane);
    __syncthreads();
    fdm_frag<n, T>(sS2, true, lane, af);
    for (int tile = wv; tile < NT; tile += NW) fdm_tile_f<n, T, 2>(sA, sB, af, tile, lane);
    __syncthreads();
    for (int q = t; q < P3; q += NTHR) {
      const int a = q % n, b = (q / n) % n, c = q / P2;
      sB[q] = sB[q] / (sL[a] + sL[n + b] + sL[2 * n + c]);
    }
    __syncthreads();
    fdm_frag<n, T>(sS2, false, lane, af);
    for (int tile = wv; tile < NT; tile += NW) fdm_tile_f<n, T, 2>(sB, sA, af, tile, lane);
    __syncthreads();
    fdm_frag<n, T>(sS1, false, lane, af);
    for (int tile = wv; tile < NT; tile += NW) fdm_tile_f<n, T, 1>(sA, sB, af, tile, lane);
    __syncthreads();
    fdm_frag<n, T>(sS0, false, lane, af);
    for (int tile = wv; tile < NT; tile += NW) fdm_tile_f<n, T, 0>(sB, sA, af, tile, lane);
    __syncthreads();
    for (int q = t; q < P3; q += NTHR) out[e * P3 + q] = sA[q];
    __syncthreads();  // sA and sF are restaged for the next element
  }
}

// Small boxes (n <= 8, N <= 5): one wavefront per element, four elements per
// workgroup.  A wavefront's LDS operations complete in program order, so the
// six transforms need no workgroup barrier; a wavefront-scope fence between
// them keeps the compiler from reordering them.
constexpr int kFdmWaves = 4;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <int n, typename T>
__global__ __launch_bounds__(64 * kFdmWaves) void fdm_wave_kernel(
    int64_t E, const int32_t* __restrict__ xmap, const T* __restrict__ S,
    const T* __restrict__ lam, const T* __restrict__ r, T* __restrict__ out,
    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int P2 = n * n, P3 = P2 * n, NT = (P2 + 15) / 16;
  __shared__ T sA[kFdmWaves][P3];
  __shared__ T sB[kFdmWaves][P3];
  __shared__ T sS[kFdmWaves][3][P2];
  __shared__ T sL[kFdmWaves][3][n];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * kFdmWaves + w;
  if (e >= E) return;  // the whole wavefront (no workgroup barrier follows)
  T* A = sA[w];
  T* B = sB[w];
  T* Sw = &sS[w][0][0];
  T* Lw = &sL[w][0][0];
  for (int q = lane; q < 3 * P2; q += 64) Sw[q] = S[e * 3 * P2 + q];
  for (int q = lane; q < 3 * n; q += 64) Lw[q] = lam[e * 3 * n + q];
  gather_box<P3, 64>(xmap + e * P3, r, A, lane);
  wave_sync();
  for (int tile = 0; tile < NT; ++tile) fdm_tile<n, T, 0, true>(A, B, Sw, tile, lane);
  wave_sync();
  for (int tile = 0; tile < NT; ++tile) fdm_tile<n, T, 1, true>(B, A, Sw + P2, tile, lane);
  wave_sync();
  for (int tile = 0; tile < NT; ++tile) fdm_tile<n, T, 2, true>(A, B, Sw + 2 * P2, tile, lane);
  wave_sync();
  for (int q = lane; q < P3; q += 64) {
    const int a = q % n, b = (q / n) % n, c = q / P2;
    B[q] = B[q] / (Lw[a] + Lw[n + b] + Lw[2 * n + c]);
  }
  wave_sync();
  for (int tile = 0; tile < NT; ++tile) fdm_tile<n, T, 2, false>(B, A, Sw + 2 * P2, tile, lane);
  wave_sync();
  for (int tile = 0; tile < NT; ++tile) fdm_tile<n, T, 1, false>(A, B, Sw + P2, tile, lane);
  wave_sync();
  for (int tile = 0; tile < NT; ++tile) fdm_tile<n, T, 0, false>(B, A, Sw, tile, lane);
  wave_sync();
  for (int q = lane; q < P3; q += 64) out[e * P3 + q] = A[q];
}

// The small-box kernel on a persistent grid: each wavefront walks the
// elements w0, w0 + W, ... (W wavefronts in the grid) and keeps the next
// element's subdomain map (during the first transform), residual gathers and
// S, lam factors (during the others) in flight, as fdm_pipe_kernel does per
// workgroup; each transform's fragments of S are loaded once for its tiles.
template <int n, typename T>
__global__ __launch_bounds__(64 * kFdmWaves) void fdm_wave_pipe_kernel(
    int64_t E, const int32_t* __restrict__ xmap, const T* __restrict__ S,
    const T* __restrict__ lam, const T* __restrict__ r, T* __restrict__ out,
    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int P2 = n * n, P3 = P2 * n, NT = (P2 + 15) / 16;
  constexpr int NF = 3 * P2 + 3 * n;  // S then lam of one element
  constexpr int PPT = (P3 + 63) / 64, FPT = (NF + 63) / 64;
  __shared__ T sA[kFdmWaves][P3];
  __shared__ T sB[kFdmWaves][P3];
  __shared__ T sF[kFdmWaves][NF];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  T* A = sA[w];
  T* B = sB[w];
  T* F = sF[w];
  const int64_t nw = (int64_t)gridDim.x * kFdmWaves;
  int64_t e = (int64_t)blockIdx.x * kFdmWaves + w;
  if (e >= E) return;  // the whole wavefront (no workgroup barrier follows)
  int32_t gi[PPT];
  T rv[PPT], fv[FPT];
  T af[(n + 3) / 4];
  auto load_map = [&](int64_t el) {
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
      const int q = lane + 64 * s;
      gi[s] = q < P3 ? xmap[el * P3 + q] : -1;
    }
  };
  auto load_vals = [&](int64_t el) {
#pragma unroll
    for (int s = 0; s < PPT; ++s) rv[s] = gi[s] >= 0 ? r[gi[s]] : T(0);
#pragma unroll
    for (int s = 0; s < FPT; ++s) {
      const int f = lane + 64 * s;
      fv[s] = f < 3 * P2 ? S[el * 3 * P2 + f] : f < NF ? lam[el * 3 * n + (f - 3 * P2)] : T(0);
    }
  };
  load_map(e);
  load_vals(e);
  for (; e < E; e += nw) {
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
      const int q = lane + 64 * s;
      if (q < P3) A[q] = rv[s];
    }
#pragma unroll
    for (int s = 0; s < FPT; ++s) {
      const int f = lane + 64 * s;
      if (f < NF) F[f] = fv[s];
    }
    wave_sync();
    const int64_t en = e + nw;
    const bool more = en < E;
    if (more) load_map(en);
    fdm_frag<n, T>(F, true, lane, af);
    for (int tile = 0; tile < NT; ++tile) fdm_tile_f<n, T, 0>(A, B, af, tile, lane);
    wave_sync();
    if (more) load_vals(en);
    fdm_frag<n, T>(F + P2, true, lane, af);
    for (int tile = 0; tile < NT; ++tile) fdm_tile_f<n, T, 1>(B, A, af, tile, lane);
    wave_sync();
    fdm_frag<n, T>(F + 2 * P2, true, lane, af);
    for (int tile = 0; tile < NT; ++tile) fdm_tile_f<n, T, 2>(A, B, af, tile, lane);
    wave_sync();
    const T* L = F + 3 * P2;
    for (int q = lane; q < P3; q += 64) {
      const int a = q % n, b = (q / n) % n, c = q / P2;
      B[q] = B[q] / (L[a] + L[n + b] + L[2 * n + c]);
    }
    wave_sync();
    fdm_frag<n, T>(F + 2 * P2, false, lane, af);
    for (int tile = 0; tile < NT; ++tile) fdm_tile_f<n, T, 2>(B, A, af, tile, lane);
    wave_sync();
    fdm_frag<n, T>(F + P2, false, lane, af);
    for (int tile = 0; tile < NT; ++tile) fdm_tile_f<n, T, 1>(A, B, af, tile, lane);
    wave_sync();
    fdm_frag<n, T>(F, false, lane, af);
    for (int tile = 0; tile < NT; ++tile) fdm_tile_f<n, T, 0>(B, A, af, tile, lane);
    wave_sync();
    for (int q = lane; q < P3; q += 64) out[e * P3 + q] = A[q];
    wave_sync();  // A and F are restaged for the next element
  }
}

#ifndef SEM_FDM_WAVE_PIPE
#define SEM_FDM_WAVE_PIPE 1
#endif

template <int n, typename T>
hipError_t run_fdm(int64_t E, const int32_t* xmap, const T* S, const T* lam, const T* r, T* out,
                   const int32_t* skip, hipStream_t s) {
  if constexpr (n <= 8) {
#if SEM_FDM_WAVE_PIPE
    // persistent grid: the resident workgroups of the device, at most one
    // wavefront per element
    static int resident = 0;
    if (resident == 0) {
      int dev = 0, cus = 0, per_cu = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fdm_wave_pipe_kernel<n, T>,
                                                       64 * kFdmWaves, 0) != hipSuccess)
        return hipErrorUnknown;
      resident = std::max(1, cus * per_cu);
    }
    const int64_t grid = std::min<int64_t>((E + kFdmWaves - 1) / kFdmWaves, resident);
    hipLaunchKernelGGL((fdm_wave_pipe_kernel<n, T>), dim3((unsigned)grid), dim3(64 * kFdmWaves),
                       0, s, E, xmap, S, lam, r, out, skip);
#else
    const int64_t grid = (E + kFdmWaves - 1) / kFdmWaves;
    hipLaunchKernelGGL((fdm_wave_kernel<n, T>), dim3((unsigned)grid), dim3(64 * kFdmWaves), 0, s,
                       E, xmap, S, lam, r, out, skip);
#endif
  } else {
    constexpr int NW = fdm_waves(n);
#if SEM_FDM_PIPE
    // persistent grid: the resident workgroups of the device, at most one per element
    static int resident = 0;
    if (resident == 0) {
      int dev = 0, cus = 0, per_cu = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fdm_pipe_kernel<n, T, NW>,
                                                       64 * NW, 0) != hipSuccess)
        return hipErrorUnknown;
      resident = std::max(1, cus * per_cu);
    }
    const int64_t grid = std::min<int64_t>(E, resident);
    hipLaunchKernelGGL((fdm_pipe_kernel<n, T, NW>), dim3((unsigned)grid), dim3(64 * NW), 0, s, E,
                       xmap, S, lam, r, out, skip);
#else
    hipLaunchKernelGGL((fdm_kernel<n, T, NW>), dim3((unsigned)E), dim3(64 * NW), 0, s, xmap, S,
                       lam, r, out, skip);
#endif
  }
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_fdm(const SchwarzDev& X, int64_t E, const T* r, T* box_out,
                      const int32_t* skip, hipStream_t s) {
  const int32_t* xm = X.xmap.as<int32_t>();
  const T* S = sizeof(T) == 8 ? (const T*)X.S64.p : (const T*)X.S32.p;
  const T* L = sizeof(T) == 8 ? (const T*)X.L64.p : (const T*)X.L32.p;
  switch (X.nx) {
    case 4: return run_fdm<4, T>(E, xm, S, L, r, box_out, skip, s);
    case 5: return run_fdm<5, T>(E, xm, S, L, r, box_out, skip, s);
    case 6: return run_fdm<6, T>(E, xm, S, L, r, box_out, skip, s);
    case 7: return run_fdm<7, T>(E, xm, S, L, r, box_out, skip, s);
    case 8: return run_fdm<8, T>(E, xm, S, L, r, box_out, skip, s);
    case 9: return run_fdm<9, T>(E, xm, S, L, r, box_out, skip, s);
    case 10: return run_fdm<10, T>(E, xm, S, L, r, box_out, skip, s);
    case 11: return run_fdm<11, T>(E, xm, S, L, r, box_out, skip, s);
    case 12: return run_fdm<12, T>(E, xm, S, L, r, box_out, skip, s);
    case 13: return run_fdm<13, T>(E, xm, S, L, r, box_out, skip, s);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_fdm<double>(const SchwarzDev&, int64_t, const double*, double*,
                                       const int32_t*, hipStream_t);
template hipError_t launch_fdm<float>(const SchwarzDev&, int64_t, const float*, float*,
                                      const int32_t*, hipStream_t);

}  // namespace sem
