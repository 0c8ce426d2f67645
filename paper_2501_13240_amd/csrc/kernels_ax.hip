// Element operator kernels for gfx950 (wave64).
//
// A_L(k) u = sum_ab D_a^T diag(k G_ab) D_b u + h2 B u on every element: the
// matrix-free tensor-product operator of Sec. 2.2, whose leading work is
// dense (N+1)x(N+1) contractions identical for all elements.
//
// Mapping: one thread per local point (two for N = 10), one element (or a
// few small ones) per workgroup.  Every thread issues all of its global loads
// -- u (or its gather through the free numbering), the six geometric factors
// and k -- before the first barrier, so a workgroup has its whole element in
// flight at once; the streamed arrays are read and w written with
// nontemporal hints (each byte is touched once).  The in-solve form's
// shared-copy outputs are plain stores instead when the local array is small
// enough: the segmented sum reads them right after and finds most of them in
// the memory-side cache (28 -> 22 us per iteration on the 32x32x16, N = 7
// box, against 2 us more for the operator).  The element
// block and D live in LDS; the reference-gradient phase and the transposed
// phase are separated by one barrier.  For N = 7 a wavefront is exactly one k-plane,
// so the t-direction coefficients D[k][l] are wave-uniform and come from
// scalar loads instead of LDS.
//
// For larger N the scalar contractions make the kernel LDS-bound (each
// point reads 2 (N+1) values per direction per phase from LDS).  There the
// contractions run on the matrix cores instead (ax_mfma_kernel): each
// direction is a batch of 16-column tiles C = D X (or D^T X) with X gathered
// from the element block in LDS, 16x16x4 MFMAs in FP64 or FP32, so every LDS
// value feeds a whole tile column instead of one output.
//
// Per local point the FP64 apply streams u (8 B), six geometric factors
// (48 B, planar layout [E][6][P]) and w (8 B): 64 B.
//
// Inside the CG (N >= 5) the matrix-core kernel also splits its output: the
// nodes with a single local copy are finished by the element itself, so it
// stores w there straight into the free vector (with the p.w, w, p sums of
// the iteration's dot products), and only the shared copies go through the
// segmented sum, from the element's surface slots.
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include <hip/hip_ext.h>

#include "common.hpp"
#include "mfma_16x16x4.hpp"

namespace sem {
namespace {

// elements per workgroup and points per thread, chosen so that the workgroup
// fills whole wavefronts with little idle work and stays within 1024 threads
constexpr int pick_epb(int P) {
  return P <= 8 ? 32 : P <= 27 ? 9 : P <= 64 ? 4 : P <= 343 ? 2 : 1;
}

template <int N>
struct Shape {
  static constexpr int n1 = N + 1;
  static constexpr int P2 = n1 * n1;
  static constexpr int P = P2 * n1;
  static constexpr int PPT = P > 1024 ? 2 : 1;          // points per thread
  static constexpr int TPE = (P + PPT - 1) / PPT;       // threads per element
  static constexpr int EPB = pick_epb(P);
  static constexpr int BT = ((EPB * TPE + 63) / 64) * 64;
  static constexpr bool kUniform = (P2 == 64 && PPT == 1);  // a wavefront = one k-plane
};

template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void st_stream(T v, T* p) {
  __builtin_nontemporal_store(v, p);
}

template <int N, typename T, bool GATHER>
__global__ __launch_bounds__(Shape<N>::BT) void ax_kernel(
    const T* __restrict__ u, const int32_t* __restrict__ lmap, T* __restrict__ w,
    const T* __restrict__ kf, const T h2, const T* __restrict__ G, const T* __restrict__ B,
    const T* __restrict__ D, const int64_t E, const int32_t* __restrict__ skip) {
  using S = Shape<N>;
  constexpr int n1 = S::n1, P2 = S::P2, P = S::P, EPB = S::EPB, PPT = S::PPT, TPE = S::TPE;
  if (skip && *skip) return;  // uniform over the grid
  __shared__ T su[EPB][P];
  __shared__ T sv[EPB][3][P];
  __shared__ T sD[n1 * n1];

  const int t = threadIdx.x;
  const int slot = t / TPE;
  const int tl = t - slot * TPE;
  const int64_t e = xcd_block(blockIdx.x, gridDim.x) * EPB + slot;
  const bool ok_e = slot < EPB && e < E;
  const int ss = slot < EPB ? slot : 0;
  const bool use_k = kf != nullptr;
  const bool use_h2 = h2 != T(0);

  // Idle threads (tail of the last workgroup, padding lanes) load from a
  // clamped valid address and discard the values, so every load below is
  // unconditional and issued back to back.
  const int64_t ec = ok_e ? e : E - 1;
  for (int a = t; a < n1 * n1; a += S::BT) sD[a] = D[a];
  T uq[PPT], gq[PPT][6], kq[PPT];
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int qr = tl + s * TPE;
    const int q = qr < P ? qr : P - 1;
    const int64_t idx = ec * P + q;
    T v;
    if constexpr (GATHER) {
      const int32_t lm = ld_stream(lmap + idx);
      v = u[lm >= 0 ? lm : 0];
      v = lm >= 0 ? v : T(0);
    } else {
      v = ld_stream(u + idx);
    }
    uq[s] = ok_e ? v : T(0);
    const T* g = G + ec * 6 * P + q;
#pragma unroll
    for (int c = 0; c < 6; ++c) gq[s][c] = ld_stream(g + c * P);
    kq[s] = use_k ? ld_stream(kf + idx) : T(1);
  }
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int q = tl + s * TPE;
    if (slot < EPB && q < P) su[ss][q] = uq[s];
  }
  __syncthreads();

  // reference gradient, metric, conductivity
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int q = tl + s * TPE;
    if (slot < EPB && q < P) {
      const int i = q % n1, j = (q / n1) % n1;
      const int k = S::kUniform ? __builtin_amdgcn_readfirstlane(q / P2) : q / P2;
      const T* uk = &su[ss][k * P2];
      T ur = T(0), us = T(0), ut = T(0);
#pragma unroll
      for (int l = 0; l < n1; ++l) {
        ur += sD[i * n1 + l] * uk[j * n1 + l];
        us += sD[j * n1 + l] * uk[l * n1 + i];
        const T dkl = S::kUniform ? D[k * n1 + l] : sD[k * n1 + l];
        ut += dkl * su[ss][l * P2 + j * n1 + i];
      }
      const T* gc = gq[s];
      T vr = gc[0] * ur + gc[1] * us + gc[2] * ut;
      T vs = gc[1] * ur + gc[3] * us + gc[4] * ut;
      T vt = gc[2] * ur + gc[4] * us + gc[5] * ut;
      if (use_k) {
        vr *= kq[s];
        vs *= kq[s];
        vt *= kq[s];
      }
      sv[ss][0][q] = vr;
      sv[ss][1][q] = vs;
      sv[ss][2][q] = vt;
    }
  }
  __syncthreads();

  // transposed contractions (+ mass term)
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int q = tl + s * TPE;
    if (ok_e && q < P) {
      const int i = q % n1, j = (q / n1) % n1;
      const int k = S::kUniform ? __builtin_amdgcn_readfirstlane(q / P2) : q / P2;
      const T* vr = &sv[ss][0][k * P2];
      const T* vs = &sv[ss][1][k * P2];
      T acc = T(0);
#pragma unroll
      for (int l = 0; l < n1; ++l) {
        acc += sD[l * n1 + i] * vr[j * n1 + l];
        acc += sD[l * n1 + j] * vs[l * n1 + i];
        const T dlk = S::kUniform ? D[l * n1 + k] : sD[l * n1 + k];
        acc += dlk * sv[ss][2][l * P2 + j * n1 + i];
      }
      const int64_t idx = e * P + q;
      if (use_h2) acc += h2 * ld_stream(B + idx) * uq[s];
      st_stream(acc, w + idx);
    }
  }
}


// ------------------------------------------------------------ matrix cores

// One 16-column tile of a contraction along direction DIR of the element
// block src ([k][j][i], n1 per direction): out[.., row, ..] = sum_l A[row][l]
// src[.., l, ..], A = D (forward) or D^T (transposed), given as per-lane
// fragments.  Columns enumerate the two other indices: DIR 0 (along i):
// col = k n1 + j; DIR 1 (along j): col = k n1 + i; DIR 2 (along k): col =
// j n1 + i.  ACC adds into dst instead of storing.
template <int n1, typename T, int DIR, bool ACC>
__device__ __forceinline__ void contract_tile(const T* __restrict__ src, T* __restrict__ dst,
                                              const T (&afrag)[(n1 + 3) / 4], int tile, int lane) {
  constexpr int P2 = n1 * n1, KS = (n1 + 3) / 4;
  const int col = tile * 16 + (lane & 15);
  const int kk = lane >> 4;
  const bool cval = col < P2;
  const int c1 = cval ? col / n1 : 0, c0 = cval ? col % n1 : 0;
  typename Mm<T>::V acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int l = 4 * s + kk;
    T b = T(0);
    if (cval && l < n1) {
      const int a = DIR == 0 ? c1 * P2 + c0 * n1 + l : DIR == 1 ? c1 * P2 + l * n1 + c0 : l * P2 + col;
      b = src[a];
    }
    acc = Mm<T>::mma(afrag[s], b, acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = Mm<T>::row(lane, r);
    if (cval && row < n1) {
      const int a =
          DIR == 0 ? c1 * P2 + c0 * n1 + row : DIR == 1 ? c1 * P2 + row * n1 + c0 : row * P2 + col;
      if (ACC) dst[a] += acc[r];
      else dst[a] = acc[r];
    }
  }
}

typedef _Float16 v4h_t __attribute__((ext_vector_type(4)));
typedef __bf16 v4bf_t __attribute__((ext_vector_type(4)));

// 16x16x16 MFMA with 16-bit operands and FP32 accumulation (products of two
// 16-bit values are exact in FP32): A[i][k] in lane i + 16 (k / 4), vector
// element k % 4; B[k][j] in lane j + 16 (k / 4), element k % 4; result laid
// out as in the FP32 16x16x4 form (checked on the device).  One instruction
// covers a whole contraction: K = 16 >= N + 1, the rest padded with zeros.
// LP = 1: bfloat16 operands; LP = 2: IEEE half operands.  Conversions round
// to nearest, ties to even.
template <int LP>
struct Mfma16;
template <>
struct Mfma16<1> {
  typedef v4bf_t V;
  static __device__ __forceinline__ __bf16 cvt(float x) { return (__bf16)x; }
  static __device__ __forceinline__ v4f_t mma(V a, V b, v4f_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma16<2> {
  typedef v4h_t V;
  static __device__ __forceinline__ _Float16 cvt(float x) { return (_Float16)x; }
  static __device__ __forceinline__ v4f_t mma(V a, V b, v4f_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
  }
};

// contract_tile with 16-bit operands: each source value is multiplied by the
// block scale `sc` (a power of two, exact) before rounding, and each result
// by `inv` = 1 / sc after accumulation.
template <int n1, int LP, int DIR, bool ACC>
__device__ __forceinline__ void contract_tile16(const float* __restrict__ src,
                                                float* __restrict__ dst,
                                                typename Mfma16<LP>::V afrag, int tile, int lane,
                                                float sc, float inv) {
  constexpr int P2 = n1 * n1;
  const int col = tile * 16 + (lane & 15);
  const int kk = lane >> 4;
  const bool cval = col < P2;
  const int c1 = cval ? col / n1 : 0, c0 = cval ? col % n1 : 0;
  typename Mfma16<LP>::V b;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int l = 4 * kk + e;
    float x = 0.0f;
    if (cval && l < n1) {
      const int a = DIR == 0 ? c1 * P2 + c0 * n1 + l : DIR == 1 ? c1 * P2 + l * n1 + c0 : l * P2 + col;
      x = src[a];
    }
    b[e] = Mfma16<LP>::cvt(x * sc);
  }
  v4f_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
  acc = Mfma16<LP>::mma(afrag, b, acc);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 4 * (lane >> 4) + r;
    if (cval && row < n1) {
      const int a =
          DIR == 0 ? c1 * P2 + c0 * n1 + row : DIR == 1 ? c1 * P2 + row * n1 + c0 : row * P2 + col;
      if (ACC) dst[a] += acc[r] * inv;
      else dst[a] = acc[r] * inv;
    }
  }
}

// Power-of-two scale that puts a block maximum m in [2^14, 2^15) (IEEE half
// keeps all its bits there and cannot overflow), with the exponent kept in
// FP32's normal range; 1 for zero or non-finite m.
__device__ __forceinline__ float half_block_scale(float m) {
  if (!(m > 0.0f) || !(m <= 3.402823466e38f)) return 1.0f;
  int ex;
  (void)frexpf(m, &ex);
  const int k = min(max(15 - ex, -126), 126);
  return ldexpf(1.0f, k);
}


__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

template <int N>
struct MShape {
  static constexpr int n1 = N + 1;
  static constexpr int P2 = n1 * n1;
  static constexpr int P = P2 * n1;
  // threads per element (= per workgroup).  N = 9 (1000 points) takes 256
  // threads with four points each rather than 512 with two: as many waves
  // per CU hold more elements (FP32: 7 instead of 4, FP64: 4 instead of 3),
  // stand-alone apply 241 -> 221 us (FP32) and 395 -> 385 us (FP64) on the
  // 32^3 cube.  N = 10 keeps 512 (six points per thread would cost registers).
  static constexpr int TPB =
      P <= 64 ? 64 : P <= 128 ? 128 : P <= 1000 ? 256 : 512;
  static constexpr int PPT = (P + TPB - 1) / TPB;    // points per thread
  static constexpr int NT = (P2 + 15) / 16;          // 16-column tiles per direction
  static constexpr int KS = (n1 + 3) / 4;            // K steps of 4
  static constexpr int NW = TPB / 64;                // wavefronts
};

// Operator with matrix-core contractions, one element per workgroup.
// Phases: loads -> forward contractions (3 NT tiles over the wavefronts) ->
// pointwise metric and k -> transposed contractions accumulated direction
// by direction into the (now free) input block -> stores.
// LP = 0: contractions in T (FP64 or FP32 MFMA).  LP = 1 / 2 (T = float):
// bfloat16 / half operands for D, the u block and each v_a block, FP32
// accumulation; for half each block is scaled by its power-of-two block
// scale, whose maxima are reduced before the barriers the phases already have.
// MODE 0: u and w local [E][P].  MODE 1: u gathered from a free vector
// through lmap.  MODE 2 (in-solve split): lmap holds v >= 0 for a free node v
// with one local copy, -(v + 2) for a shared free node v, -1 for a Dirichlet
// copy; single-copy results go straight to the free vector wf[v], shared
// copies' results to w (local, for the segmented sum), and epart[2 (NW e +
// wave) + a] receives each wavefront's sums of p w and of w over all its
// free copies (p = the gathered input; over the copies of a shared node
// they add up to p_g w_g and w_g), reduced in a fixed order.  MODE 3: MODE 2
// with nontemporal shared-copy stores (for local arrays larger than the
// memory-side cache).  MODE 4 / 5: MODE 2 / 3 without the wavefront sums (a
// Chebyshev pass needs none).  MODE 6 / 7: MODE 2 / 3 with p w only (sum(w)
// serves the null-space projection alone).  Each sum costs the kernel more
// than its instructions suggest (measured per launch, N = 9 FP64: no sums
// 375 us, p w 390 us, three sums 440-460 us; N = 7 FP64: 89, 92, 95 us).
// Waves per SIMD the split in-solve form asks for: the gather form's
// occupancy at N = 6 and N = 9, which a few extra registers would cost it
// (at N = 9, with 512-thread workgroups, one fewer resident workgroup per CU
// once made the kernel 1.8x slower).
constexpr int split_min_waves(int N) { return N == 6 ? 7 : N == 9 ? 4 : 1; }

template <int N, typename T, int MODE, int LP>
__global__ __launch_bounds__(MShape<N>::TPB) __attribute__((
    amdgpu_waves_per_eu(MODE >= 2 && sizeof(T) == 8 ? split_min_waves(N) : 1))) void ax_mfma_kernel(
    const T* __restrict__ u, const int32_t* __restrict__ lmap, T* __restrict__ w,
    const T* __restrict__ kf, const T h2, const T* __restrict__ G, const T* __restrict__ B,
    const T* __restrict__ D, const int64_t E, const int32_t* __restrict__ skip,
    T* __restrict__ wf, double* __restrict__ epart) {
  using S = MShape<N>;
  constexpr int n1 = S::n1, P = S::P, TPB = S::TPB, PPT = S::PPT, NT = S::NT, KS = S::KS,
                NW = S::NW;
  static_assert(LP == 0 || std::is_same<T, float>::value, "16-bit operands need FP32 data");
  // wavefront sums into epart: 2 (p w, w) or 1 (p w)
  constexpr int kSums = (MODE == 2 || MODE == 3) ? 2 : (MODE == 6 || MODE == 7) ? 1 : 0;
  constexpr bool kDots = kSums > 0;
  constexpr bool kNtShared = (MODE == 3 || MODE == 5 || MODE == 7);  // nontemporal shared-copy stores
  constexpr bool kScale = LP == 2;
  if (skip && *skip) return;  // uniform over the grid
  __shared__ T su[P];
  __shared__ T sa[3][P];
  __shared__ float smax[4][NW];  // block maxima of u, v_r, v_s, v_t per wavefront (LP = 2)
  T* so = su;  // output accumulator, reuses the input block after the forward phase
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t e = blockIdx.x;
  const bool use_k = kf != nullptr;
  const bool use_h2 = h2 != T(0);
  (void)E;

  T uq[PPT], gq[PPT][6], kq[PPT];
  // MODE 2: each point's routing code, kept in LDS until the stores (in
  // registers it cost the N = 9 kernel a wave per SIMD)
  __shared__ int32_t scode[MODE >= 2 ? P : 1];
  // MODE >= 1: every routing code of this thread first, then the gathers
  // through them (0.6 % faster in-solve and p-multigrid iterations)
  int32_t lvq[PPT];
  (void)lvq;
  if constexpr (MODE >= 1) {
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
      const int qr = t + s * TPB;
      lvq[s] = ld_stream(lmap + e * P + (qr < P ? qr : P - 1));
    }
  }
  // the geometric factors (and k) are requested before the first routing
  // code is used, so the bulk of the stream does not wait for the codes
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int qr = t + s * TPB;
    const int q = qr < P ? qr : P - 1;
    const int64_t idx = e * P + q;
    const T* g = G + e * 6 * P + q;
#pragma unroll
    for (int c = 0; c < 6; ++c) gq[s][c] = ld_stream(g + c * P);
    kq[s] = use_k ? ld_stream(kf + idx) : T(1);
  }
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int qr = t + s * TPB;
    const int q = qr < P ? qr : P - 1;
    const int64_t idx = e * P + q;
    if constexpr (MODE >= 1) {
      const int32_t lv = lvq[s];
      const int32_t lm = MODE >= 2 ? (lv >= 0 ? lv : lv <= -2 ? -(lv + 2) : -1) : lv;
      if constexpr (MODE >= 2)
        if (qr < P) scode[qr] = lv;
      const T v = u[lm >= 0 ? lm : 0];
      uq[s] = lm >= 0 ? v : T(0);
    } else {
      uq[s] = ld_stream(u + idx);
    }
  }
  // derivative-matrix fragments: forward A = D, transposed A = D^T
  T af[KS], at[KS];
  typename Mfma16<LP == 0 ? 1 : LP>::V af16, at16;
  {
    const int row = lane & 15, kk = lane >> 4;
    if constexpr (LP == 0) {
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int l = 4 * s + kk;
        const bool ok = row < n1 && l < n1;
        af[s] = ok ? D[row * n1 + l] : T(0);
        at[s] = ok ? D[l * n1 + row] : T(0);
      }
    } else {
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int l = 4 * kk + x;
        const bool ok = row < n1 && l < n1;
        af16[x] = Mfma16<LP>::cvt(ok ? D[row * n1 + l] : 0.0f);
        at16[x] = Mfma16<LP>::cvt(ok ? D[l * n1 + row] : 0.0f);
      }
    }
  }
  (void)af;
  (void)at;
  (void)af16;
  (void)at16;
  if constexpr (kScale) {
    float mu = 0.0f;
#pragma unroll
    for (int s = 0; s < PPT; ++s) mu = fmaxf(mu, fabsf((float)uq[s]));
    mu = wave_max(mu);
    if (lane == 0) smax[0][wv] = mu;
  }
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int q = t + s * TPB;
    if (q < P) su[q] = uq[s];
  }
  __syncthreads();
  if constexpr (LP == 0) {
    for (int job = wv; job < 3 * NT; job += NW) {
      const int dir = job / NT, tile = job - dir * NT;
      if (dir == 0) contract_tile<n1, T, 0, false>(su, sa[0], af, tile, lane);
      else if (dir == 1) contract_tile<n1, T, 1, false>(su, sa[1], af, tile, lane);
      else contract_tile<n1, T, 2, false>(su, sa[2], af, tile, lane);
    }
  } else {
    float sc = 1.0f;
    if constexpr (kScale) {
      float m = 0.0f;
#pragma unroll
      for (int x = 0; x < NW; ++x) m = fmaxf(m, smax[0][x]);
      sc = half_block_scale(m);
    }
    const float inv = 1.0f / sc;
    for (int job = wv; job < 3 * NT; job += NW) {
      const int dir = job / NT, tile = job - dir * NT;
      if (dir == 0) contract_tile16<n1, LP, 0, false>(su, sa[0], af16, tile, lane, sc, inv);
      else if (dir == 1) contract_tile16<n1, LP, 1, false>(su, sa[1], af16, tile, lane, sc, inv);
      else contract_tile16<n1, LP, 2, false>(su, sa[2], af16, tile, lane, sc, inv);
    }
  }
  __syncthreads();
  float mv[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int q = t + s * TPB;
    if (q < P) {
      const T ur = sa[0][q], us = sa[1][q], ut = sa[2][q];
      const T* gc = gq[s];
      T vr = gc[0] * ur + gc[1] * us + gc[2] * ut;
      T vs = gc[1] * ur + gc[3] * us + gc[4] * ut;
      T vt = gc[2] * ur + gc[4] * us + gc[5] * ut;
      if (use_k) {
        vr *= kq[s];
        vs *= kq[s];
        vt *= kq[s];
      }
      sa[0][q] = vr;
      sa[1][q] = vs;
      sa[2][q] = vt;
      if constexpr (kScale) {
        mv[0] = fmaxf(mv[0], fabsf((float)vr));
        mv[1] = fmaxf(mv[1], fabsf((float)vs));
        mv[2] = fmaxf(mv[2], fabsf((float)vt));
      }
    }
  }
  if constexpr (kScale) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float m = wave_max(mv[d]);
      if (lane == 0) smax[1 + d][wv] = m;
    }
  }
  __syncthreads();
  if constexpr (LP == 0) {
    for (int tile = wv; tile < NT; tile += NW) contract_tile<n1, T, 0, false>(sa[0], so, at, tile, lane);
    __syncthreads();
    for (int tile = wv; tile < NT; tile += NW) contract_tile<n1, T, 1, true>(sa[1], so, at, tile, lane);
    __syncthreads();
    for (int tile = wv; tile < NT; tile += NW) contract_tile<n1, T, 2, true>(sa[2], so, at, tile, lane);
  } else {
    float sc[3] = {1.0f, 1.0f, 1.0f};
    if constexpr (kScale) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        float m = 0.0f;
#pragma unroll
        for (int x = 0; x < NW; ++x) m = fmaxf(m, smax[1 + d][x]);
        sc[d] = half_block_scale(m);
      }
    }
    for (int tile = wv; tile < NT; tile += NW)
      contract_tile16<n1, LP, 0, false>(sa[0], so, at16, tile, lane, sc[0], 1.0f / sc[0]);
    __syncthreads();
    for (int tile = wv; tile < NT; tile += NW)
      contract_tile16<n1, LP, 1, true>(sa[1], so, at16, tile, lane, sc[1], 1.0f / sc[1]);
    __syncthreads();
    for (int tile = wv; tile < NT; tile += NW)
      contract_tile16<n1, LP, 2, true>(sa[2], so, at16, tile, lane, sc[2], 1.0f / sc[2]);
  }
  __syncthreads();
  double ps[2] = {0.0, 0.0};
  (void)ps;
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int q = t + s * TPB;
    if (q < P) {
      const int64_t idx = e * P + q;
      T acc = so[q];
      if (use_h2) acc += h2 * ld_stream(B + idx) * uq[s];
      if constexpr (MODE >= 2) {
        const int32_t c = scode[q];
        if (c >= 0) {
          st_stream(acc, wf + c);
        } else if (c <= -2) {
          // shared copy: at its surface slot of the element's block
          T* dst = w + e * P + surface_rank(q % n1, (q / n1) % n1, q / (n1 * n1), N);
          if constexpr (kNtShared)
            st_stream(acc, dst);
          else
            *dst = acc;
        }
        if constexpr (kDots) {
          if (c != -1) {  // free copies only
            ps[0] += (double)uq[s] * (double)acc;
            if constexpr (kSums == 2) ps[1] += (double)acc;
          }
        }
      } else {
        st_stream(acc, w + idx);
      }
    }
  }
  if constexpr (kDots) {
    // the sums of one wavefront: no barrier, no LDS.  Lane 0 is found by
    // mbcnt here rather than from the lane index computed at the start,
    // which the compiler would otherwise keep (and at N = 9 spill) all along.
    // (Tried and not kept: the sums on the matrix cores, 16 instead of 30
    // vector instructions per sum, and the three DPP chains interleaved:
    // both as slow or slower.)
    const bool first_lane = __builtin_amdgcn_mbcnt_lo(~0u, 0u) == 0;
#pragma unroll
    for (int a = 0; a < kSums; ++a) {
      const double x = wave_sum_d(ps[a]);
      if (first_lane) epart[(e * NW + wv) * 2 + a] = x;
    }
  }
}

// The matrix-core kernel exists from N = 5 on (below that a 16-wide tile
// wastes most of its lanes).  Which kernel serves a launch: the environment
// variable SEM_AX_KERNEL = scalar | mfma forces one (read once per process),
// otherwise the measured default of prefer_mfma.
constexpr bool has_mfma(int N) { return N >= 5; }
enum class AxChoice { Auto, Scalar, Mfma };
AxChoice ax_choice() {
  static const AxChoice c = [] {
    const char* e = std::getenv("SEM_AX_KERNEL");
    if (e && std::strcmp(e, "scalar") == 0) return AxChoice::Scalar;
    if (e && std::strcmp(e, "mfma") == 0) return AxChoice::Mfma;
    return AxChoice::Auto;
  }();
  return c;
}
bool prefer_mfma(int N, bool gather, bool fp32) {
  (void)gather;
  (void)fp32;
  return N >= 5;
}

// kbar_q = sign sum_ab (D_a wbar)_q G_ab,q (D_b u)_q: the derivative of the
// operator in k contracted with a cotangent (same mapping, 72 B per point);
// sign = -1 gives the gradient of a solve (exact negation).
template <int N>
__global__ __launch_bounds__(Shape<N>::BT) void kbar_kernel(
    const double* __restrict__ u, const double* __restrict__ wb, double* __restrict__ kbar,
    const double* __restrict__ G, const double* __restrict__ D, const int64_t E,
    const double sign) {
  using S = Shape<N>;
  constexpr int n1 = S::n1, P2 = S::P2, P = S::P, EPB = S::EPB, PPT = S::PPT, TPE = S::TPE;
  __shared__ double su[EPB][P];
  __shared__ double sw[EPB][P];
  __shared__ double sD[n1 * n1];
  const int t = threadIdx.x;
  const int slot = t / TPE;
  const int tl = t - slot * TPE;
  const int64_t e = (int64_t)blockIdx.x * EPB + slot;
  const bool ok_e = slot < EPB && e < E;
  const int ss = slot < EPB ? slot : 0;
  const int64_t ec = ok_e ? e : E - 1;
  double gq[PPT][6];
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int qr = tl + s * TPE;
    const int q = qr < P ? qr : P - 1;
    const double* g = G + ec * 6 * P + q;
#pragma unroll
    for (int c = 0; c < 6; ++c) gq[s][c] = ld_stream(g + c * P);
    const double uv = ld_stream(u + ec * P + q), wv = ld_stream(wb + ec * P + q);
    if (slot < EPB && qr < P) {
      su[ss][q] = ok_e ? uv : 0.0;
      sw[ss][q] = ok_e ? wv : 0.0;
    }
  }
  for (int a = t; a < n1 * n1; a += S::BT) sD[a] = D[a];
  __syncthreads();
#pragma unroll
  for (int s = 0; s < PPT; ++s) {
    const int q = tl + s * TPE;
    if (ok_e && q < P) {
      const int i = q % n1, j = (q / n1) % n1, k = q / P2;
      double ur = 0, us = 0, ut = 0, wr = 0, ws = 0, wt = 0;
#pragma unroll
      for (int l = 0; l < n1; ++l) {
        const double dil = sD[i * n1 + l], djl = sD[j * n1 + l], dkl = sD[k * n1 + l];
        const int qr = k * P2 + j * n1 + l, qs = k * P2 + l * n1 + i, qt = l * P2 + j * n1 + i;
        ur += dil * su[ss][qr];
        us += djl * su[ss][qs];
        ut += dkl * su[ss][qt];
        wr += dil * sw[ss][qr];
        ws += djl * sw[ss][qs];
        wt += dkl * sw[ss][qt];
      }
      const double* gc = gq[s];
      const double vr = gc[0] * ur + gc[1] * us + gc[2] * ut;
      const double vs = gc[1] * ur + gc[3] * us + gc[4] * ut;
      const double vt = gc[2] * ur + gc[4] * us + gc[5] * ut;
      st_stream(sign * (wr * vr + ws * vs + wt * vt), kbar + e * P + q);
    }
  }
}

template <typename T>
__global__ void mass_kernel(int64_t n, const T* __restrict__ B, const T* __restrict__ u,
                            T* __restrict__ w) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x)
    w[q] = B[q] * u[q];
}

// A launch that, when ev0 / ev1 are given, has the runtime stamp them with the
// kernel's own start and end (the solve's operator timing): an event recorded
// before the launch would also count the dispatch latency.
#define SEM_LAUNCH(ev0, ev1, kernel, grid, block, stream, ...)                           \
  do {                                                                                 \
    if ((ev0) != nullptr || (ev1) != nullptr)                                          \
      hipExtLaunchKernelGGL(kernel, grid, block, 0, stream, ev0, ev1, 0, __VA_ARGS__); \
    else                                                                               \
      hipLaunchKernelGGL(kernel, grid, block, 0, stream, __VA_ARGS__);                 \
  } while (0)

template <int N, typename T, int LP>
hipError_t run_ax_mfma(const sem_mesh* m, const T* u, const int32_t* lmap, T* w, const T* k, T h2,
                       const T* G, const T* B, const T* D, hipStream_t s, const int32_t* skip,
                       hipEvent_t ev0, hipEvent_t ev1) {
  using M = MShape<N>;
  if (lmap)
    SEM_LAUNCH(ev0, ev1, (ax_mfma_kernel<N, T, 1, LP>), dim3((unsigned)m->E), dim3(M::TPB), s, u,
               lmap, w, k, h2, G, B, D, m->E, skip, (T*)nullptr, (double*)nullptr);
  else
    SEM_LAUNCH(ev0, ev1, (ax_mfma_kernel<N, T, 0, LP>), dim3((unsigned)m->E), dim3(M::TPB), s, u,
               lmap, w, k, h2, G, B, D, m->E, skip, (T*)nullptr, (double*)nullptr);
  return hipGetLastError();
}

template <int N, typename T>
hipError_t run_ax(const sem_mesh* m, const T* u, const int32_t* lmap, T* w, const T* k, T h2,
                  const T* G, const T* B, const T* D, hipStream_t s, const int32_t* skip, int lp,
                  hipEvent_t ev0, hipEvent_t ev1) {
  if constexpr (std::is_same<T, float>::value) {
    if (lp == 1) return run_ax_mfma<N, float, 1>(m, u, lmap, w, k, h2, G, B, D, s, skip, ev0, ev1);
    if (lp == 2) return run_ax_mfma<N, float, 2>(m, u, lmap, w, k, h2, G, B, D, s, skip, ev0, ev1);
  }
  if (lp != 0) return hipErrorInvalidValue;
  if constexpr (has_mfma(N)) {
    const AxChoice c = ax_choice();
    const bool mfma = c == AxChoice::Auto ? prefer_mfma(N, lmap != nullptr, sizeof(T) == 4)
                                          : c == AxChoice::Mfma;
    if (mfma) return run_ax_mfma<N, T, 0>(m, u, lmap, w, k, h2, G, B, D, s, skip, ev0, ev1);
  }
  using S = Shape<N>;
  const int64_t grid = (m->E + S::EPB - 1) / S::EPB;
  if (lmap)
    SEM_LAUNCH(ev0, ev1, (ax_kernel<N, T, true>), dim3((unsigned)grid), dim3(S::BT), s, u, lmap,
               w, k, h2, G, B, D, m->E, skip);
  else
    SEM_LAUNCH(ev0, ev1, (ax_kernel<N, T, false>), dim3((unsigned)grid), dim3(S::BT), s, u, lmap,
               w, k, h2, G, B, D, m->E, skip);
  return hipGetLastError();
}

template <int N>
hipError_t run_kbar(const sem_mesh* m, const double* u, const double* wb, double* kbar,
                    double sign, hipStream_t s) {
  using S = Shape<N>;
  const int64_t grid = (m->E + S::EPB - 1) / S::EPB;
  hipLaunchKernelGGL((kbar_kernel<N>), dim3((unsigned)grid), dim3(S::BT), 0, s, u, wb, kbar,
                     m->G64.as<double>(), m->D64.as<double>(), m->E, sign);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_ax(const sem_mesh* m, const T* u, const int32_t* lmap, T* w, const T* k, T h2,
                     const T* G, const T* B, const T* D, hipStream_t s, const int32_t* skip,
                     int lp, hipEvent_t ev0, hipEvent_t ev1) {
  switch (m->N) {
    case 1: return run_ax<1, T>(m, u, lmap, w, k, h2, G, B, D, s, skip, lp, ev0, ev1);
    case 2: return run_ax<2, T>(m, u, lmap, w, k, h2, G, B, D, s, skip, lp, ev0, ev1);
    case 3: return run_ax<3, T>(m, u, lmap, w, k, h2, G, B, D, s, skip, lp, ev0, ev1);
    case 4: return run_ax<4, T>(m, u, lmap, w, k, h2, G, B, D, s, skip, lp, ev0, ev1);
    case 5: return run_ax<5, T>(m, u, lmap, w, k, h2, G, B, D, s, skip, lp, ev0, ev1);
    case 6: return run_ax<6, T>(m, u, lmap, w, k, h2, G, B, D, s, skip, lp, ev0, ev1);
    case 7: return run_ax<7, T>(m, u, lmap, w, k, h2, G, B, D, s, skip, lp, ev0, ev1);
    case 8: return run_ax<8, T>(m, u, lmap, w, k, h2, G, B, D, s, skip, lp, ev0, ev1);
    case 9: return run_ax<9, T>(m, u, lmap, w, k, h2, G, B, D, s, skip, lp, ev0, ev1);
    case 10: return run_ax<10, T>(m, u, lmap, w, k, h2, G, B, D, s, skip, lp, ev0, ev1);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_ax<double>(const sem_mesh*, const double*, const int32_t*, double*,
                                      const double*, double, const double*, const double*,
                                      const double*, hipStream_t, const int32_t*, int, hipEvent_t,
                                      hipEvent_t);
template hipError_t launch_ax<float>(const sem_mesh*, const float*, const int32_t*, float*,
                                     const float*, float, const float*, const float*,
                                     const float*, hipStream_t, const int32_t*, int, hipEvent_t,
                                     hipEvent_t);

namespace {
template <int N, typename T>
hipError_t run_ax_split(const sem_mesh* m, const T* u, T* wf, T* wL, double* epart, bool mean_sums,
                        const T* k, T h2, const T* G, const T* B, const T* D, hipStream_t s,
                        const int32_t* skip, hipEvent_t ev0, hipEvent_t ev1) {
  if constexpr (has_mfma(N)) {
    using M = MShape<N>;
    // shared-copy results stay in the memory-side cache for the segmented
    // sum when the local array fits well inside it (256 MB): plain stores up
    // to m->ax_nt_bytes, 128 MB by default (the 32x32x16, N = 7 box: 67 MB,
    // 1.1 % faster per iteration), nontemporal above (the 32^3, N = 9 cube:
    // 262 MB, 2.2 %) (a run-time switch in the kernel cost what the
    // nontemporal stores save).  Sums: p w and sum(w) (MODE 2 / 3) when the
    // solve projects out the constants, p w alone (MODE 6 / 7) otherwise,
    // none without epart (MODE 4 / 5).
    const bool plain = m->nL * (int64_t)sizeof(T) <= m->ax_nt_bytes;
    const int mode = !epart ? (plain ? 4 : 5) : mean_sums ? (plain ? 2 : 3) : (plain ? 6 : 7);
    const dim3 grid((unsigned)m->E), block(M::TPB);
    const int32_t* lm = m->lmap2.as<int32_t>();
#define SEM_SPLIT_CASE(MD)                                                                   \
  case MD:                                                                                   \
    SEM_LAUNCH(ev0, ev1, (ax_mfma_kernel<N, T, MD, 0>), grid, block, s, u, lm, wL, k, h2, G, B, \
               D, m->E, skip, wf, epart);                                                    \
    break;
    switch (mode) {
      SEM_SPLIT_CASE(2)
      SEM_SPLIT_CASE(3)
      SEM_SPLIT_CASE(4)
      SEM_SPLIT_CASE(5)
      SEM_SPLIT_CASE(6)
      SEM_SPLIT_CASE(7)
    }
#undef SEM_SPLIT_CASE
    return hipGetLastError();
  } else {
    return hipErrorNotSupported;
  }
}
}  // namespace

int ax_split_parts(int N) {
  switch (N) {
    case 5: return MShape<5>::NW;
    case 6: return MShape<6>::NW;
    case 7: return MShape<7>::NW;
    case 8: return MShape<8>::NW;
    case 9: return MShape<9>::NW;
    case 10: return MShape<10>::NW;
    default: return 0;
  }
}

bool ax_split_available(const sem_mesh* m) {
  // SEM_AX_SPLIT=0 (read once) keeps the gather form in the solve
  static const bool enabled = [] {
    const char* e = std::getenv("SEM_AX_SPLIT");
    return !(e && std::strcmp(e, "0") == 0);
  }();
  if (!enabled || !has_mfma(m->N) || !m->lmap2.p || !m->split_ok) return false;
  const AxChoice c = ax_choice();
  return c == AxChoice::Auto ? prefer_mfma(m->N, true, false) : c == AxChoice::Mfma;
}

template <typename T>
hipError_t launch_ax_split(const sem_mesh* m, const T* u, T* wf, T* wL, double* epart,
                           bool mean_sums, const T* k, T h2, const T* G, const T* B, const T* D,
                           hipStream_t s, const int32_t* skip, hipEvent_t ev0, hipEvent_t ev1) {
  if (!ax_split_available(m)) return hipErrorNotSupported;
  switch (m->N) {
    case 5: return run_ax_split<5, T>(m, u, wf, wL, epart, mean_sums, k, h2, G, B, D, s, skip,
                                           ev0, ev1);
    case 6: return run_ax_split<6, T>(m, u, wf, wL, epart, mean_sums, k, h2, G, B, D, s, skip,
                                           ev0, ev1);
    case 7: return run_ax_split<7, T>(m, u, wf, wL, epart, mean_sums, k, h2, G, B, D, s, skip,
                                           ev0, ev1);
    case 8: return run_ax_split<8, T>(m, u, wf, wL, epart, mean_sums, k, h2, G, B, D, s, skip,
                                           ev0, ev1);
    case 9: return run_ax_split<9, T>(m, u, wf, wL, epart, mean_sums, k, h2, G, B, D, s, skip,
                                           ev0, ev1);
    case 10: return run_ax_split<10, T>(m, u, wf, wL, epart, mean_sums, k, h2, G, B, D, s, skip,
                                           ev0, ev1);
    default: return hipErrorNotSupported;
  }
}
template hipError_t launch_ax_split<double>(const sem_mesh*, const double*, double*, double*,
                                            double*, bool, const double*, double, const double*,
                                            const double*, const double*, hipStream_t,
                                            const int32_t*, hipEvent_t, hipEvent_t);
template hipError_t launch_ax_split<float>(const sem_mesh*, const float*, float*, float*, double*,
                                           bool, const float*, float, const float*, const float*,
                                           const float*, hipStream_t, const int32_t*, hipEvent_t,
                                           hipEvent_t);

hipError_t launch_ax_kbar(const sem_mesh* m, const double* u, const double* wbar, double* kbar,
                          double sign, hipStream_t s) {
  switch (m->N) {
    case 1: return run_kbar<1>(m, u, wbar, kbar, sign, s);
    case 2: return run_kbar<2>(m, u, wbar, kbar, sign, s);
    case 3: return run_kbar<3>(m, u, wbar, kbar, sign, s);
    case 4: return run_kbar<4>(m, u, wbar, kbar, sign, s);
    case 5: return run_kbar<5>(m, u, wbar, kbar, sign, s);
    case 6: return run_kbar<6>(m, u, wbar, kbar, sign, s);
    case 7: return run_kbar<7>(m, u, wbar, kbar, sign, s);
    case 8: return run_kbar<8>(m, u, wbar, kbar, sign, s);
    case 9: return run_kbar<9>(m, u, wbar, kbar, sign, s);
    case 10: return run_kbar<10>(m, u, wbar, kbar, sign, s);
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
