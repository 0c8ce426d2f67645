// Preconditioned conjugate gradients on the assembled operator (the pressure
// Poisson solve of Sec. 2.2), fourth-kind Chebyshev acceleration of Jacobi
// (Sec. 2.2), FP32 preconditioner work (Sec. 2.2), and FP64 iterative
// refinement around an FP32 inner solve.
//
// Vectors of the solve live on the free unique nodes (length n_free; the
// n_single nodes with one local copy first).  One iteration is
//   ax (gathers p through lmap, writes the element-local result w_L; from
//   N = 5 on it writes w at the single-copy nodes directly, and each
//   wavefront's p.w over all its copies)
//   -> segmented sum w = R Q^T w_L fused with p.w (over the shared nodes)
//   -> alpha on the device -> residual update fused with r.r (and r.S r)
//   -> beta on the device -> p update, which also applies x += alpha p (it
//   reads p anyway).  Jacobi keeps z = S r in place of r, and from N = 5 on
//   folds the segmented sum into the residual update (w is summed there at
//   the shared nodes, never stored), after a short kernel that reduces the
//   operator's p.w sums.
// All scalars stay on the device (CgScalars); the host only polls the `done`
// flag every few iterations with one chunk of iterations always queued ahead,
// and every kernel of a finished solve returns at once.  Reductions use a
// fixed grid and a fixed summation order, so solves are bit-reproducible.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "solver.hpp"

namespace sem {

// ---------------------------------------------------------------- helpers
namespace {

// Largest solve (free nodes) that replays captured iteration graphs:
// kGraphMaxFree, or the environment variable SEM_GRAPH_MAX_FREE (read once).
int64_t graph_max_free() {
  static const int64_t v = [] {
    const char* e = std::getenv("SEM_GRAPH_MAX_FREE");
    return e && *e ? (int64_t)std::strtoll(e, nullptr, 10) : kGraphMaxFree;
  }();
  return v;
}

#define GRID_STRIDE(idx, n)                                                        \
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < (n); \
       idx += (int64_t)gridDim.x * blockDim.x)

__device__ __forceinline__ double wave_sum(double x) { return wave_sum_d(x); }

// per-block partial sums of NV values -> part[blockIdx.x * NV + a]
template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double* __restrict__ part) {
  __shared__ double red[NV][kVecBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < NV; ++a) {
    const double x = wave_sum(v[a]);
    if (lane == 0) red[a][wid] = x;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int w = 0; w < kVecBlock / 64; ++w) s += red[threadIdx.x][w];
    part[blockIdx.x * NV + threadIdx.x] = s;
  }
}

// one block sums nblk partials in a fixed order; every thread gets S
template <int NV>
__device__ __forceinline__ void block_total(const double* __restrict__ part, int nblk,
                                            double (&S)[NV]) {
  __shared__ double red[NV][kVecBlock / 64];
  __shared__ double tot[NV];
  double v[NV];
#pragma unroll
  for (int a = 0; a < NV; ++a) v[a] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
#pragma unroll
    for (int a = 0; a < NV; ++a) v[a] += part[b * NV + a];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < NV; ++a) {
    const double x = wave_sum(v[a]);
    if (lane == 0) red[a][wid] = x;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int w = 0; w < kVecBlock / 64; ++w) s += red[threadIdx.x][w];
    tot[threadIdx.x] = s;
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < NV; ++a) S[a] = tot[a];
}

__device__ __forceinline__ bool finite(double x) { return x == x && fabs(x) <= 1.7976931348623157e308; }

// ------------------------------------------------------------- CG kernels
//
// No finalisation launches and no grid-wide fences: a reducing kernel writes
// per-block partial sums, and every block of the kernel that consumes them
// sums all partials itself in the same fixed order, so all blocks obtain
// bit-identical scalars (alpha, beta, the convergence decision).  Block 0
// records them in CgScalars for the host and for later kernels.  rho is kept
// in two slots indexed by the iteration's parity so that block 0 can store
// the next value while other blocks still read the current one.

// w = R Q^T w_L (segmented sum); partials of p.w and sum(w)
template <typename T>
__global__ __launch_bounds__(kVecBlock) void k_gsum_pw(int64_t nf, const int32_t* __restrict__ seg,
                                                       const int32_t* __restrict__ perm,
                                                       const T* __restrict__ wL,
                                                       const T* __restrict__ p, T* __restrict__ w,
                                                       double* __restrict__ part,
                                                       CgScalars* __restrict__ sc) {
  // the previous iteration's direction update has completed
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->pending = 0;
  if (sc->done) return;
  double v[2] = {0.0, 0.0};
  BLOCK_CHUNK(g, nf) {
    const T s = segment_sum<T>(perm, wL, seg[g], seg[g + 1]);
    w[g] = s;
    v[0] += (double)p[g] * (double)s;
    v[1] += (double)s;
  }
  block_partials<2>(v, part);
}

// this block's chunk of the ne partial pairs, in order (sum(w), the second
// of a pair, serves the null-space projection only)
__device__ __forceinline__ void epart_chunk(int64_t ne, const double* __restrict__ epart,
                                            bool mean, double (&v)[2]) {
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t ch = (ne + gridDim.x - 1) / gridDim.x;
  const int64_t lo = lb * ch, hi = lo + ch < ne ? lo + ch : ne;
  for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
    v[0] += epart[2 * e];
    if (mean) v[1] += epart[2 * e + 1];
  }
}

// The same for the split operator, which has already written w at the
// single-copy free nodes [0, n1) and the partial sums (ne pairs, one per
// wavefront of each element: p.w and sum(w) over all its copies, p.w alone
// without the null-space projection): segmented sums over the shared free
// nodes [n1, nf) only, plus this block's chunk of the partial pairs (in
// order, so the totals stay deterministic).
template <typename T>
__global__ __launch_bounds__(kVecBlock) void k_gsum_split_pw(
    int64_t n1, int64_t nf, const int32_t* __restrict__ seg, const int32_t* __restrict__ perm,
    const T* __restrict__ wL, T* __restrict__ w, int64_t ne, const double* __restrict__ epart,
    double* __restrict__ part, CgScalars* __restrict__ sc) {
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->pending = 0;
  if (sc->done) return;
  double v[2] = {0.0, 0.0};
  epart_chunk(ne, epart, sc->neumann != 0, v);
  BLOCK_CHUNK(i, nf - n1) {
    const int64_t g = n1 + i;
    w[g] = segment_sum<T>(perm, wL, seg[g], seg[g + 1]);
  }
  block_partials<2>(v, part);
}

// The partial pairs alone (the split Jacobi iteration, whose residual update
// sums the shared nodes' copies itself), on a grid of kEpartBlocks
constexpr int kEpartBlocks = 64;
__global__ __launch_bounds__(kVecBlock) void k_epart_sum(int64_t ne,
                                                         const double* __restrict__ epart,
                                                         double* __restrict__ part,
                                                         CgScalars* __restrict__ sc) {
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->pending = 0;
  if (sc->done) return;
  double v[2] = {0.0, 0.0};
  epart_chunk(ne, epart, sc->neumann != 0, v);
  block_partials<2>(v, part);
}

// What the residual vector of a CG iteration holds, and which partials the
// update forms: r (and r.r only), r (r.r and r.S r, Jacobi), or z = S r in
// place of r (Jacobi: r = z / S is recovered in registers, so the direction
// update p = z + beta p reads neither r nor S).  In the first and the last
// mode x += alpha p is left to the direction update (k_pupdate_flex,
// k_pupdate_jac), which reads p anyway.
enum UpdMode { kUpdR = 0, kUpdJacR = 1, kUpdJacZ = 2 };

// The Jacobi p update walks pairs of consecutive elements (one 16-byte access
// per lane in FP64: 1.5 % faster per iteration than 8-byte accesses; the same
// in the residual update was 0.3 % slower) when its vectors are 16-byte
// aligned, as they are when each starts an allocation; else one element at a
// time.  BLOCK_CHUNK over the nf / 2 pairs, the odd last element by one thread.
__device__ __forceinline__ bool aligned16(const void* a, const void* b, const void* c) {
  return (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15) == 0;
}

// alpha = rho / p.w and, for the null-space projection, mean_w = sum(w) / n
// from the p.w and sum(w) partials (sum(w) vanishes up to rounding, as A
// annihilates the constants: subtracting mean_w keeps r exactly free of them,
// as the projection of r after each update does), the same in every block;
// block 0 records alpha, mean_w and the iteration in
// progress (the iteration index lives on the device, so a captured chunk of
// iterations can be replayed: only later kernels advance it).  False on a
// breakdown (p.w <= 0 or not finite), which ends the solve.
__device__ __forceinline__ bool cg_alpha(const double* __restrict__ part_in, int nblk,
                                         CgScalars* __restrict__ sc, double* __restrict__ ahist,
                                         bool set_pending, double& alpha, double& mw) {
  const int kit = sc->it;
  double S[2];
  block_total<2>(part_in, nblk, S);
  const double pw = S[0];
  mw = sc->neumann ? S[1] * sc->inv_n : 0.0;
  if (!(pw > 0.0) || !finite(pw)) {  // same decision in every block
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->status = 2;
      sc->done = 1;
    }
    return false;
  }
  alpha = sc->rho2[kit & 1] / pw;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->alpha = alpha;
    sc->mean_w = mw;
    sc->kcur = kit;
    if (set_pending) sc->pending = 1;
    if (ahist) ahist[kit] = alpha;
  }
  return true;
}

// alpha from the p.w partials; x += alpha p (kUpdJacR only);
// r -= alpha (w - mean_w); partials of r.r (and r.S r)
constexpr int kPrefetch = 8;
template <typename T, int MODE>
__global__ __launch_bounds__(kVecBlock) void k_update(int64_t nf, T* __restrict__ x,
                                                      const T* __restrict__ p, T* __restrict__ r,
                                                      const T* __restrict__ w,
                                                      const T* __restrict__ dinv,
                                                      const double* __restrict__ part_in, int nblk,
                                                      double* __restrict__ part,
                                                      CgScalars* __restrict__ sc,
                                                      double* __restrict__ ahist) {
  // kUpdJacZ: this thread's first kPrefetch points of its chunk are requested
  // before alpha is formed (which waits for the scalars and partial sums), so
  // the stream starts while the block reduces
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t chunk = (nf + gridDim.x - 1) / gridDim.x;
  const int64_t lo = lb * chunk + threadIdx.x, hi = lb * chunk + chunk < nf ? lb * chunk + chunk : nf;
  T pd[kPrefetch], pr[kPrefetch], pw[kPrefetch];
  if constexpr (MODE == kUpdJacZ) {
#pragma unroll
    for (int j = 0; j < kPrefetch; ++j) {
      const int64_t g = lo + (int64_t)j * blockDim.x;
      if (g < hi) {
        pd[j] = __builtin_nontemporal_load(dinv + g);
        pr[j] = r[g];
        pw[j] = w[g];
      }
    }
  }
  if (sc->done) return;
  double alpha, mw;
  if (!cg_alpha(part_in, nblk, sc, ahist, MODE != kUpdJacR, alpha, mw)) return;
  const T a = (T)alpha, mwt = (T)mw;
  double v[2] = {0.0, 0.0};
  if constexpr (MODE == kUpdJacZ) {
    // S and x (in the p update) are touched once per iteration: nontemporal,
    // so the memory-side cache keeps p, z and w, which are re-read a kernel later
    auto point = [&](int64_t g, T d, T rz, T wg) {
      const T rg = rz / d - a * (wg - mwt);
      const T zg = d * rg;
      r[g] = zg;
      v[0] += (double)rg * (double)rg;
      v[1] += (double)rg * (double)zg;
    };
#pragma unroll
    for (int j = 0; j < kPrefetch; ++j) {
      const int64_t g = lo + (int64_t)j * blockDim.x;
      if (g < hi) point(g, pd[j], pr[j], pw[j]);
    }
    for (int64_t g = lo + (int64_t)kPrefetch * blockDim.x; g < hi; g += blockDim.x)
      point(g, __builtin_nontemporal_load(dinv + g), r[g], w[g]);
  } else {
    BLOCK_CHUNK(g, nf) {
      if constexpr (MODE == kUpdJacR) x[g] = x[g] + a * p[g];
      const T rg = r[g] - a * (w[g] - mwt);
      r[g] = rg;
      const double rd = (double)rg;
      v[0] += rd * rd;
      if (MODE == kUpdJacR) v[1] += rd * rd * (double)dinv[g];
    }
  }
  block_partials<2>(v, part);
}

// kUpdJacZ for the split operator with the segmented sum folded in: w is
// read from the operator's output at the single-copy nodes [0, n1) and summed
// over the copies at their surface slots (seg, perm into wL) at the shared
// nodes [n1, nf), which the iteration then never stores.  Each block takes
// one chunk of either range, so the gathers spread over the whole grid.
template <typename T>
__global__ __launch_bounds__(kVecBlock) void k_update_split(
    int64_t n1, int64_t nf, const int32_t* __restrict__ seg, const int32_t* __restrict__ perm,
    const T* __restrict__ wL, T* __restrict__ r, const T* __restrict__ w,
    const T* __restrict__ dinv, const double* __restrict__ part_in, int nblk,
    double* __restrict__ part, CgScalars* __restrict__ sc, double* __restrict__ ahist) {
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t c1 = (n1 + gridDim.x - 1) / gridDim.x;
  const int64_t lo = lb * c1 + threadIdx.x, hi = lb * c1 + c1 < n1 ? lb * c1 + c1 : n1;
  T pd[kPrefetch], pr[kPrefetch], pw[kPrefetch];
#pragma unroll
  for (int j = 0; j < kPrefetch; ++j) {
    const int64_t g = lo + (int64_t)j * blockDim.x;
    if (g < hi) {
      pd[j] = __builtin_nontemporal_load(dinv + g);
      pr[j] = r[g];
      pw[j] = w[g];
    }
  }
  if (sc->done) return;
  double alpha, mw;
  if (!cg_alpha(part_in, nblk, sc, ahist, true, alpha, mw)) return;
  const T a = (T)alpha, mwt = (T)mw;
  double v[2] = {0.0, 0.0};
  auto point = [&](int64_t g, T d, T rz, T wg) {
    const T rg = rz / d - a * (wg - mwt);
    const T zg = d * rg;
    r[g] = zg;
    v[0] += (double)rg * (double)rg;
    v[1] += (double)rg * (double)zg;
  };
#pragma unroll
  for (int j = 0; j < kPrefetch; ++j) {
    const int64_t g = lo + (int64_t)j * blockDim.x;
    if (g < hi) point(g, pd[j], pr[j], pw[j]);
  }
  // the shared nodes' chains (offsets -> copy indices -> copy values) are
  // interleaved with the single-copy stream: each step takes one point of
  // each range, so the stream's loads are in flight while a chain waits
  const int64_t ns = nf - n1;
  const int64_t c2 = (ns + gridDim.x - 1) / gridDim.x;
  const int64_t lo2 = lb * c2 + threadIdx.x, hi2 = lb * c2 + c2 < ns ? lb * c2 + c2 : ns;
  int64_t g = lo + (int64_t)kPrefetch * blockDim.x;
  for (int64_t i = lo2; i < hi2; i += blockDim.x) {
    const int64_t gs = n1 + i;
    const bool one = g < hi;
    const int64_t gq = one ? g : gs;
    const T d1 = __builtin_nontemporal_load(dinv + gq), r1 = r[gq], w1 = w[gq];
    const T ds = __builtin_nontemporal_load(dinv + gs), rs = r[gs];
    const T ws = segment_sum<T>(perm, wL, seg[gs], seg[gs + 1]);
    if (one) point(g, d1, r1, w1);
    point(gs, ds, rs, ws);
    g += blockDim.x;
  }
  for (; g < hi; g += blockDim.x) point(g, __builtin_nontemporal_load(dinv + g), r[g], w[g]);
  block_partials<2>(v, part);
}

// convergence decision from the r.r partial (identical in every block);
// block 0 records it.  Returns true if the solve continues.
__device__ __forceinline__ bool cg_check(double rr, int kit, CgScalars* __restrict__ sc,
                                         double* __restrict__ hist) {
  const int it = kit + 1;
  int status = 0;
  bool stop = false;
  if (!finite(rr)) {
    status = 3;
    stop = true;
  } else if (!sc->fixed && rr <= sc->tol2) {
    status = 1;
    stop = true;
  } else if (it >= sc->max_it) {
    stop = true;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->it = it;
    sc->rr = rr;
    if (hist) hist[it] = sqrt(rr);
    if (stop) {
      sc->status = status;
      sc->done = 1;
    }
  }
  return !stop;
}

// Jacobi: check, beta = r.S r / rho, p = S r + beta p.  ZS: r holds z = S r,
// and x += alpha p (alpha of the update kernel) is applied here first, also
// in the iteration that stops the solve.  The guard is then the pending flag,
// which no block of this kernel writes (block 0 sets done while other blocks
// may still be starting).
template <typename T, bool ZS>
__global__ __launch_bounds__(kVecBlock) void k_pupdate_jac(int64_t nf, T* __restrict__ p,
                                                           T* __restrict__ x,
                                                           const T* __restrict__ r,
                                                           const T* __restrict__ dinv,
                                                           const double* __restrict__ part_in,
                                                           int nblk, CgScalars* __restrict__ sc,
                                                           double* __restrict__ hist,
                                                           double* __restrict__ bhist) {
  // ZS with 16-byte aligned vectors: this thread's first kPrefetch pairs of
  // p, x and z are requested before the partial sums are reduced
  typedef T V2 __attribute__((ext_vector_type(2)));
  const bool vec2 = ZS && aligned16(p, x, r);
  const int64_t nh = nf / 2;
  const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
  const int64_t chunk = (nh + gridDim.x - 1) / gridDim.x;
  const int64_t lo = lb * chunk + threadIdx.x, hi = lb * chunk + chunk < nh ? lb * chunk + chunk : nh;
  V2 pp[kPrefetch], px[kPrefetch], pz[kPrefetch];
  if (vec2) {
    const V2* p2 = reinterpret_cast<const V2*>(p);
    const V2* x2 = reinterpret_cast<const V2*>(x);
    const V2* z2 = reinterpret_cast<const V2*>(r);
#pragma unroll
    for (int j = 0; j < kPrefetch; ++j) {
      const int64_t h = lo + (int64_t)j * blockDim.x;
      if (h < hi) {
        pp[j] = p2[h];
        px[j] = __builtin_nontemporal_load(x2 + h);
        pz[j] = z2[h];
      }
    }
  }
  if (ZS ? !sc->pending : sc->done) return;
  const int kit = sc->kcur;
  const double rho = sc->rho2[kit & 1];
  const T a = (T)sc->alpha;
  double S[2];
  block_total<2>(part_in, nblk, S);
  if (!cg_check(S[0], kit, sc, hist)) {
    if constexpr (ZS) {
      BLOCK_CHUNK(g, nf) x[g] = x[g] + a * p[g];
    }
    return;
  }
  const double rz = S[1];
  const double beta = rz / rho;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->rho2[(kit + 1) & 1] = rz;
    sc->beta = beta;
    if (bhist) bhist[kit] = beta;
  }
  const T b = (T)beta;
  if constexpr (ZS) {
    if (vec2) {
      V2* p2 = reinterpret_cast<V2*>(p);
      V2* x2 = reinterpret_cast<V2*>(x);
      const V2* z2 = reinterpret_cast<const V2*>(r);
#pragma unroll
      for (int j = 0; j < kPrefetch; ++j) {
        const int64_t h = lo + (int64_t)j * blockDim.x;
        if (h < hi) {
          __builtin_nontemporal_store(px[j] + a * pp[j], x2 + h);
          p2[h] = pz[j] + b * pp[j];
        }
      }
      for (int64_t h = lo + (int64_t)kPrefetch * blockDim.x; h < hi; h += blockDim.x) {
        const V2 pg = p2[h];
        __builtin_nontemporal_store(__builtin_nontemporal_load(x2 + h) + a * pg, x2 + h);
        p2[h] = z2[h] + b * pg;
      }
      if ((nf & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const T pg = p[nf - 1];
        x[nf - 1] = x[nf - 1] + a * pg;
        p[nf - 1] = r[nf - 1] + b * pg;
      }
    } else {
      BLOCK_CHUNK(g, nf) {
        const T pg = p[g];
        __builtin_nontemporal_store(__builtin_nontemporal_load(x + g) + a * pg, x + g);
        p[g] = r[g] + b * pg;
      }
    }
  } else {
    BLOCK_CHUNK(g, nf) p[g] = dinv[g] * r[g] + b * p[g];
  }
}

// flexible CG: beta = z_{k+1}.(r_{k+1} - r_k) / rho_k = -alpha z.(w - mean_w) / rho_k
// from the preconditioner pass's partials (z.r, z.(w - mean_w)); p = z + beta p.
// x += alpha p (alpha of the residual update) is applied here first, also in
// the iteration that stops the solve (at the preconditioner's convergence
// gate, or here on a breakdown); the guard is the pending flag, which the
// residual update sets and the next iteration's segmented sum clears.
template <typename T, typename Tz>
__global__ __launch_bounds__(kVecBlock) void k_pupdate_flex(int64_t nf, T* __restrict__ p,
                                                            T* __restrict__ x,
                                                            const Tz* __restrict__ z,
                                                            const double* __restrict__ part_in,
                                                            int nblk, CgScalars* __restrict__ sc,
                                                            double* __restrict__ bhist) {
  if (!sc->pending) return;
  const T a = (T)sc->alpha;
  if (sc->done) {
    BLOCK_CHUNK(g, nf) x[g] = x[g] + a * p[g];
    return;
  }
  const int kit = sc->kcur;
  double S[2];
  block_total<2>(part_in, nblk, S);
  const double rz = S[0], zw = S[1];
  const double beta = -sc->alpha * zw / sc->rho2[kit & 1];
  if (!finite(rz) || !finite(beta)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->status = 3;
      sc->done = 1;
    }
    BLOCK_CHUNK(g, nf) x[g] = x[g] + a * p[g];
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->rho2[(kit + 1) & 1] = rz;
    sc->beta = beta;
    if (bhist) bhist[kit] = beta;
  }
  const T b = (T)beta;
  BLOCK_CHUNK(g, nf) {
    const T pg = p[g];
    x[g] = x[g] + a * pg;
    p[g] = (T)z[g] + b * pg;
  }
}

// ----------------------------------------------------- init / misc kernels

// r = b - R Q^T w_L; partials of r.r and sum(r)
template <typename T>
__global__ __launch_bounds__(kVecBlock) void k_residual(int64_t nf, const int32_t* __restrict__ seg,
                                                        const int32_t* __restrict__ perm,
                                                        const T* __restrict__ wL,
                                                        const T* __restrict__ b, T* __restrict__ r,
                                                        double* __restrict__ part) {
  double v[2] = {0.0, 0.0};
  BLOCK_CHUNK(g, nf) {
    const T s = segment_sum<T>(perm, wL, seg[g], seg[g + 1]);
    const T rg = b[g] - s;
    r[g] = rg;
    v[0] += (double)rg * (double)rg;
    v[1] += (double)rg;
  }
  block_partials<2>(v, part);
}

// partials of a.b, a.a, sum(a) (b may be null -> a.a twice)
template <typename T>
__global__ __launch_bounds__(kVecBlock) void k_dots(int64_t nf, const T* __restrict__ a,
                                                    const T* __restrict__ b,
                                                    double* __restrict__ part) {
  double v[3] = {0.0, 0.0, 0.0};
  BLOCK_CHUNK(g, nf) {
    const double ag = (double)a[g];
    const double bg = b ? (double)b[g] : ag;
    v[0] += ag * bg;
    v[1] += ag * ag;
    v[2] += ag;
  }
  block_partials<3>(v, part);
}

template <int NV>
__global__ __launch_bounds__(kVecBlock) void k_totals(const double* __restrict__ part, int nblk,
                                                      double* __restrict__ out) {
  double S[NV];
  block_total<NV>(part, nblk, S);
  if (threadIdx.x < NV) out[threadIdx.x] = S[threadIdx.x];
}

// p = z; partials of r.p
template <typename T>
__global__ __launch_bounds__(kVecBlock) void k_init_p(int64_t nf, T* __restrict__ p,
                                                      const T* __restrict__ r,
                                                      const T* __restrict__ z,
                                                      double* __restrict__ part) {
  double v[1] = {0.0};
  BLOCK_CHUNK(g, nf) {
    const T pg = z[g];
    p[g] = pg;
    v[0] += (double)pg * (double)r[g];
  }
  block_partials<1>(v, part);
}

// Jacobi with z kept in place of r: z = S r, p = z; partials of r.z
template <typename T>
__global__ __launch_bounds__(kVecBlock) void k_init_pz(int64_t nf, T* __restrict__ p,
                                                       T* __restrict__ rz,
                                                       const T* __restrict__ dinv,
                                                       double* __restrict__ part) {
  double v[1] = {0.0};
  BLOCK_CHUNK(g, nf) {
    const T rg = rz[g], zg = dinv[g] * rg;
    p[g] = zg;
    rz[g] = zg;
    v[0] += (double)zg * (double)rg;
  }
  block_partials<1>(v, part);
}

template <typename T>
__global__ void k_shift(int64_t n, T* __restrict__ a, double s) {
  GRID_STRIDE(g, n) a[g] = (T)((double)a[g] - s);
}

template <typename T>
__global__ void k_copy(int64_t n, const T* __restrict__ a, T* __restrict__ b) {
  GRID_STRIDE(g, n) b[g] = a[g];
}

// r32 = float((r64 - shift) * scale)
__global__ void k_ir_prepare(int64_t n, const double* __restrict__ r, float* __restrict__ r32,
                             double shift, double scale) {
  GRID_STRIDE(g, n) r32[g] = (float)((r[g] - shift) * scale);
}

// x64 += s * e32
__global__ void k_ir_update(int64_t n, double* __restrict__ x, const float* __restrict__ e,
                            double s) {
  GRID_STRIDE(g, n) x[g] += s * (double)e[g];
}

// --------------------------------------------------------- Chebyshev kernels
//
// Inside a flexible CG (FLEX) the first pass also takes the convergence
// decision from the r.r partials of the update, and the last pass reduces
// z.r and z.(w - mean_w) for beta.

template <bool FLEX>
__device__ __forceinline__ bool cheb_gate(const double* __restrict__ check_in, int nblk,
                                          CgScalars* __restrict__ sc, double* __restrict__ hist) {
  if (!FLEX) return true;
  const int kit = sc->kcur;
  double S[2];  // the update kernel writes two partials per block (r.r and an unused slot)
  block_total<2>(check_in, nblk, S);
  return cg_check(S[0], kit, sc, hist);
}

// d = c0 S r; r_k = r; z = d
template <typename Tr, typename Tp, bool FLEX, bool DOTS>
__global__ __launch_bounds__(kVecBlock) void k_cheb_init(
    int64_t nf, const Tr* __restrict__ r, const Tp* __restrict__ dinv, Tp* __restrict__ d,
    Tp* __restrict__ rk, Tr* __restrict__ z, double c0, const Tr* __restrict__ wcg,
    const double* __restrict__ check_in, int nblk, double* __restrict__ part,
    CgScalars* __restrict__ sc, double* __restrict__ hist) {
  if (sc && sc->done) return;
  if (!cheb_gate<FLEX>(check_in, nblk, sc, hist)) return;
  const double mw = DOTS ? sc->mean_w : 0.0;
  double v[2] = {0.0, 0.0};
  BLOCK_CHUNK(g, nf) {
    const Tp rg = (Tp)r[g];
    const Tp dg = (Tp)c0 * dinv[g] * rg;
    d[g] = dg;
    rk[g] = rg;
    z[g] = (Tr)dg;
    if (DOTS) {
      v[0] += (double)dg * (double)r[g];
      v[1] += (double)dg * ((double)wcg[g] - mw);
    }
  }
  if constexpr (DOTS) block_partials<2>(v, part);
}

// r_k -= R Q^T w_L;  d = a d + b S r_k;  z += d
template <typename Tp, typename Tr, bool DOTS>
__global__ __launch_bounds__(kVecBlock) void k_cheb_step(
    int64_t nf, const int32_t* __restrict__ seg, const int32_t* __restrict__ perm,
    const Tp* __restrict__ wL, Tp* __restrict__ rk, Tp* __restrict__ d,
    const Tp* __restrict__ dinv, Tr* __restrict__ z, double ca, double cb,
    const Tr* __restrict__ rcg, const Tr* __restrict__ wcg, double* __restrict__ part,
    const CgScalars* __restrict__ sc) {
  if (sc && sc->done) return;
  const double mw = DOTS ? sc->mean_w : 0.0;
  double v[2] = {0.0, 0.0};
  BLOCK_CHUNK(g, nf) {
    const Tp s = segment_sum<Tp>(perm, wL, seg[g], seg[g + 1]);
    const Tp rkg = rk[g] - s;
    const Tp dg = (Tp)ca * d[g] + (Tp)cb * dinv[g] * rkg;
    rk[g] = rkg;
    d[g] = dg;
    const Tr zg = z[g] + (Tr)dg;
    z[g] = zg;
    if (DOTS) {
      v[0] += (double)zg * (double)rcg[g];
      v[1] += (double)zg * ((double)wcg[g] - mw);
    }
  }
  if constexpr (DOTS) block_partials<2>(v, part);
}

// ------------------------------------------ Chebyshev fused into the CG
//
// Inside a flexible CG whose preconditioner is Chebyshev of order m >= 2 on
// the split operator (the in-solve operator form, in the preconditioner's
// precision Tp), the pass runs in the CG's own kernels:
//   update:  alpha; x += alpha p; r -= alpha (w - mean_w); r.r partials; and
//            d_0 = c0 S r (no separate start kernel, r itself serves as r_0);
//   step k:  s = R Q^T A d_{k-1}, read at the single-copy nodes from the
//            operator's free-vector output and summed over the surface slots
//            at the shared ones; r_k = r_{k-1} - s; d_k = a_k d_{k-1} + b_k S r_k;
//            z_k = z_{k-1} + d_k (z_0 = d_0);
// the first step takes the convergence decision on the update's r.r
// partials, the last one writes z in Tp (not r_m, d_m) with the z.r and
// z.(w - mean_w) partials for beta.  z is formed in Tp arithmetic anyway,
// so storing it in Tp loses nothing.

// alpha; r -= alpha (w - mean_w); partials of r.r; d0 = c0 S r (x += alpha p
// is left to k_pupdate_flex)
template <typename T, typename Tp>
__global__ __launch_bounds__(kVecBlock) void k_update_cheb0(
    int64_t nf, T* __restrict__ r, const T* __restrict__ w, const Tp* __restrict__ sinv,
    Tp* __restrict__ d0, double c0, const double* __restrict__ part_in, int nblk,
    double* __restrict__ part, CgScalars* __restrict__ sc, double* __restrict__ ahist) {
  if (sc->done) return;
  double alpha, mw;
  if (!cg_alpha(part_in, nblk, sc, ahist, true, alpha, mw)) return;
  const T a = (T)alpha, mwt = (T)mw;
  const Tp c = (Tp)c0;
  double v[2] = {0.0, 0.0};
  BLOCK_CHUNK(g, nf) {
    const T rg = r[g] - a * (w[g] - mwt);
    r[g] = rg;
    d0[g] = c * sinv[g] * (Tp)rg;
    const double rd = (double)rg;
    v[0] += rd * rd;
  }
  block_partials<2>(v, part);
}

// one step of the fused pass (see above); FIRST: r_{k-1} = r (type T) and
// z_{k-1} = d_{k-1}, and the convergence gate; LAST: z_k to z, partials of
// z.r and z.(w - mean_w)
template <typename T, typename Tp, bool FIRST, bool LAST>
__global__ __launch_bounds__(kVecBlock) void k_cheb_fstep(
    int64_t n1, int64_t nf, const int32_t* __restrict__ seg, const int32_t* __restrict__ perm,
    const Tp* __restrict__ wf, const Tp* __restrict__ wL, const T* __restrict__ r,
    Tp* __restrict__ rk, Tp* __restrict__ d, const Tp* __restrict__ sinv, Tp* __restrict__ za,
    Tp* __restrict__ z, const T* __restrict__ w, double ca, double cb,
    const double* __restrict__ check_in, int nblk, double* __restrict__ part,
    CgScalars* __restrict__ sc, double* __restrict__ hist) {
  if (sc->done) return;
  if (FIRST && !cheb_gate<true>(check_in, nblk, sc, hist)) return;
  const double mw = LAST ? sc->mean_w : 0.0;
  const Tp a = (Tp)ca, b = (Tp)cb;
  double v[2] = {0.0, 0.0};
  auto step = [&](int64_t g, Tp s) {
    const Tp rprev = FIRST ? (Tp)r[g] : rk[g];
    const Tp dprev = d[g];
    const Tp rkg = rprev - s;
    const Tp dg = a * dprev + b * sinv[g] * rkg;
    const Tp zg = (FIRST ? dprev : za[g]) + dg;
    if constexpr (LAST) {
      z[g] = zg;
      v[0] += (double)zg * (double)r[g];
      v[1] += (double)zg * ((double)w[g] - mw);
    } else {
      rk[g] = rkg;
      d[g] = dg;
      za[g] = zg;
    }
  };
  // every block takes a chunk of the single-copy nodes [0, n1) and one of the
  // shared nodes [n1, nf), so the segmented sums are spread over all blocks
  {
    BLOCK_CHUNK(g, n1) step(g, wf[g]);
  }
  {
    BLOCK_CHUNK(i, nf - n1) {
      const int64_t g = n1 + i;
      step(g, segment_sum<Tp>(perm, wL, seg[g], seg[g + 1]));
    }
  }
  if constexpr (LAST) block_partials<2>(v, part);
}

// ------------------------------------------- fixed-count CG on the device
//
// The coarsest level of the multigrid cycle runs a fixed number of Jacobi-PCG
// iterations from zero with no host read-back: the initial scalars are formed
// on the device and the usual iteration kernels follow.  Every kernel returns
// at once when the enclosing solve (`outer`) has finished.

// partials of sum(b) (mean of a singular problem's right-hand side)
template <typename T>
__global__ __launch_bounds__(kVecBlock) void k_fcg_sum(int64_t nf, const T* __restrict__ b,
                                                       double* __restrict__ part,
                                                       const CgScalars* __restrict__ outer) {
  if (outer && outer->done) return;
  double v[1] = {0.0};
  BLOCK_CHUNK(g, nf) v[0] += (double)b[g];
  block_partials<1>(v, part);
}

// x = 0; r = b (minus its mean when singular); p = S r; partials of r.p
template <typename T>
__global__ __launch_bounds__(kVecBlock) void k_fcg_init(
    int64_t nf, const T* __restrict__ b, T* __restrict__ x, T* __restrict__ r, T* __restrict__ p,
    const T* __restrict__ dinv, const double* __restrict__ part_in, int nblk, int neumann,
    double inv_n, double* __restrict__ part, const CgScalars* __restrict__ outer) {
  if (outer && outer->done) return;
  double mean = 0.0;
  if (neumann) {
    double S[1];
    block_total<1>(part_in, nblk, S);
    mean = S[0] * inv_n;
  }
  const T mt = (T)mean;
  double v[1] = {0.0};
  BLOCK_CHUNK(g, nf) {
    const T rg = b[g] - mt;
    const T pg = dinv[g] * rg;
    x[g] = T(0);
    r[g] = rg;
    p[g] = pg;
    v[0] += (double)rg * (double)pg;
  }
  block_partials<1>(v, part);
}

// one block: the solve's scalars from the r.p partials (done at once when the
// enclosing solve has finished or the right-hand side vanishes)
__global__ __launch_bounds__(kVecBlock) void k_fcg_scalars(const double* __restrict__ part,
                                                           int nblk, CgScalars* __restrict__ sc,
                                                           int iters, int neumann, double inv_n,
                                                           const CgScalars* __restrict__ outer) {
  double S[1];
  block_total<1>(part, nblk, S);
  if (threadIdx.x == 0) {
    const double rho = S[0];
    const bool stop = (outer && outer->done) || !(rho > 0.0) || !finite(rho) || iters <= 0;
    sc->rho = rho;
    sc->alpha = 0.0;
    sc->beta = 0.0;
    sc->bb = 0.0;
    sc->tol2 = 0.0;
    sc->rr = 0.0;
    sc->mean_w = 0.0;
    sc->inv_n = inv_n;
    sc->zw = 0.0;
    sc->it = 0;
    sc->done = stop ? 1 : 0;
    sc->status = 0;
    sc->max_it = iters;
    sc->fixed = 1;
    sc->neumann = neumann;
    sc->flexible = 0;
    sc->kcur = 0;
    sc->rho2[0] = rho;
    sc->rho2[1] = 0.0;
  }
}

// convergence decision of a flexible CG iteration whose preconditioner does
// not take it itself (one block; the update wrote two partials per block)
__global__ __launch_bounds__(kVecBlock) void k_gate(const double* __restrict__ check_in, int nblk,
                                                    CgScalars* __restrict__ sc,
                                                    double* __restrict__ hist) {
  if (sc->done) return;
  const int kit = sc->kcur;
  double S[2];
  block_total<2>(check_in, nblk, S);
  (void)cg_check(S[0], kit, sc, hist);
}

// z = x (to the CG's type); with a solve: partials of z.r and z.(w - mean_w)
template <typename Tr, typename Tp>
__global__ __launch_bounds__(kVecBlock) void k_flex_dots(int64_t nf, const Tp* __restrict__ x,
                                                         Tr* __restrict__ z,
                                                         const Tr* __restrict__ r,
                                                         const Tr* __restrict__ w,
                                                         double* __restrict__ part,
                                                         const CgScalars* __restrict__ sc) {
  if (sc && sc->done) return;
  const double mw = sc ? sc->mean_w : 0.0;
  double v[2] = {0.0, 0.0};
  BLOCK_CHUNK(g, nf) {
    const Tr zg = (Tr)x[g];
    z[g] = zg;
    if (sc) {
      v[0] += (double)zg * (double)r[g];
      v[1] += (double)zg * ((double)w[g] - mw);
    }
  }
  if (sc) block_partials<2>(v, part);
}

template <typename Tin, typename Tout>
__global__ void k_convert_skip(int64_t n, const Tin* __restrict__ a, Tout* __restrict__ b,
                               const CgScalars* __restrict__ sc) {
  if (sc && sc->done) return;
  GRID_STRIDE(g, n) b[g] = (Tout)a[g];
}

inline unsigned vgrid(int64_t n) {
  int64_t b = (n + kVecBlock - 1) / kVecBlock;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, kReduceBlocks));
}

}  // namespace

// ------------------------------------------------------------ SolveWork

sem_status SolveWork::capture_stream(hipStream_t* out) {
  if (!cap) SEM_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  *out = cap;
  return SEM_OK;
}

SolveWork::~SolveWork() {
  if (cap) (void)hipStreamDestroy(cap);
  if (h_sc) (void)hipHostFree(h_sc);
  if (h_red) (void)hipHostFree(h_red);
  for (auto& e : ev) (void)hipEventDestroy(e);
}

sem_status SolveWork::init(const sem_mesh* m, int max_iter) {
  const int64_t nf = std::max<int64_t>(m->n_free, 1);
  if (!h_sc) SEM_HIP(hipHostMalloc((void**)&h_sc, 4 * sizeof(CgScalars)));
  if (!h_red) SEM_HIP(hipHostMalloc((void**)&h_red, 64 * sizeof(double)));
  sem_status st;
  if ((st = part.ensure(3 * kReduceBlocks * kMaxReduce * sizeof(double)))) return st;
  if ((st = sc.ensure(sizeof(CgScalars)))) return st;
  if ((st = red.ensure(64 * sizeof(double)))) return st;
  const size_t hb = (size_t)(max_iter + 2) * sizeof(double);
  if ((st = hist.ensure(hb)) || (st = ahist.ensure(hb)) || (st = bhist.ensure(hb))) return st;
  (void)nf;
  return SEM_OK;
}

template <typename T>
T* SolveWork::vec(DevBuf& b, int64_t n) {
  if (b.ensure((size_t)std::max<int64_t>(n, 1) * sizeof(T)) != SEM_OK) return nullptr;
  return b.as<T>();
}
template double* SolveWork::vec<double>(DevBuf&, int64_t);
template float* SolveWork::vec<float>(DevBuf&, int64_t);

// ----------------------------------------------------- small host helpers

template <typename T>
static sem_status reduce_dots(const sem_mesh* m, SolveWork& W, const T* a, const T* b, double out[3],
                              hipStream_t s) {
  const int64_t nf = m->n_free;
  const unsigned nb = vgrid(nf);
  hipLaunchKernelGGL((k_dots<T>), dim3(nb), dim3(kVecBlock), 0, s, nf, a, b, W.part.as<double>());
  hipLaunchKernelGGL((k_totals<3>), dim3(1), dim3(kVecBlock), 0, s, W.part.as<double>(), (int)nb,
                     W.red.as<double>());
  SEM_CHECK_LAUNCH("dot products");
  SEM_HIP(hipMemcpyAsync(W.h_red, W.red.p, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < 3; ++i) out[i] = W.h_red[i];
  return SEM_OK;
}

template <typename T>
static sem_status remove_mean(const sem_mesh* m, SolveWork& W, T* a, hipStream_t s) {
  double d[3];
  sem_status st = reduce_dots<T>(m, W, a, nullptr, d, s);
  if (st) return st;
  const double mean = d[2] / (double)m->n_free;
  hipLaunchKernelGGL((k_shift<T>), dim3(vgrid(m->n_free)), dim3(kVecBlock), 0, s, m->n_free, a, mean);
  SEM_CHECK_LAUNCH("mean removal");
  return SEM_OK;
}

// ----------------------------------------------------------- the operator

template <typename T>
sem_status apply_op(const sem_mesh* m, SolveWork& W, const Op<T>& op, const T* xf, T* wL,
                    hipStream_t s, bool timed, T* wf, double* epart, bool mean_sums) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timed) {
    if (W.ev_used + 2 > (int)W.ev.size()) {
      hipEvent_t a, b;
      SEM_HIP(hipEventCreate(&a));
      SEM_HIP(hipEventCreate(&b));
      W.ev.push_back(a);
      W.ev.push_back(b);
    }
    e0 = W.ev[W.ev_used];
    e1 = W.ev[W.ev_used + 1];
    W.ev_used += 2;
  }
  // timed: the runtime stamps e0 / e1 with the kernel's own start and end
  hipError_t e =
      wf ? launch_ax_split<T>(m, xf, wf, wL, epart, mean_sums, op.k, op.h2, op.G, op.B, op.D, s,
                              op.skip, e0, e1)
         : launch_ax<T>(m, xf, m->lmap.as<int32_t>(), wL, op.k, op.h2, op.G, op.B, op.D, s,
                        op.skip, op.lp, e0, e1);
  if (e != hipSuccess) return hip_fail(e, "operator kernel");
  return SEM_OK;
}
template sem_status apply_op<double>(const sem_mesh*, SolveWork&, const Op<double>&, const double*,
                                     double*, hipStream_t, bool, double*, double*, bool);
template sem_status apply_op<float>(const sem_mesh*, SolveWork&, const Op<float>&, const float*,
                                    float*, hipStream_t, bool, float*, double*, bool);

// ------------------------------------------------------ Chebyshev on device

// fourth kind (default) or first kind on [lmax/10, lmax]: the kernels take
// d = c0 S r, then d = ca d + cb S r_k; only the coefficients differ
void cheb_coeffs(int order, double lmax, int kind, double* c0, std::vector<double>& ca,
                 std::vector<double>& cb) {
  const bool first = (kind == 1);
  const double lo = lmax / 10.0, theta = 0.5 * (lmax + lo), delta = 0.5 * (lmax - lo);
  const double sigma = theta / delta;
  double rho_prev = 1.0 / sigma;
  *c0 = first ? 1.0 / theta : 4.0 / (3.0 * lmax);
  ca.assign(std::max(order, 1), 0.0);
  cb.assign(std::max(order, 1), 0.0);
  for (int k = 1; k < order; ++k) {
    if (first) {
      const double rho = 1.0 / (2.0 * sigma - rho_prev);
      ca[k] = rho * rho_prev;
      cb[k] = 2.0 * rho / delta;
      rho_prev = rho;
    } else {
      ca[k] = (2.0 * k - 1.0) / (2.0 * k + 3.0);
      cb[k] = (8.0 * k + 4.0) / ((2.0 * k + 3.0) * lmax);
    }
  }
}

template <typename Tr, typename Tp>
sem_status cheb_apply_dev(const sem_mesh* m, SolveWork& W, const Op<Tp>& op, const Tp* dinv,
                          const Tr* r, Tr* z, int order, double lmax, const ChebCg& cg,
                          hipStream_t s, int* applies, int kind) {
  ChebBufs<Tp> b;
  b.d = W.vec<Tp>(sizeof(Tp) == 8 ? W.cd : W.cd32, m->n_free);
  b.rk = W.vec<Tp>(sizeof(Tp) == 8 ? W.crk : W.crk32, m->n_free);
  b.wL = W.vec<Tp>(sizeof(Tp) == 8 ? W.wL : W.wL32, m->nL);
  if (!b.d || !b.rk || !b.wL) return fail(SEM_ENOMEM, "Chebyshev work space");
  return cheb_apply_bufs<Tr, Tp>(m, op, dinv, r, z, order, lmax, cg, s, applies, kind, b);
}

template <typename Tr, typename Tp>
sem_status cheb_apply_bufs(const sem_mesh* m, const Op<Tp>& op, const Tp* dinv, const Tr* r,
                           Tr* z, int order, double lmax, const ChebCg& cg, hipStream_t s,
                           int* applies, int kind, const ChebBufs<Tp>& b) {
  const int64_t nf = m->n_free;
  const unsigned nb = vgrid(nf);
  Tp* d = b.d;
  Tp* rk = b.rk;
  Tp* wL = b.wL;
  const bool flex = cg.sc != nullptr;
  const Tr* wcg = static_cast<const Tr*>(cg.w);
  double c0;
  std::vector<double> cav, cbv;
  cheb_coeffs(order, lmax, kind, &c0, cav, cbv);
  Op<Tp> opk = op;
  if (flex) opk.skip = &cg.sc->done;
  else if (cg.skip_sc) opk.skip = &cg.skip_sc->done;
  CgScalars* skip_sc = const_cast<CgScalars*>(cg.skip_sc);
  if (flex && order == 1)
    hipLaunchKernelGGL((k_cheb_init<Tr, Tp, true, true>), dim3(nb), dim3(kVecBlock), 0, s, nf, r,
                       dinv, d, rk, z, c0, wcg, cg.check_in, cg.nblk, cg.part_out, cg.sc,
                       cg.hist);
  else if (flex)
    hipLaunchKernelGGL((k_cheb_init<Tr, Tp, true, false>), dim3(nb), dim3(kVecBlock), 0, s, nf, r,
                       dinv, d, rk, z, c0, wcg, cg.check_in, cg.nblk, cg.part_out, cg.sc,
                       cg.hist);
  else
    hipLaunchKernelGGL((k_cheb_init<Tr, Tp, false, false>), dim3(nb), dim3(kVecBlock), 0, s, nf, r,
                       dinv, d, rk, z, c0, wcg, cg.check_in, cg.nblk, cg.part_out, skip_sc,
                       cg.hist);
  SEM_CHECK_LAUNCH("Chebyshev init");
  for (int k = 1; k < order; ++k) {
    const hipError_t e = launch_ax<Tp>(m, d, m->lmap.as<int32_t>(), wL, opk.k, opk.h2, opk.G,
                                       opk.B, opk.D, s, opk.skip, opk.lp);
    if (e != hipSuccess) return hip_fail(e, "operator kernel");
    if (applies) ++*applies;
    const double ca = cav[k], cb = cbv[k];
    if (flex && k == order - 1)
      hipLaunchKernelGGL((k_cheb_step<Tp, Tr, true>), dim3(nb), dim3(kVecBlock), 0, s, nf,
                         m->fseg.as<int32_t>(), m->fperm.as<int32_t>(), wL, rk, d, dinv, z, ca, cb,
                         r, wcg, cg.part_out, cg.sc);
    else
      hipLaunchKernelGGL((k_cheb_step<Tp, Tr, false>), dim3(nb), dim3(kVecBlock), 0, s, nf,
                         m->fseg.as<int32_t>(), m->fperm.as<int32_t>(), wL, rk, d, dinv, z, ca, cb,
                         r, wcg, cg.part_out, flex ? cg.sc : cg.skip_sc);
    SEM_CHECK_LAUNCH("Chebyshev step");
  }
  return SEM_OK;
}
template sem_status cheb_apply_dev<double, double>(const sem_mesh*, SolveWork&, const Op<double>&,
                                                   const double*, const double*, double*, int,
                                                   double, const ChebCg&, hipStream_t, int*, int);
template sem_status cheb_apply_dev<double, float>(const sem_mesh*, SolveWork&, const Op<float>&,
                                                  const float*, const double*, double*, int, double,
                                                  const ChebCg&, hipStream_t, int*, int);
template sem_status cheb_apply_dev<float, float>(const sem_mesh*, SolveWork&, const Op<float>&,
                                                 const float*, const float*, float*, int, double,
                                                 const ChebCg&, hipStream_t, int*, int);
template sem_status cheb_apply_bufs<double, double>(const sem_mesh*, const Op<double>&,
                                                    const double*, const double*, double*, int,
                                                    double, const ChebCg&, hipStream_t, int*, int,
                                                    const ChebBufs<double>&);
template sem_status cheb_apply_bufs<double, float>(const sem_mesh*, const Op<float>&,
                                                   const float*, const double*, double*, int,
                                                   double, const ChebCg&, hipStream_t, int*, int,
                                                   const ChebBufs<float>&);

// ------------------------------------------------------------------- CG

template <typename T, typename Tp>
sem_status cg_solve(const sem_mesh* m, SolveWork& W, const CgArgs<T, Tp>& a, CgResult& res,
                    hipStream_t s) {
  const int64_t nf = m->n_free;
  const unsigned nb = vgrid(nf);
  const bool jac = (a.precond == SEM_PRECOND_JACOBI);
  double* part = W.part.as<double>();
  CgScalars* sc = W.sc.as<CgScalars>();
  sem_status st;
  res = CgResult();

  T* x = a.x;
  T* r = a.r;
  T* p = a.p;
  T* w = a.w;
  T* z = a.z;
  T* wL = a.wL;

  // r = b - A x0 (or b)
  if (a.x_zero) {
    SEM_HIP(launch_fill<T>(x, nf, T(0), s));
    hipLaunchKernelGGL((k_copy<T>), dim3(vgrid(nf)), dim3(kVecBlock), 0, s, nf, a.b, r);
    SEM_CHECK_LAUNCH("copy");
  } else {
    if ((st = apply_op<T>(m, W, a.op, x, wL, s, a.profile))) return st;
    res.applies++;
    hipLaunchKernelGGL((k_residual<T>), dim3(nb), dim3(kVecBlock), 0, s, nf, m->fseg.as<int32_t>(),
                       m->fperm.as<int32_t>(), wL, a.b, r, part);
    SEM_CHECK_LAUNCH("residual");
  }
  double bd[3], rd[3];
  if ((st = reduce_dots<T>(m, W, a.b, nullptr, bd, s))) return st;
  if ((st = reduce_dots<T>(m, W, r, nullptr, rd, s))) return st;
  const double bb = bd[0], rr0 = rd[0];
  res.bnorm = std::sqrt(bb);
  res.rnorm = std::sqrt(rr0);
  if (a.hist) a.hist[0] = res.rnorm;
  if (bb == 0.0 || !std::isfinite(bb)) {
    if (!std::isfinite(bb)) return fail(SEM_EINVAL, "right-hand side is not finite");
    SEM_HIP(launch_fill<T>(x, nf, T(0), s));
    res.converged = true;
    return SEM_OK;
  }
  const double tol2 = a.rtol * a.rtol * bb;
  if (!a.fixed && rr0 <= tol2) {
    res.converged = true;
    return SEM_OK;
  }

  // z0 = M r0, p0 = z0, rho = r0.z0
  // (Jacobi: from here on r holds z = S r; nothing reads r after the solve)
  if (jac) {
    hipLaunchKernelGGL((k_init_pz<T>), dim3(nb), dim3(kVecBlock), 0, s, nf, p, r, a.dinv, part);
  } else {
    if ((st = a.cheb(m, W, r, z, ChebCg(), s, &res.applies))) return st;
    hipLaunchKernelGGL((k_init_p<T>), dim3(nb), dim3(kVecBlock), 0, s, nf, p, r, z, part);
  }
  hipLaunchKernelGGL((k_totals<1>), dim3(1), dim3(kVecBlock), 0, s, part, (int)nb, W.red.as<double>());
  SEM_CHECK_LAUNCH("initial direction");
  SEM_HIP(hipMemcpyAsync(W.h_red, W.red.p, sizeof(double), hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  const double rho0 = W.h_red[0];
  if (!(rho0 > 0.0) || !std::isfinite(rho0)) {
    res.status = 2;
    return SEM_OK;
  }

  CgScalars h{};
  h.rho = rho0;
  h.rho2[0] = rho0;
  h.bb = bb;
  h.tol2 = tol2;
  h.rr = rr0;
  h.inv_n = 1.0 / (double)nf;
  h.it = 0;
  h.done = 0;
  h.status = 0;
  h.max_it = a.max_it;
  h.fixed = a.fixed ? 1 : 0;
  h.neumann = a.neumann ? 1 : 0;
  h.flexible = jac ? 0 : 1;
  W.h_sc[3] = h;
  SEM_HIP(hipMemcpyAsync(sc, &W.h_sc[3], sizeof(CgScalars), hipMemcpyHostToDevice, s));

  double* hist = W.hist.as<double>();
  double* ahist = W.ahist.as<double>();
  double* bhist = W.bhist.as<double>();

  Op<T> op_it = a.op;
  op_it.skip = &sc->done;
  double* partA = part;
  double* partB = part + kReduceBlocks * kMaxReduce;
  double* partC = part + 2 * kReduceBlocks * kMaxReduce;
  // single-copy free nodes leave the operator directly (see launch_ax_split)
  const bool split = op_it.lp == 0 && ax_split_available(m);
  const int64_t nparts = split ? m->E * ax_split_parts(m->N) : 0;
  double* epart = split ? W.vec<double>(W.epart, 2 * nparts) : nullptr;
  if (split && !epart) return fail(SEM_ENOMEM, "work space");
  // Chebyshev fused into the iteration's kernels (needs the split operator)
  const ChebFuse<Tp>& fu = a.fuse;
  const bool fused = !jac && fu.on && split && fu.order >= 2 && fu.op.lp == 0;
  Op<Tp> fop = fu.op;
  fop.skip = &sc->done;
  Tp *fd = nullptr, *frk = nullptr, *fwf = nullptr, *fza = nullptr, *fz = nullptr, *fwL = nullptr;
  double fc0 = 0.0;
  std::vector<double> fca, fcb;
  if (fused) {
    fd = W.vec<Tp>(sizeof(Tp) == 8 ? W.cd : W.cd32, nf);
    frk = W.vec<Tp>(sizeof(Tp) == 8 ? W.crk : W.crk32, nf);
    fwf = W.vec<Tp>(W.cwf, nf);
    fza = W.vec<Tp>(W.cza, nf);
    fz = W.vec<Tp>(W.cz, nf);
    fwL = W.vec<Tp>(sizeof(Tp) == 8 ? W.wL : W.wL32, m->nL);
    if (!fd || !frk || !fwf || !fza || !fz || !fwL) return fail(SEM_ENOMEM, "Chebyshev work space");
    cheb_coeffs(fu.order, fu.lmax, fu.kind, &fc0, fca, fcb);
  }
  auto fused_pass = [&](hipStream_t ss) -> sem_status {
    hipLaunchKernelGGL((k_update_cheb0<T, Tp>), dim3(nb), dim3(kVecBlock), 0, ss, nf, r, w,
                       fu.dinv, fd, fc0, partA, (int)nb, partB, sc, ahist);
    for (int k = 1; k < fu.order; ++k) {
      const hipError_t he = launch_ax_split<Tp>(m, fd, fwf, fwL, nullptr, false, fop.k, fop.h2,
                                                fop.G, fop.B, fop.D, ss, fop.skip);
      if (he != hipSuccess) return hip_fail(he, "Chebyshev operator");
      const bool first = (k == 1), last = (k == fu.order - 1);
#define SEM_FSTEP(F, L)                                                                        \
  hipLaunchKernelGGL((k_cheb_fstep<T, Tp, F, L>), dim3(nb), dim3(kVecBlock), 0, ss, m->n_single, \
                     nf, m->fseg.as<int32_t>(), m->fperm2.as<int32_t>(), fwf, fwL, r, frk, fd,    \
                     fu.dinv, fza, fz, w, fca[k], fcb[k], partB, (int)nb, partC, sc, hist)
      if (first && last) SEM_FSTEP(true, true);
      else if (first) SEM_FSTEP(true, false);
      else if (last) SEM_FSTEP(false, true);
      else SEM_FSTEP(false, false);
#undef SEM_FSTEP
    }
    hipLaunchKernelGGL((k_pupdate_flex<T, Tp>), dim3(nb), dim3(kVecBlock), 0, ss, nf, p, x, fz,
                       partC, (int)nb, sc, bhist);
    return SEM_OK;
  };
  auto iteration = [&](hipStream_t ss) -> sem_status {
    sem_status e;
    if (split && jac) {
      // the segmented sum folded into the residual update; the operator's
      // sums reduced by a grid of kEpartBlocks (a short head reduction for
      // every block of the update)
      if ((e = apply_op<T>(m, W, op_it, p, wL, ss, a.profile, w, epart, a.neumann))) return e;
      hipLaunchKernelGGL(k_epart_sum, dim3(kEpartBlocks), dim3(kVecBlock), 0, ss, nparts, epart,
                         partA, sc);
      hipLaunchKernelGGL((k_update_split<T>), dim3(nb), dim3(kVecBlock), 0, ss, m->n_single, nf,
                         m->fseg.as<int32_t>(), m->fperm2.as<int32_t>(), wL, r, w, a.dinv, partA,
                         kEpartBlocks, partB, sc, ahist);
      hipLaunchKernelGGL((k_pupdate_jac<T, true>), dim3(nb), dim3(kVecBlock), 0, ss, nf, p, x, r,
                         a.dinv, partB, (int)nb, sc, hist, bhist);
      SEM_CHECK_LAUNCH("CG iteration");
      return SEM_OK;
    }
    if (split) {
      if ((e = apply_op<T>(m, W, op_it, p, wL, ss, a.profile, w, epart, a.neumann))) return e;
      hipLaunchKernelGGL((k_gsum_split_pw<T>), dim3(nb), dim3(kVecBlock), 0, ss, m->n_single,
                         nf, m->fseg.as<int32_t>(), m->fperm2.as<int32_t>(), wL, w, nparts,
                         epart, partA, sc);
    } else {
      if ((e = apply_op<T>(m, W, op_it, p, wL, ss, a.profile))) return e;
      hipLaunchKernelGGL((k_gsum_pw<T>), dim3(nb), dim3(kVecBlock), 0, ss, nf,
                         m->fseg.as<int32_t>(), m->fperm.as<int32_t>(), wL, p, w, partA, sc);
    }
    if (jac) {
      hipLaunchKernelGGL((k_update<T, kUpdJacZ>), dim3(nb), dim3(kVecBlock), 0, ss, nf, x, p, r,
                         w, a.dinv, partA, (int)nb, partB, sc, ahist);
      hipLaunchKernelGGL((k_pupdate_jac<T, true>), dim3(nb), dim3(kVecBlock), 0, ss, nf, p, x, r,
                         a.dinv, partB, (int)nb, sc, hist, bhist);
    } else if (fused) {
      if ((e = fused_pass(ss))) return e;
    } else {
      hipLaunchKernelGGL((k_update<T, kUpdR>), dim3(nb), dim3(kVecBlock), 0, ss, nf, x, p, r, w,
                         a.dinv, partA, (int)nb, partB, sc, ahist);
      ChebCg cg;
      cg.sc = sc;
      cg.w = w;
      cg.check_in = partB;
      cg.nblk = (int)nb;
      cg.part_out = partC;
      cg.hist = hist;
      if ((e = a.cheb(m, W, r, z, cg, ss, nullptr))) return e;
      hipLaunchKernelGGL((k_pupdate_flex<T, T>), dim3(nb), dim3(kVecBlock), 0, ss, nf, p, x, z,
                         partC, (int)nb, sc, bhist);
    }
    SEM_CHECK_LAUNCH("CG iteration");
    return SEM_OK;
  };

  // Iterations between convergence read-backs; one chunk is always queued
  // ahead of the one being polled, and kernels of a finished solve return at
  // once, so overshooting the last iteration costs only empty launches.
  int chunk = a.check_every;
  if (chunk <= 0)
    chunk = (int)std::max<int64_t>(
        1, std::min<int64_t>(a.max_chunk, 2000000 / std::max<int64_t>(nf, 1)));
  chunk = std::max(1, std::min(chunk, std::max(a.max_it, 1)));
  // Small problems are launch-bound: capture one chunk of iterations as a HIP
  // graph (the iteration index lives on the device, so the same graph serves
  // every chunk) and replay it.
  hipGraphExec_t gexec = nullptr;
  struct GraphGuard {
    hipGraphExec_t* g;
    ~GraphGuard() {
      if (*g) (void)hipGraphExecDestroy(*g);
    }
  } gguard{&gexec};
  if (!a.profile && nf <= graph_max_free() && a.max_it > 0) {
    hipStream_t cs;
    if ((st = W.capture_stream(&cs))) return st;
    SEM_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    sem_status cst = SEM_OK;
    for (int c = 0; c < chunk && !cst; ++c) cst = iteration(cs);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(cs, &graph);
    if (cst) {
      if (graph) (void)hipGraphDestroy(graph);
      return cst;
    }
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
    ce = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ce != hipSuccess) {
      gexec = nullptr;
      return hip_fail(ce, "hipGraphInstantiate");
    }
  }
  auto run_chunk = [&](int n) -> sem_status {
    if (gexec) {
      SEM_HIP(hipGraphLaunch(gexec, s));
      return SEM_OK;
    }
    for (int c = 0; c < n; ++c) {
      sem_status e = iteration(s);
      if (e) return e;
    }
    return SEM_OK;
  };

  int enq = 0;
  if (a.fixed) {
    while (enq < a.max_it) {
      const int n_now = gexec ? chunk : a.max_it - enq;
      if ((st = run_chunk(n_now))) return st;
      enq += n_now;
    }
    SEM_HIP(hipMemcpyAsync(&W.h_sc[0], sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    h = W.h_sc[0];
  } else {
    hipEvent_t evs[2];
    SEM_HIP(hipEventCreateWithFlags(&evs[0], hipEventDisableTiming));
    SEM_HIP(hipEventCreateWithFlags(&evs[1], hipEventDisableTiming));
    int slot = 0;
    bool have_prev = false;
    bool finished = false;
    while (!finished) {
      const int n_now = gexec ? chunk : std::min(chunk, a.max_it - enq);
      if ((st = run_chunk(n_now))) break;
      enq += n_now;
      SEM_HIP(hipMemcpyAsync(&W.h_sc[slot], sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
      SEM_HIP(hipEventRecord(evs[slot], s));
      if (have_prev || enq >= a.max_it) {
        const int ps = (enq >= a.max_it) ? slot : 1 - slot;
        SEM_HIP(hipEventSynchronize(evs[ps]));
        if (W.h_sc[ps].done || enq >= a.max_it) {
          if (enq >= a.max_it) SEM_HIP(hipEventSynchronize(evs[slot]));
          finished = true;
        }
      }
      have_prev = true;
      slot = 1 - slot;
    }
    SEM_HIP(hipStreamSynchronize(s));
    (void)hipEventDestroy(evs[0]);
    (void)hipEventDestroy(evs[1]);
    if (st) return st;
    SEM_HIP(hipMemcpy(&W.h_sc[0], sc, sizeof(CgScalars), hipMemcpyDeviceToHost));
    h = W.h_sc[0];
  }
  res.iters = h.it;
  res.applies += h.it + (jac ? 0 : h.it * (a.cheb_order - 1));
  res.rnorm = std::sqrt(h.rr);
  res.status = h.status;
  res.converged = (h.status == 1) || (a.fixed && h.rr <= tol2);
  if (a.hist && h.it > 0)
    SEM_HIP(hipMemcpy(a.hist + 1, hist + 1, h.it * sizeof(double), hipMemcpyDeviceToHost));
  if (a.alpha_out && h.it > 0) {
    a.alpha_out->resize(h.it);
    a.beta_out->resize(h.it);
    SEM_HIP(hipMemcpy(a.alpha_out->data(), ahist, h.it * sizeof(double), hipMemcpyDeviceToHost));
    SEM_HIP(hipMemcpy(a.beta_out->data(), bhist, h.it * sizeof(double), hipMemcpyDeviceToHost));
  }
  return SEM_OK;
}
template sem_status cg_solve<double, double>(const sem_mesh*, SolveWork&, const CgArgs<double, double>&,
                                             CgResult&, hipStream_t);
template sem_status cg_solve<double, float>(const sem_mesh*, SolveWork&, const CgArgs<double, float>&,
                                            CgResult&, hipStream_t);
template sem_status cg_solve<float, float>(const sem_mesh*, SolveWork&, const CgArgs<float, float>&,
                                           CgResult&, hipStream_t);

// ----------------------------------------------------- exported helpers

sem_status free_remove_mean_f64(const sem_mesh* m, SolveWork& W, double* a, hipStream_t s) {
  return remove_mean<double>(m, W, a, s);
}
sem_status free_dots_f64(const sem_mesh* m, SolveWork& W, const double* a, const double* b,
                         double out[3], hipStream_t s) {
  return reduce_dots<double>(m, W, a, b, out, s);
}

sem_status ir_residual(const sem_mesh* m, SolveWork& W, const Op<double>& op, const double* x,
                       const double* b, double* r, double out[2], hipStream_t s, bool timed) {
  double* wL = W.vec<double>(W.wL, m->nL);
  if (!wL) return fail(SEM_ENOMEM, "work space");
  sem_status st = apply_op<double>(m, W, op, x, wL, s, timed);
  if (st) return st;
  const unsigned nb = vgrid(m->n_free);
  hipLaunchKernelGGL((k_residual<double>), dim3(nb), dim3(kVecBlock), 0, s, m->n_free,
                     m->fseg.as<int32_t>(), m->fperm.as<int32_t>(), wL, b, r, W.part.as<double>());
  hipLaunchKernelGGL((k_totals<2>), dim3(1), dim3(kVecBlock), 0, s, W.part.as<double>(), (int)nb,
                     W.red.as<double>());
  SEM_CHECK_LAUNCH("residual");
  SEM_HIP(hipMemcpyAsync(W.h_red, W.red.p, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  out[0] = W.h_red[0];
  out[1] = W.h_red[1];
  return SEM_OK;
}

sem_status ir_prepare(const sem_mesh* m, const double* r, float* r32, double shift, double scale,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_ir_prepare, dim3(vgrid(m->n_free)), dim3(kVecBlock), 0, s, m->n_free, r, r32,
                     shift, scale);
  SEM_CHECK_LAUNCH("refinement prepare");
  return SEM_OK;
}

sem_status ir_update(const sem_mesh* m, double* x, const float* e, double sc, hipStream_t s) {
  hipLaunchKernelGGL(k_ir_update, dim3(vgrid(m->n_free)), dim3(kVecBlock), 0, s, m->n_free, x, e, sc);
  SEM_CHECK_LAUNCH("refinement update");
  return SEM_OK;
}

// ------------------------------------------------ multigrid coarse-level pieces

unsigned vec_grid(int64_t n) { return vgrid(n); }

template <typename T>
sem_status cg_fixed_device(const sem_mesh* m, SolveWork& W, const Op<T>& op, const T* dinv,
                           const T* b, T* x, T* r, T* p, T* w, T* wL, int iters, bool neumann,
                           const CgScalars* outer, hipStream_t s) {
  const int64_t nf = m->n_free;
  const unsigned nb = vgrid(nf);
  double* partA = W.part.as<double>();
  double* partB = partA + kReduceBlocks * kMaxReduce;
  CgScalars* sc = W.sc.as<CgScalars>();
  if (!partA || !sc) return fail(SEM_EINVAL, "coarse solve work space not initialised");
  const double inv_n = 1.0 / (double)std::max<int64_t>(nf, 1);
  if (neumann)
    hipLaunchKernelGGL((k_fcg_sum<T>), dim3(nb), dim3(kVecBlock), 0, s, nf, b, partA, outer);
  hipLaunchKernelGGL((k_fcg_init<T>), dim3(nb), dim3(kVecBlock), 0, s, nf, b, x, r, p, dinv, partA,
                     (int)nb, neumann ? 1 : 0, inv_n, partB, outer);
  hipLaunchKernelGGL(k_fcg_scalars, dim3(1), dim3(kVecBlock), 0, s, partB, (int)nb, sc, iters,
                     neumann ? 1 : 0, inv_n, outer);
  SEM_CHECK_LAUNCH("coarse CG start");
  Op<T> opi = op;
  opi.skip = &sc->done;
  for (int it = 0; it < iters; ++it) {
    sem_status st = apply_op<T>(m, W, opi, p, wL, s, false);
    if (st) return st;
    hipLaunchKernelGGL((k_gsum_pw<T>), dim3(nb), dim3(kVecBlock), 0, s, nf, m->fseg.as<int32_t>(),
                       m->fperm.as<int32_t>(), wL, p, w, partA, sc);
    hipLaunchKernelGGL((k_update<T, kUpdJacR>), dim3(nb), dim3(kVecBlock), 0, s, nf, x, p, r, w, dinv,
                       partA, (int)nb, partB, sc, (double*)nullptr);
    hipLaunchKernelGGL((k_pupdate_jac<T, false>), dim3(nb), dim3(kVecBlock), 0, s, nf, p, x, r, dinv,
                       partB, (int)nb, sc, (double*)nullptr, (double*)nullptr);
  }
  SEM_CHECK_LAUNCH("coarse CG");
  return SEM_OK;
}
template sem_status cg_fixed_device<double>(const sem_mesh*, SolveWork&, const Op<double>&,
                                            const double*, const double*, double*, double*,
                                            double*, double*, double*, int, bool,
                                            const CgScalars*, hipStream_t);
template sem_status cg_fixed_device<float>(const sem_mesh*, SolveWork&, const Op<float>&,
                                           const float*, const float*, float*, float*, float*,
                                           float*, float*, int, bool, const CgScalars*,
                                           hipStream_t);

sem_status launch_cg_gate(const double* check_in, int nblk, CgScalars* sc, double* hist,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_gate, dim3(1), dim3(kVecBlock), 0, s, check_in, nblk, sc, hist);
  SEM_CHECK_LAUNCH("convergence gate");
  return SEM_OK;
}

template <typename Tr, typename Tp>
sem_status launch_flex_dots(int64_t nf, const Tp* x, Tr* z, const Tr* r, const Tr* w,
                            double* part, const CgScalars* sc, hipStream_t s) {
  hipLaunchKernelGGL((k_flex_dots<Tr, Tp>), dim3(vgrid(nf)), dim3(kVecBlock), 0, s, nf, x, z, r,
                     w, part, sc);
  SEM_CHECK_LAUNCH("preconditioner output");
  return SEM_OK;
}
template sem_status launch_flex_dots<double, double>(int64_t, const double*, double*,
                                                     const double*, const double*, double*,
                                                     const CgScalars*, hipStream_t);
template sem_status launch_flex_dots<double, float>(int64_t, const float*, double*, const double*,
                                                    const double*, double*, const CgScalars*,
                                                    hipStream_t);
template sem_status launch_flex_dots<float, float>(int64_t, const float*, float*, const float*,
                                                   const float*, double*, const CgScalars*,
                                                   hipStream_t);

template <typename Tin, typename Tout>
sem_status launch_convert_skip(int64_t n, const Tin* a, Tout* b, const CgScalars* sc,
                               hipStream_t s) {
  hipLaunchKernelGGL((k_convert_skip<Tin, Tout>), dim3(vgrid(n)), dim3(kVecBlock), 0, s, n, a, b,
                     sc);
  SEM_CHECK_LAUNCH("convert");
  return SEM_OK;
}
template sem_status launch_convert_skip<double, float>(int64_t, const double*, float*,
                                                       const CgScalars*, hipStream_t);
template sem_status launch_convert_skip<double, double>(int64_t, const double*, double*,
                                                        const CgScalars*, hipStream_t);
template sem_status launch_convert_skip<float, float>(int64_t, const float*, float*,
                                                      const CgScalars*, hipStream_t);

}  // namespace sem
