// Internal declarations shared by the host drivers and the HIP kernels of libsem.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "sem.h"

namespace sem {

constexpr int kMaxOrder = 10;           // the solver family uses p <= 10 (Sec. 4.1)
constexpr int kVecBlock = 512;          // threads per block of the vector kernels
constexpr int kReduceBlocks = 512;      // fixed grid of reducing kernels (deterministic sums)
constexpr int kMaxReduce = 4;           // values reduced per pass
constexpr int64_t kGraphMaxFree = 262144;  // solves up to this size replay captured iteration graphs

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
sem_status fail(sem_status s, const std::string& msg);
sem_status hip_fail(hipError_t e, const char* what);

#define SEM_HIP(call)                                       \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return ::sem::hip_fail(e_, #call); \
  } while (0)

#define SEM_CHECK_LAUNCH(name)                                   \
  do {                                                           \
    hipError_t e_ = hipGetLastError();                           \
    if (e_ != hipSuccess) return ::sem::hip_fail(e_, name);      \
  } while (0)

// ------------------------------------------------------ device allocation
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  sem_status ensure(size_t nbytes);  // grow-only
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// ----------------------------------------------------------- host numbering
struct HostNumbering {
  int64_t n_unique = 0, n_free = 0, n_shared = 0;
  int64_t n_single = 0;               // free nodes with one local copy: indices [0, n_single)
  std::vector<int32_t> lmap;          // [nL] free index or -1: single-copy nodes first, then
                                      // shared ones, each class in first-touch order
  std::vector<int32_t> fseg, fperm;   // CSR over free unique nodes -> local copies (ascending)
  std::vector<int32_t> gseg, gperm;   // CSR over shared unique nodes (all, incl. Dirichlet)
  std::vector<int32_t> dlist;         // local indices of Dirichlet copies
};
sem_status build_numbering(int N, int64_t E, const int64_t* gid, const uint8_t* dirichlet,
                           HostNumbering& out);
sem_status host_gll(int N, double* xi, double* rho, double* D);

// ------------------------------------------------------ device scalars
// Scalars of a CG iteration, resident on the device: the vector kernels read
// alpha/beta from here so the host never sits between two kernels of an
// iteration; it only polls `done` every few iterations.
struct CgScalars {
  double rho;       // r.z of the current iterate
  double alpha, beta;
  double bb;        // ||b||^2
  double tol2;      // (rtol ||b||)^2
  double rr;        // ||r||^2 of the latest iterate
  double mean_w;    // null-space projection: mean of w over unique nodes
  double inv_n;     // 1 / n_free
  double zw;        // flexible CG: z.w
  double pad[3];
  int32_t it;       // completed iterations
  int32_t done;     // 1 = converged or failed: every later kernel of the solve is a no-op
  int32_t status;   // 0 ok, 1 converged, 2 breakdown, 3 non-finite
  int32_t max_it;
  int32_t fixed;    // 1 = never stop before max_it
  int32_t neumann;  // 1 = project out the constant mode
  int32_t flexible; // 1 = Polak-Ribiere beta
  int32_t kcur;     // index of the iteration in progress (set by the update kernel)
  double rho2[2];   // r.z of iteration k in slot k & 1
  int32_t pending;  // 1 = x += alpha p of iteration kcur still to apply (set by the
                    // residual update, cleared by the next segmented sum; applied by
                    // the direction update)
  int32_t pad2;
};

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b % 8), each with its own L2.  xcd_block() renumbers them so that every
// XCD works on one contiguous range of the index space: neighbouring elements
// and nodes, which share data, then share an L2.  Off by default: measured on
// the benchmark meshes it gained nothing (the memory-side Infinity Cache
// already serves the cross-XCD re-reads); enable with -DSEM_XCD_REMAP=1.
#ifndef SEM_XCD_REMAP
#define SEM_XCD_REMAP 0
#endif
constexpr int kNumXcd = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
#if SEM_XCD_REMAP
  const int64_t x = b % kNumXcd, i = b / kNumXcd;
  const int64_t per = nb / kNumXcd, rem = nb % kNumXcd;
  return x * per + (x < rem ? x : rem) + i;
#else
  (void)nb;
  return b;
#endif
}

// The XCD-contiguous order unconditionally: workgroup b (on XCD b % 8) gets
// place xcd_order(b, nb) in [0, nb), the workgroups of one XCD one
// contiguous range of places.  The stand-alone gather-scatter uses it: its
// neighbouring workgroups read and write the same 32-byte sectors, which
// then pass through one L2 (38 -> 31 us on the 32x32x16, N = 7 box, traffic
// 194 MB -> 162 MB, its sector floor).  In the element operator and the
// multigrid kernels, which mostly read shared sectors, the same order was
// measured 1-4 % slower.
__device__ __forceinline__ int64_t xcd_order(int64_t b, int64_t nb) {
  const int64_t x = b % kNumXcd, i = b / kNumXcd;
  const int64_t per = nb / kNumXcd, rem = nb % kNumXcd;
  return x * per + (x < rem ? x : rem) + i;
}

// Loop over this workgroup's contiguous chunk of [0, n) (chunks follow the
// XCD-aware block order).
#define BLOCK_CHUNK(idx, n)                                                          \
  const int64_t lb_ = xcd_block(blockIdx.x, gridDim.x);                              \
  const int64_t chunk_ = ((int64_t)(n) + gridDim.x - 1) / gridDim.x;                  \
  const int64_t lo_ = lb_ * chunk_;                                                  \
  const int64_t hi_ = lo_ + chunk_ < (int64_t)(n) ? lo_ + chunk_ : (int64_t)(n);       \
  for (int64_t idx = lo_ + threadIdx.x; idx < hi_; idx += blockDim.x)

// lane i of each row of 16 receives lane i - SHIFT's value (0 below the row)
template <int SHIFT>
__device__ __forceinline__ double dpp_row_shr(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x110 + SHIFT, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x110 + SHIFT, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_value(double x, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                          __builtin_amdgcn_readlane(__double2loint(x), l));
}
// Sum over the wavefront, the same on every lane and in a fixed order: a
// scan within each row of 16 by DPP row shifts (lane 15 of a row ends with
// the row's sum), then the four rows in order.  (Six cross-lane
// shuffles per value made the in-solve operator 6 % slower.)
__device__ __forceinline__ double wave_sum_d(double v) {
  v += dpp_row_shr<1>(v);
  v += dpp_row_shr<2>(v);
  v += dpp_row_shr<4>(v);
  v += dpp_row_shr<8>(v);
  return ((lane_value(v, 15) + lane_value(v, 31)) + lane_value(v, 47)) + lane_value(v, 63);
}

// Sum of the local copies perm[a..b) of one global node, in ascending order
// (deterministic).  The index loads of up to 8 copies are issued together,
// then the value loads, instead of one dependent pair per copy.
template <typename Tacc, typename T>
__device__ __forceinline__ Tacc segment_sum(const int32_t* __restrict__ perm,
                                            const T* __restrict__ v, int32_t a, int32_t b) {
  Tacc s = Tacc(0);
  for (int32_t q0 = a; q0 < b; q0 += 8) {
    int32_t idx[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) idx[c] = (q0 + c < b) ? perm[q0 + c] : -1;
    T val[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) val[c] = idx[c] >= 0 ? v[idx[c]] : T(0);
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (q0 + c < b) s += (Tacc)val[c];
  }
  return s;
}

// Position of point (i, j, k) of an order-N element among the element's
// surface points, in a fixed order: the k = 0 layer, then for k = 1..N-1 the
// ring of the layer (row j = 0, the two end points of rows 1..N-1, row j =
// N), then the k = N layer; -1 for an interior point.  The surface has
// 2 (N+1)^2 + 4 N (N-1) points.  The in-solve operator stores shared copies
// at this position of the element's local block (see launch_ax_split).
// Written as selects rather than early returns: the operator evaluates it per
// point in its stores, where branches cost the FP32 kernel several percent.
__host__ __device__ inline int surface_rank(int i, int j, int k, int N) {
  const int n = N + 1;
  const int base = n * n + (k - 1) * 4 * N;
  int r = base + n + 2 * (j - 1) + (i == N ? 1 : 0);  // end points of rows 1..N-1
  r = (i == 0 || i == N) ? r : -1;
  r = j == N ? base + n + 2 * (N - 1) + i : r;
  r = j == 0 ? base + i : r;
  r = k == N ? n * n + (N - 1) * 4 * N + j * n + i : r;
  r = k == 0 ? j * n + i : r;
  return r;
}
__host__ __device__ constexpr int surface_points(int N) {
  return 2 * (N + 1) * (N + 1) + 4 * N * (N - 1);
}

// ------------------------------------------------------------- the mesh
struct SolveWork;
struct Pmg;
struct AdvRule;

}  // namespace sem

struct sem_mesh {
  int N = 0, n1 = 0, P = 0;
  int64_t E = 0, nL = 0, n_unique = 0, n_free = 0, n_shared = 0, n_dloc = 0;
  bool nullspace = false;
  int device = 0;
  double h_D[(sem::kMaxOrder + 1) * (sem::kMaxOrder + 1)];
  sem::DevBuf D64, D32;                 // derivative matrix
  sem::DevBuf G64, B64, G32, B32;       // geometry [E][6][P], [E][P]
  sem::DevBuf lmap, fseg, fperm;        // solver numbering (free unique nodes)
  sem::DevBuf lmap2;                    // in-solve operator routing (see launch_ax_split)
  sem::DevBuf fperm2;                   // fperm with shared copies at their surface slots
  int64_t n_single = 0;                 // free nodes [0, n_single) have one local copy
  bool split_ok = false;                // every shared copy lies on its element's surface
  // the in-solve operator stores shared copies nontemporally when the local
  // array is larger than this (plain stores keep them in the memory-side
  // cache for the segmented sum that follows): 128 MB, or SEM_AX_NT_BYTES
  // read at sem_setup_mesh
  int64_t ax_nt_bytes = int64_t(128) << 20;
  sem::DevBuf gseg, gperm, dlist;       // local gather-scatter tables, Dirichlet copies
  // cached Jacobi inverse and Chebyshev bound for k == NULL
  double cached_h2 = -1.0;
  bool dinv_valid = false;
  double cached_lmax_h2 = -1.0;
  double cached_lmax = 0.0;
  sem::SolveWork* work = nullptr;
  sem::Pmg* pmg = nullptr;              // p-multigrid hierarchy (sem_setup_pmg)
  sem::AdvRule* adv[2] = {nullptr, nullptr};  // convective-term rules (sem_setup_advection)
  ~sem_mesh();
};

namespace sem {

// ----------------------------------------------------------- launchers
// All launchers enqueue on `s` and return hipGetLastError().

// element operator, FP64/FP32; `lmap` != nullptr: gather the input from a
// free-unique vector (x_L = x[lmap], 0 where lmap < 0)
// `skip` (device, nullable): nonzero -> the kernel returns at once
// `lp` (FP32 only): 0 FP32 contractions, 1 bfloat16 and 2 half operands on
// the matrix cores (hipErrorInvalidValue for other values or FP64 with lp != 0)
// ev0 / ev1 (nullable): events stamped with the kernel's own start and end
template <typename T>
hipError_t launch_ax(const sem_mesh* m, const T* u, const int32_t* lmap, T* w, const T* k, T h2,
                     const T* G, const T* B, const T* D, hipStream_t s,
                     const int32_t* skip = nullptr, int lp = 0, hipEvent_t ev0 = nullptr,
                     hipEvent_t ev1 = nullptr);
// In-solve operator with split output (matrix-core kernel, N >= 5, FP64 or
// FP32 contractions): u gathered from the free vector through m->lmap2;
// results at free nodes with one local copy go straight to wf (free
// vector), at shared free nodes to wL at e P + surface_rank (local, for the
// segmented sum over [n_single, n_free) through fperm2); epart[2 (parts e +
// i) + {0, 1}] (parts = ax_split_parts(N), one per wavefront i) = that
// wavefront's sums of u w and of w over its free copies; with mean_sums
// false only entry 0 (u w) is written (sum(w) serves the null-space
// projection alone).  epart nullable: then no sums are formed.
// hipErrorNotSupported when unavailable (see ax_split_available).
template <typename T>
hipError_t launch_ax_split(const sem_mesh* m, const T* u, T* wf, T* wL, double* epart,
                           bool mean_sums, const T* k, T h2, const T* G, const T* B, const T* D, hipStream_t s,
                           const int32_t* skip, hipEvent_t ev0 = nullptr,
                           hipEvent_t ev1 = nullptr);
bool ax_split_available(const sem_mesh* m);
int ax_split_parts(int N);
// kbar = sign sum_ab (D_a wbar) G_ab (D_b u) at every local point
hipError_t launch_ax_kbar(const sem_mesh* m, const double* u, const double* wbar, double* kbar,
                          double sign, hipStream_t s);
template <typename T>
hipError_t launch_mass(int64_t n, const T* B, const T* u, T* w, hipStream_t s);

// setup
hipError_t launch_geometry(const sem_mesh* m, const double* xyz, double* G, double* B, float* G32,
                           float* B32, int* bad_count, hipStream_t s);
hipError_t launch_local_diag(const sem_mesh* m, const double* k, double h2, double* dL,
                             hipStream_t s);

// gather-scatter on local vectors
template <typename T>
hipError_t launch_gs_local(const sem_mesh* m, T* v, hipStream_t s);
template <typename T>
hipError_t launch_mask_local(const sem_mesh* m, T* v, hipStream_t s);

// layout conversions between local copy-consistent vectors and free unique vectors
template <typename Tin, typename Tout>
hipError_t launch_local_to_free_avg(const sem_mesh* m, const Tin* vL, Tout* vf, hipStream_t s);
template <typename Tin, typename Tout>
hipError_t launch_free_to_local(const sem_mesh* m, const Tin* vf, Tout* vL, hipStream_t s);
template <typename Tin, typename Tout>
hipError_t launch_free_sum(const sem_mesh* m, const Tin* wL, Tout* wf, hipStream_t s);
// vL[q] = vf[f] / (copies of f), f = lmap[q] (0 at Dirichlet copies)
hipError_t launch_free_to_local_per_copy(const sem_mesh* m, const double* vf, double* vL,
                                         hipStream_t s);

// generic small kernels
template <typename T>
hipError_t launch_fill(T* p, int64_t n, T v, hipStream_t s);
template <typename Tin, typename Tout>
hipError_t launch_convert(const Tin* a, Tout* b, int64_t n, double scale, hipStream_t s);
hipError_t launch_reciprocal_mask(double* d, float* d32, int64_t n, hipStream_t s);
hipError_t launch_pseudo_random(double* v, int64_t n, uint64_t seed, hipStream_t s);

}  // namespace sem
