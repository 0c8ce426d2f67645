// Gather-scatter and layout kernels.
//
// Direct-stiffness summation (the exchange step of Sec. 2.2) is done by
// sorted-index segmented sums: every global node owns a contiguous segment
// of a permutation listing its local copies in ascending order, so one thread
// per node sums its copies in a fixed order (bit-reproducible, no atomics).
#include <climits>

#include "common.hpp"

namespace sem {
namespace {

inline unsigned grid_for(int64_t n, int64_t cap = 65536) {
  int64_t b = (n + kVecBlock - 1) / kVecBlock;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

#define GRID_STRIDE(idx, n)                                                        \
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < (n); \
       idx += (int64_t)gridDim.x * blockDim.x)

// v <- Q Q^T v on local copies of shared nodes (single-copy nodes are fixed points).
// Workgroups in the XCD-contiguous order (xcd_order): the copies of
// neighbouring nodes, which share 32-byte sectors, are read and written
// through one L2.
template <typename T>
__global__ __launch_bounds__(kVecBlock) void gs_local_kernel(int64_t ns,
                                                             const int32_t* __restrict__ seg,
                                                             const int32_t* __restrict__ perm,
                                                             T* __restrict__ v) {
  const int64_t g = xcd_order(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (g >= ns) return;
  const int32_t a = seg[g], c = seg[g + 1];
  const T s = segment_sum<T>(perm, v, a, c);
  for (int32_t p = a; p < c; ++p) v[perm[p]] = s;
}

template <typename T>
__global__ void mask_kernel(int64_t nd, const int32_t* __restrict__ dlist, T* __restrict__ v) {
  GRID_STRIDE(a, nd) v[dlist[a]] = T(0);
}

// vf[g] = mean of the local copies of free node g
template <typename Tin, typename Tout>
__global__ void local_to_free_avg_kernel(int64_t nf, const int32_t* __restrict__ seg,
                                         const int32_t* __restrict__ perm,
                                         const Tin* __restrict__ vL, Tout* __restrict__ vf) {
  GRID_STRIDE(g, nf) {
    const int32_t a = seg[g], b = seg[g + 1];
    const double s = segment_sum<double>(perm, vL, a, b);
    vf[g] = (Tout)(s / (double)(b - a));
  }
}

// wf[g] = sum of the local copies of free node g  (R Q^T)
template <typename Tin, typename Tout>
__global__ void free_sum_kernel(int64_t nf, const int32_t* __restrict__ seg,
                                const int32_t* __restrict__ perm, const Tin* __restrict__ wL,
                                Tout* __restrict__ wf) {
  GRID_STRIDE(g, nf) {
    wf[g] = (Tout)segment_sum<Tin>(perm, wL, seg[g], seg[g + 1]);
  }
}

// vL[q] = vf[lmap[q]] (0 at Dirichlet copies)  (Q R^T)
template <typename Tin, typename Tout>
__global__ void free_to_local_kernel(int64_t nL, const int32_t* __restrict__ lmap,
                                     const Tin* __restrict__ vf, Tout* __restrict__ vL) {
  GRID_STRIDE(q, nL) {
    const int32_t f = lmap[q];
    vL[q] = f >= 0 ? (Tout)vf[f] : Tout(0);
  }
}

// vL[q] = vf[f] / (number of copies of f), f = lmap[q]; 0 at Dirichlet copies
__global__ void free_to_local_per_copy_kernel(int64_t nL, const int32_t* __restrict__ lmap,
                                              const int32_t* __restrict__ seg,
                                              const double* __restrict__ vf,
                                              double* __restrict__ vL) {
  GRID_STRIDE(q, nL) {
    const int32_t f = lmap[q];
    vL[q] = f >= 0 ? vf[f] / (double)(seg[f + 1] - seg[f]) : 0.0;
  }
}

template <typename T>
__global__ void fill_kernel(T* __restrict__ p, int64_t n, T v) {
  GRID_STRIDE(a, n) p[a] = v;
}

template <typename Tin, typename Tout>
__global__ void convert_kernel(const Tin* __restrict__ a, Tout* __restrict__ b, int64_t n,
                               double scale) {
  GRID_STRIDE(q, n) b[q] = (Tout)((double)a[q] * scale);
}

__global__ void reciprocal_kernel(double* __restrict__ d, float* __restrict__ d32, int64_t n) {
  GRID_STRIDE(q, n) {
    const double r = 1.0 / d[q];
    d[q] = r;
    if (d32) d32[q] = (float)r;
  }
}

// splitmix64 -> uniform in [-1, 1): a fixed pseudo-random start vector
__global__ void pseudo_random_kernel(double* __restrict__ v, int64_t n, uint64_t seed) {
  GRID_STRIDE(q, n) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(q + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    v[q] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

}  // namespace

template <typename T>
hipError_t launch_gs_local(const sem_mesh* m, T* v, hipStream_t s) {
  if (m->n_shared == 0) return hipSuccess;
  // one node per thread (the grid covers every node; no grid-stride loop)
  const int64_t blocks = (m->n_shared + kVecBlock - 1) / kVecBlock;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((gs_local_kernel<T>), dim3((unsigned)blocks), dim3(kVecBlock), 0, s,
                     m->n_shared, m->gseg.as<int32_t>(), m->gperm.as<int32_t>(), v);
  return hipGetLastError();
}
template hipError_t launch_gs_local<double>(const sem_mesh*, double*, hipStream_t);
template hipError_t launch_gs_local<float>(const sem_mesh*, float*, hipStream_t);

template <typename T>
hipError_t launch_mask_local(const sem_mesh* m, T* v, hipStream_t s) {
  if (m->n_dloc == 0) return hipSuccess;
  hipLaunchKernelGGL((mask_kernel<T>), dim3(grid_for(m->n_dloc)), dim3(kVecBlock), 0, s,
                     m->n_dloc, m->dlist.as<int32_t>(), v);
  return hipGetLastError();
}
template hipError_t launch_mask_local<double>(const sem_mesh*, double*, hipStream_t);
template hipError_t launch_mask_local<float>(const sem_mesh*, float*, hipStream_t);

template <typename Tin, typename Tout>
hipError_t launch_local_to_free_avg(const sem_mesh* m, const Tin* vL, Tout* vf, hipStream_t s) {
  if (m->n_free == 0) return hipSuccess;
  hipLaunchKernelGGL((local_to_free_avg_kernel<Tin, Tout>), dim3(grid_for(m->n_free)),
                     dim3(kVecBlock), 0, s, m->n_free, m->fseg.as<int32_t>(),
                     m->fperm.as<int32_t>(), vL, vf);
  return hipGetLastError();
}
template hipError_t launch_local_to_free_avg<double, double>(const sem_mesh*, const double*,
                                                            double*, hipStream_t);

template <typename Tin, typename Tout>
hipError_t launch_free_sum(const sem_mesh* m, const Tin* wL, Tout* wf, hipStream_t s) {
  if (m->n_free == 0) return hipSuccess;
  hipLaunchKernelGGL((free_sum_kernel<Tin, Tout>), dim3(grid_for(m->n_free)), dim3(kVecBlock), 0,
                     s, m->n_free, m->fseg.as<int32_t>(), m->fperm.as<int32_t>(), wL, wf);
  return hipGetLastError();
}
template hipError_t launch_free_sum<double, double>(const sem_mesh*, const double*, double*,
                                                    hipStream_t);

template <typename Tin, typename Tout>
hipError_t launch_free_to_local(const sem_mesh* m, const Tin* vf, Tout* vL, hipStream_t s) {
  hipLaunchKernelGGL((free_to_local_kernel<Tin, Tout>), dim3(grid_for(m->nL)), dim3(kVecBlock), 0,
                     s, m->nL, m->lmap.as<int32_t>(), vf, vL);
  return hipGetLastError();
}
template hipError_t launch_free_to_local<double, double>(const sem_mesh*, const double*, double*,
                                                        hipStream_t);

hipError_t launch_free_to_local_per_copy(const sem_mesh* m, const double* vf, double* vL,
                                         hipStream_t s) {
  hipLaunchKernelGGL(free_to_local_per_copy_kernel, dim3(grid_for(m->nL)), dim3(kVecBlock), 0, s,
                     m->nL, m->lmap.as<int32_t>(), m->fseg.as<int32_t>(), vf, vL);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* p, int64_t n, T v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((fill_kernel<T>), dim3(grid_for(n)), dim3(kVecBlock), 0, s, p, n, v);
  return hipGetLastError();
}
template hipError_t launch_fill<double>(double*, int64_t, double, hipStream_t);
template hipError_t launch_fill<float>(float*, int64_t, float, hipStream_t);
template hipError_t launch_fill<int>(int*, int64_t, int, hipStream_t);

template <typename Tin, typename Tout>
hipError_t launch_convert(const Tin* a, Tout* b, int64_t n, double scale, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((convert_kernel<Tin, Tout>), dim3(grid_for(n)), dim3(kVecBlock), 0, s, a, b,
                     n, scale);
  return hipGetLastError();
}
template hipError_t launch_convert<double, float>(const double*, float*, int64_t, double,
                                                  hipStream_t);
template hipError_t launch_convert<float, double>(const float*, double*, int64_t, double,
                                                  hipStream_t);
template hipError_t launch_convert<double, double>(const double*, double*, int64_t, double,
                                                   hipStream_t);

hipError_t launch_reciprocal_mask(double* d, float* d32, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(reciprocal_kernel, dim3(grid_for(n)), dim3(kVecBlock), 0, s, d, d32, n);
  return hipGetLastError();
}

hipError_t launch_pseudo_random(double* v, int64_t n, uint64_t seed, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(pseudo_random_kernel, dim3(grid_for(n)), dim3(kVecBlock), 0, s, v, n, seed);
  return hipGetLastError();
}

}  // namespace sem
