// sem_cheb_apply_noalloc: the Chebyshev-Jacobi preconditioner of
// sem_cheb_apply with its work space in one fixed device array instead of the
// mesh's lazily allocated buffers, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).
//
// The array `scratch` below is a file-scope device variable: each device the
// library runs on holds its own copy (kScratchBytes) until the process ends.
// Host code never passes the variable's name to a kernel (in host code it
// names a host-side stand-in); the device address is looked up once per device
// with hipGetSymbolAddress on the first call made for a mesh of that device,
// and only that address is used afterwards.
//
// Every call on one device shares that device's array and leaves its last
// contents there.  Nothing in it has to start at zero: each slice is written
// in full by the call before it is read (the local diagonal, the Jacobi
// inverse, the free-node copy of r, the Chebyshev vectors d, r_k, z and the
// element-local operator output).  Calls that overlap in time on one device
// (two streams, or two host threads) race on the array; calls ordered on one
// stream do not.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "common.hpp"
#include "solver.hpp"

// 64 MiB per device
static constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace sem {
namespace {

constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on device `dev` (looked up once per device,
// with that device current)
sem_status scratch_address(int dev, unsigned char** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices) return fail(SEM_EDEVICE, "device index out of range");
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    SEM_HIP(hipGetDevice(&cur));
    if (cur != dev) SEM_HIP(hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(SEM_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return SEM_OK;
}

inline size_t round256(size_t x) { return (x + 255) & ~size_t(255); }

// Offsets of the work vectors in the array.  dL (FP64 local diagonal) is
// consumed by the free-node sum that forms the Jacobi inverse and then
// reused as the operator output w_L of the Chebyshev steps.
struct Layout {
  size_t dL = 0, dinv = 0, dinv32 = 0, rf = 0, zf = 0, d = 0, rk = 0, k32 = 0, total = 0;
};

Layout layout_of(const sem_mesh* m, bool fp64, bool has_k) {
  const size_t nL = (size_t)std::max<int64_t>(m->nL, 1);
  const size_t nf = (size_t)std::max<int64_t>(m->n_free, 1);
  const size_t tp = fp64 ? sizeof(double) : sizeof(float);
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += round256(bytes);
    return at;
  };
  L.dL = take(nL * sizeof(double));
  L.dinv = take(nf * sizeof(double));
  if (!fp64) L.dinv32 = take(nf * sizeof(float));
  L.rf = take(nf * sizeof(double));
  L.zf = take(nf * sizeof(double));
  L.d = take(nf * tp);
  L.rk = take(nf * tp);
  if (!fp64 && has_k) L.k32 = take(nL * sizeof(float));
  L.total = off;
  return L;
}

}  // namespace
}  // namespace sem

using namespace sem;

extern "C" sem_status sem_cheb_apply_noalloc(const sem_mesh* m, const double* r, double* z,
                                             const double* k, double h2, int32_t order,
                                             double lmax, sem_prec prec, void* stream) {
  if (!m) return fail(SEM_EINVAL, "mesh is NULL");
  if (!r || !z) return fail(SEM_EINVAL, "r and z must not be NULL");
  if (order < 1) return fail(SEM_EINVAL, "order must be >= 1");
  if (!(lmax > 0.0) || !std::isfinite(lmax)) return fail(SEM_EINVAL, "lmax must be > 0");
  if (!(h2 >= 0.0) || !std::isfinite(h2)) return fail(SEM_EINVAL, "h2 must be finite and >= 0");
  if (prec != SEM_FP64 && prec != SEM_FP32 && prec != SEM_BF16_MFMA && prec != SEM_FP16_MFMA)
    return fail(SEM_EINVAL, "unknown precision");
  const bool fp64 = (prec == SEM_FP64);
  const Layout L = layout_of(m, fp64, k != nullptr);
  if (L.total > kScratchBytes)
    return fail(SEM_EINVAL, "sem_cheb_apply_noalloc: this mesh needs " + std::to_string(L.total) +
                                " bytes of work space, more than the fixed " +
                                std::to_string(kScratchBytes) +
                                "-byte device array holds (use sem_cheb_apply)");
  unsigned char* base = nullptr;
  if (sem_status st = scratch_address(m->device, &base)) return st;
  hipStream_t s = (hipStream_t)stream;
  double* dL = reinterpret_cast<double*>(base + L.dL);
  double* dinv = reinterpret_cast<double*>(base + L.dinv);
  float* dinv32 = fp64 ? nullptr : reinterpret_cast<float*>(base + L.dinv32);
  double* rf = reinterpret_cast<double*>(base + L.rf);
  double* zf = reinterpret_cast<double*>(base + L.zf);

  // Jacobi inverse on the free nodes (the kernels sem_cheb_apply uses)
  SEM_HIP(launch_local_diag(m, k, h2, dL, s));
  SEM_HIP((launch_free_sum<double, double>(m, dL, dinv, s)));
  SEM_HIP(launch_reciprocal_mask(dinv, dinv32, m->n_free, s));
  SEM_HIP((launch_local_to_free_avg<double, double>(m, r, rf, s)));
  sem_status st;
  if (fp64) {
    Op<double> o;
    o.G = m->G64.as<double>();
    o.B = m->B64.as<double>();
    o.D = m->D64.as<double>();
    o.k = k;
    o.h2 = h2;
    ChebBufs<double> b;
    b.d = reinterpret_cast<double*>(base + L.d);
    b.rk = reinterpret_cast<double*>(base + L.rk);
    b.wL = dL;
    st = cheb_apply_bufs<double, double>(m, o, dinv, rf, zf, order, lmax, ChebCg(), s, nullptr, 4,
                                         b);
  } else {
    Op<float> o;
    o.G = m->G32.as<float>();
    o.B = m->B32.as<float>();
    o.D = m->D32.as<float>();
    o.h2 = (float)h2;
    o.lp = prec == SEM_BF16_MFMA ? 1 : prec == SEM_FP16_MFMA ? 2 : 0;
    if (k) {
      float* k32 = reinterpret_cast<float*>(base + L.k32);
      SEM_HIP((launch_convert<double, float>(k, k32, m->nL, 1.0, s)));
      o.k = k32;
    }
    ChebBufs<float> b;
    b.d = reinterpret_cast<float*>(base + L.d);
    b.rk = reinterpret_cast<float*>(base + L.rk);
    b.wL = reinterpret_cast<float*>(dL);
    st = cheb_apply_bufs<double, float>(m, o, dinv32, rf, zf, order, lmax, ChebCg(), s, nullptr, 4,
                                        b);
  }
  if (st) return st;
  SEM_HIP((launch_free_to_local<double, double>(m, zf, z, s)));
  return SEM_OK;
}
