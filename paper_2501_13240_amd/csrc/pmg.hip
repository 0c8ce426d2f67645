// p-multigrid V-cycle on the device.
//
// V_l(r):  x = Cheb_l(r)                       pre-smoothing (fourth kind, Jacobi)
//          x += P_l V_{l+1}(P_l^T (r - A_l x))  coarse correction
//          x += Cheb_l(r - A_l x)               post-smoothing
// and a fixed number of Jacobi-PCG iterations on the coarsest level (Sec. 2.2
// names p-multigrid with Chebyshev-accelerated smoothing as the default
// pressure preconditioner).  Vectors are free-unique per level; P_l
// interpolates element blocks (tensor product of the 1-D interpolation J_l)
// and averages the copies of each fine node, P_l^T divides each fine value by
// its number of copies, applies J_l^T per element and sums the copies of each
// coarse node.  Every launch returns at once when the enclosing flexible CG
// has finished, so overshooting iterations cost nothing.
#include <type_traits>

#include "pmg.hpp"

namespace sem {
namespace {

constexpr int kN1 = kMaxOrder + 1;
constexpr int kP3 = kN1 * kN1 * kN1;
constexpr int kInterpThreads = 256;

#define GRID_STRIDE(idx, n)                                                        \
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < (n); \
       idx += (int64_t)gridDim.x * blockDim.x)

// out_L = (M x M x M) in, one element per workgroup; the three contractions
// (along i, then j, then k) go through LDS
template <typename T, int MODE>
__global__ __launch_bounds__(kInterpThreads) void interp_kernel(
    int n_in, int n_out, const T* __restrict__ M, const T* __restrict__ in,
    const int32_t* __restrict__ lmap, const int32_t* __restrict__ seg, T* __restrict__ out,
    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ T sM[kN1 * kN1];
  __shared__ T A[kP3];
  __shared__ T B[kP3];
  const int64_t e = blockIdx.x;
  const int t = threadIdx.x, nt = blockDim.x;
  const int p_in = n_in * n_in * n_in, p_out = n_out * n_out * n_out;
  for (int a = t; a < n_out * n_in; a += nt) sM[a] = M[a];
  for (int q = t; q < p_in; q += nt) {
    const int64_t idx = e * p_in + q;
    T v;
    if constexpr (MODE == 0) {
      v = in[idx];
    } else {
      const int32_t g = lmap[idx];
      v = g >= 0 ? in[g] : T(0);
      if constexpr (MODE == 2) {
        if (g >= 0) v = v / (T)(seg[g + 1] - seg[g]);
      }
    }
    A[q] = v;
  }
  __syncthreads();
  for (int o = t; o < n_in * n_in * n_out; o += nt) {  // along i
    const int a = o % n_out, kj = o / n_out;
    T s = T(0);
    for (int i = 0; i < n_in; ++i) s += sM[a * n_in + i] * A[kj * n_in + i];
    B[o] = s;
  }
  __syncthreads();
  for (int o = t; o < n_in * n_out * n_out; o += nt) {  // along j
    const int a = o % n_out, b = (o / n_out) % n_out, k = o / (n_out * n_out);
    T s = T(0);
    for (int j = 0; j < n_in; ++j) s += sM[b * n_in + j] * B[(k * n_in + j) * n_out + a];
    A[o] = s;
  }
  __syncthreads();
  const int n2 = n_out * n_out;
  for (int o = t; o < p_out; o += nt) {  // along k
    const int ba = o % n2, c = o / n2;
    T s = T(0);
    for (int k = 0; k < n_in; ++k) s += sM[c * n_in + k] * A[k * n2 + ba];
    out[e * p_out + o] = s;
  }
}

// out[g] = sum of the copies of free node g
template <typename T>
__global__ void k_seg_sum(int64_t nf, const int32_t* __restrict__ seg,
                          const int32_t* __restrict__ perm, const T* __restrict__ vL,
                          T* __restrict__ out, const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  GRID_STRIDE(g, nf) out[g] = segment_sum<T>(perm, vL, seg[g], seg[g + 1]);
}

// x[g] += mean of the copies of free node g
template <typename T>
__global__ void k_seg_add_avg(int64_t nf, const int32_t* __restrict__ seg,
                              const int32_t* __restrict__ perm, const T* __restrict__ vL,
                              T* __restrict__ x, const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  GRID_STRIDE(g, nf) {
    const int32_t a = seg[g], b = seg[g + 1];
    x[g] += segment_sum<T>(perm, vL, a, b) / (T)(b - a);
  }
}

// r[g] = b[g] - sum of the copies of free node g
template <typename T>
__global__ void k_seg_sub(int64_t nf, const int32_t* __restrict__ seg,
                          const int32_t* __restrict__ perm, const T* __restrict__ vL,
                          const T* __restrict__ b, T* __restrict__ r,
                          const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  GRID_STRIDE(g, nf) r[g] = b[g] - segment_sum<T>(perm, vL, seg[g], seg[g + 1]);
}

// r[g] -= sum of the copies of free node g (in place)
template <typename T>
__global__ void k_seg_dec(int64_t nf, const int32_t* __restrict__ seg,
                          const int32_t* __restrict__ perm, const T* __restrict__ vL,
                          T* __restrict__ r, const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  GRID_STRIDE(g, nf) r[g] -= segment_sum<T>(perm, vL, seg[g], seg[g + 1]);
}

// The same residuals from the split operator's output (levels of order >= 5
// that carry its routing): w at the single-copy nodes [0, n1) is read from
// wf, contiguous; only the shared nodes [n1, nf) sum their copies, from the
// elements' surface slots.  SUB: r = b - A d; else r -= A d.  Every block
// takes a chunk of each range, so the segmented sums are spread over all.
template <typename T, bool SUB>
__global__ __launch_bounds__(kVecBlock) void k_split_res(
    int64_t n1, int64_t nf, const int32_t* __restrict__ seg, const int32_t* __restrict__ perm,
    const T* __restrict__ wf, const T* __restrict__ wL, const T* __restrict__ b,
    T* __restrict__ r, const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  {
    BLOCK_CHUNK(g, n1) r[g] = (SUB ? b[g] : r[g]) - wf[g];
  }
  {
    BLOCK_CHUNK(i, nf - n1) {
      const int64_t g = n1 + i;
      r[g] = (SUB ? b[g] : r[g]) - segment_sum<T>(perm, wL, seg[g], seg[g + 1]);
    }
  }
}

template <typename T>
__global__ void k_vadd(int64_t n, T* __restrict__ x, const T* __restrict__ y,
                       const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  GRID_STRIDE(g, n) x[g] += y[g];
}

unsigned grid_for(int64_t n) {
  const int64_t b = (n + kVecBlock - 1) / kVecBlock;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 16384));
}

template <typename T>
const T* mat(const DevBuf& b64, const DevBuf& b32) {
  if constexpr (sizeof(T) == 8) return b64.as<double>();
  else return b32.as<float>();
}

template <typename T>
const Op<T>& op_of(const PmgLevel& L) {
  if constexpr (sizeof(T) == 8) return L.op64;
  else return L.op32;
}

template <typename T>
const T* dinv_of(const PmgLevel& L) {
  if constexpr (sizeof(T) == 8) return L.dinv64;
  else return L.dinv32;
}

template <typename T>
T* local_scratch(const sem_mesh* m) {
  SolveWork& W = *m->work;
  return W.vec<T>(sizeof(T) == 8 ? W.wL : W.wL32, m->nL);
}

// The additive Schwarz sum fused with the Chebyshev recurrence: q = sum of
// the box copies of free node g (q = S r_k), then FIRST: d = ca q, z = d;
// else d = ca d + cb q, z += d.  q itself is never stored.
template <typename T, bool FIRST>
__global__ void k_schw_sum_cheb(int64_t nf, const int32_t* __restrict__ seg,
                                const int32_t* __restrict__ perm, const T* __restrict__ box,
                                T* __restrict__ d, T* __restrict__ z, T ca, T cb,
                                const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  GRID_STRIDE(g, nf) {
    const T q = segment_sum<T>(perm, box, seg[g], seg[g + 1]);
    if constexpr (FIRST) {
      const T dg = ca * q;
      d[g] = dg;
      z[g] = dg;
    } else {
      const T dg = ca * d[g] + cb * q;
      d[g] = dg;
      z[g] += dg;
    }
  }
}

template <typename T>
T* box_of(const SchwarzDev& X) {
  if constexpr (sizeof(T) == 8) return X.box64.as<double>();
  else return X.box32.as<float>();
}

// r = b - A d (sub) or r -= A d on one level: the split operator and
// k_split_res where the level carries the split routing (order >= 5: the
// single-copy nodes skip the gather of their copies), else the gather form
// and a segmented sum over all free nodes
template <typename T>
sem_status level_residual(Pmg& P, PmgLevel& L, const Op<T>& op, const T* d, const T* b, T* r,
                          bool sub, const int32_t* skip, hipStream_t s) {
  const sem_mesh* m = L.m;
  SolveWork& W = *m->work;
  const int64_t nf = m->n_free;
  T* wL = local_scratch<T>(m);
  if (!wL) return fail(SEM_ENOMEM, "multigrid work space");
  sem_status st;
  if (op.lp == 0 && ax_split_available(m)) {
    T* wf = P.vec<T>(L, 7);
    if (!wf) return fail(SEM_ENOMEM, "multigrid work space");
    if ((st = apply_op<T>(m, W, op, d, wL, s, false, wf, nullptr))) return st;
    const int32_t* seg = m->fseg.as<int32_t>();
    const int32_t* perm = m->fperm2.as<int32_t>();
    if (sub)
      hipLaunchKernelGGL((k_split_res<T, true>), dim3(grid_for(nf)), dim3(kVecBlock), 0, s,
                         m->n_single, nf, seg, perm, wf, wL, b, r, skip);
    else
      hipLaunchKernelGGL((k_split_res<T, false>), dim3(grid_for(nf)), dim3(kVecBlock), 0, s,
                         m->n_single, nf, seg, perm, wf, wL, b, r, skip);
  } else {
    if ((st = apply_op<T>(m, W, op, d, wL, s, false))) return st;
    const int32_t* seg = m->fseg.as<int32_t>();
    const int32_t* perm = m->fperm.as<int32_t>();
    if (sub)
      hipLaunchKernelGGL((k_seg_sub<T>), dim3(grid_for(nf)), dim3(kVecBlock), 0, s, nf, seg, perm,
                         wL, b, r, skip);
    else
      hipLaunchKernelGGL((k_seg_dec<T>), dim3(grid_for(nf)), dim3(kVecBlock), 0, s, nf, seg, perm,
                         wL, r, skip);
  }
  SEM_CHECK_LAUNCH("level residual");
  return SEM_OK;
}

// z = S r: local fast-diagonalisation solves, then the sum over box copies
template <typename T>
sem_status schwarz_apply(const PmgLevel& L, const T* r, T* z, const int32_t* skip,
                         hipStream_t s) {
  const sem_mesh* m = L.m;
  T* box = box_of<T>(L.sch);
  if (!box) return fail(SEM_EINVAL, "Schwarz factors missing");
  SEM_HIP(launch_fdm<T>(L.sch, m->E, r, box, skip, s));
  hipLaunchKernelGGL((k_seg_sum<T>), dim3(grid_for(m->n_free)), dim3(kVecBlock), 0, s, m->n_free,
                     L.sch.xseg.as<int32_t>(), L.sch.xperm.as<int32_t>(), box, z, skip);
  SEM_CHECK_LAUNCH("Schwarz sum");
  return SEM_OK;
}

// z = p_m(S A) S r with the fourth-kind coefficients (as the Jacobi version).
// Each Schwarz sum carries the recurrence's d and z update (k_schw_sum_cheb),
// and the first residual r_1 = r - A d_0 is formed from r directly.
template <typename T>
sem_status cheb_schwarz(Pmg& P, PmgLevel& L, const T* r, T* z, const CgScalars* outer,
                        hipStream_t s, int* applies) {
  const sem_mesh* m = L.m;
  const int64_t nf = m->n_free;
  const int32_t* skip = outer ? &outer->done : nullptr;
  T* d = P.vec<T>(L, 5);
  T* rk = P.vec<T>(L, 6);
  T* box = box_of<T>(L.sch);
  if (!d || !rk) return fail(SEM_ENOMEM, "multigrid work space");
  if (!box) return fail(SEM_EINVAL, "Schwarz factors missing");
  Op<T> op = op_of<T>(L);
  op.skip = skip;
  const double lmax = L.rho_hat;
  const int32_t* xseg = L.sch.xseg.as<int32_t>();
  const int32_t* xperm = L.sch.xperm.as<int32_t>();
  sem_status st;
  SEM_HIP(launch_fdm<T>(L.sch, m->E, r, box, skip, s));
  hipLaunchKernelGGL((k_schw_sum_cheb<T, true>), dim3(grid_for(nf)), dim3(kVecBlock), 0, s, nf,
                     xseg, xperm, box, d, z, (T)(4.0 / (3.0 * lmax)), T(0), skip);
  for (int k = 1; k < P.smooth_order; ++k) {
    if ((st = level_residual<T>(P, L, op, d, r, rk, k == 1, skip, s))) return st;
    if (applies) ++*applies;
    SEM_HIP(launch_fdm<T>(L.sch, m->E, rk, box, skip, s));
    const double ca = (2.0 * k - 1.0) / (2.0 * k + 3.0);
    const double cb = (8.0 * k + 4.0) / ((2.0 * k + 3.0) * lmax);
    hipLaunchKernelGGL((k_schw_sum_cheb<T, false>), dim3(grid_for(nf)), dim3(kVecBlock), 0, s, nf,
                       xseg, xperm, box, d, z, (T)ca, (T)cb, skip);
  }
  SEM_CHECK_LAUNCH("Chebyshev-Schwarz");
  return SEM_OK;
}

template <typename T>
sem_status smooth(Pmg& P, PmgLevel& L, const T* r, T* z, const CgScalars* outer, hipStream_t s,
                  int* applies) {
  if (P.smoother == 1) return cheb_schwarz<T>(P, L, r, z, outer, s, applies);
  ChebCg c;
  c.skip_sc = outer;
  return cheb_apply_dev<T, T>(L.m, *L.m->work, op_of<T>(L), dinv_of<T>(L), r, z, P.smooth_order,
                              L.rho_hat, c, s, applies);
}

template <typename T>
sem_status vcycle(Pmg& P, int l, const T* r, T* x, const CgScalars* outer, hipStream_t s,
                  int* applies) {
  PmgLevel& L = P.lv[l];
  const sem_mesh* m = L.m;
  SolveWork& W = *m->work;
  const int64_t nf = m->n_free;
  const int32_t* skip = outer ? &outer->done : nullptr;
  const Op<T>& op = op_of<T>(L);
  const T* dinv = dinv_of<T>(L);
  T* t = P.vec<T>(L, 2);
  T* u = P.vec<T>(L, 3);
  T* wL = local_scratch<T>(m);
  if (!t || !u || !wL) return fail(SEM_ENOMEM, "multigrid work space");
  const bool last = (l + 1 == (int)P.lv.size());
  if (last) {
    T* w = P.vec<T>(L, 4);
    if (!w) return fail(SEM_ENOMEM, "multigrid work space");
    return cg_fixed_device<T>(m, W, op, dinv, r, x, t, u, w, wL, P.coarse_iters,
                              m->nullspace && op.h2 == T(0), outer, s);
  }
  Op<T> ops = op;
  ops.skip = skip;
  sem_status st;
  // pre-smoothing
  if ((st = smooth<T>(P, L, r, x, outer, s, applies))) return st;
  // t = r - A x, restricted to the next level
  if ((st = level_residual<T>(P, L, ops, x, r, t, true, skip, s))) return st;
  if (applies) ++*applies;
  PmgLevel& C = P.lv[l + 1];
  const sem_mesh* mc = C.m;
  T* cL = local_scratch<T>(mc);
  T* rc = P.vec<T>(C, 0);
  T* xc = P.vec<T>(C, 1);
  if (!cL || !rc || !xc) return fail(SEM_ENOMEM, "multigrid work space");
  SEM_HIP(launch_interp<T>(m->E, m->n1, mc->n1, mat<T>(L.JT64, L.JT32), 2, t,
                           m->lmap.as<int32_t>(), m->fseg.as<int32_t>(), cL, skip, s));
  hipLaunchKernelGGL((k_seg_sum<T>), dim3(grid_for(mc->n_free)), dim3(kVecBlock), 0, s,
                     mc->n_free, mc->fseg.as<int32_t>(), mc->fperm.as<int32_t>(), cL, rc, skip);
  SEM_CHECK_LAUNCH("restriction");
  if ((st = vcycle<T>(P, l + 1, rc, xc, outer, s, nullptr))) return st;
  // x += P x_c
  SEM_HIP(launch_interp<T>(m->E, mc->n1, m->n1, mat<T>(L.J64, L.J32), 1, xc,
                           mc->lmap.as<int32_t>(), nullptr, wL, skip, s));
  hipLaunchKernelGGL((k_seg_add_avg<T>), dim3(grid_for(nf)), dim3(kVecBlock), 0, s, nf,
                     m->fseg.as<int32_t>(), m->fperm.as<int32_t>(), wL, x, skip);
  SEM_CHECK_LAUNCH("prolongation");
  // post-smoothing on t = r - A x
  if ((st = level_residual<T>(P, L, ops, x, r, t, true, skip, s))) return st;
  if (applies) ++*applies;
  if ((st = smooth<T>(P, L, t, u, outer, s, applies))) return st;
  hipLaunchKernelGGL((k_vadd<T>), dim3(grid_for(nf)), dim3(kVecBlock), 0, s, nf, x, u, skip);
  SEM_CHECK_LAUNCH("post-smoothing");
  return SEM_OK;
}

}  // namespace

template <typename T>
T* Pmg::vec(PmgLevel& L, int which) {
  DevBuf* b64[8] = {&L.r64, &L.x64, &L.t64, &L.u64, &L.w64, &L.d64, &L.k64v, &L.q64};
  DevBuf* b32[8] = {&L.r32, &L.x32, &L.t32, &L.u32, &L.w32, &L.d32, &L.k32v, &L.q32};
  DevBuf& b = sizeof(T) == 8 ? *b64[which] : *b32[which];
  if (b.ensure((size_t)std::max<int64_t>(L.m->n_free, 1) * sizeof(T)) != SEM_OK) return nullptr;
  return b.as<T>();
}
template double* Pmg::vec<double>(PmgLevel&, int);
template float* Pmg::vec<float>(PmgLevel&, int);

void pmg_destroy(Pmg* p) {
  if (!p) return;
  for (auto& L : p->lv)
    if (L.owned && L.m) sem_free_mesh(L.m);
  delete p;
}

template <typename T>
hipError_t launch_interp(int64_t E, int n_in, int n_out, const T* M, int mode, const T* in,
                         const int32_t* lmap, const int32_t* seg, T* out_L, const int32_t* skip,
                         hipStream_t s) {
  if (n_in < 1 || n_in > kN1 || n_out < 1 || n_out > kN1 || E < 1) return hipErrorInvalidValue;
  const dim3 g((unsigned)E), b(kInterpThreads);
  if (mode == 0)
    hipLaunchKernelGGL((interp_kernel<T, 0>), g, b, 0, s, n_in, n_out, M, in, lmap, seg, out_L,
                       skip);
  else if (mode == 1)
    hipLaunchKernelGGL((interp_kernel<T, 1>), g, b, 0, s, n_in, n_out, M, in, lmap, seg, out_L,
                       skip);
  else
    hipLaunchKernelGGL((interp_kernel<T, 2>), g, b, 0, s, n_in, n_out, M, in, lmap, seg, out_L,
                       skip);
  return hipGetLastError();
}
template hipError_t launch_interp<double>(int64_t, int, int, const double*, int, const double*,
                                          const int32_t*, const int32_t*, double*,
                                          const int32_t*, hipStream_t);
template hipError_t launch_interp<float>(int64_t, int, int, const float*, int, const float*,
                                         const int32_t*, const int32_t*, float*, const int32_t*,
                                         hipStream_t);

template <typename Tr, typename Tp>
sem_status pmg_precond(const sem_mesh* m, SolveWork& W, const Tr* r, Tr* z, const ChebCg& cg,
                       hipStream_t s, int* applies) {
  (void)W;
  if (!m->pmg || m->pmg->lv.empty() || m->pmg->lv[0].m != m)
    return fail(SEM_EINVAL, "no multigrid hierarchy for this mesh");
  Pmg& P = *m->pmg;
  PmgLevel& L0 = P.lv[0];
  const int64_t nf = m->n_free;
  sem_status st;
  if (cg.sc && (st = launch_cg_gate(cg.check_in, cg.nblk, cg.sc, cg.hist, s))) return st;
  const Tp* r0;
  if constexpr (std::is_same<Tr, Tp>::value) {
    r0 = r;
  } else {
    Tp* rr = P.vec<Tp>(L0, 0);
    if (!rr) return fail(SEM_ENOMEM, "multigrid work space");
    if ((st = launch_convert_skip<Tr, Tp>(nf, r, rr, cg.sc, s))) return st;
    r0 = rr;
  }
  Tp* x0 = P.vec<Tp>(L0, 1);
  if (!x0) return fail(SEM_ENOMEM, "multigrid work space");
  if ((st = vcycle<Tp>(P, 0, r0, x0, cg.sc, s, applies))) return st;
  return launch_flex_dots<Tr, Tp>(nf, x0, z, r, static_cast<const Tr*>(cg.w), cg.part_out, cg.sc,
                                  s);
}
template sem_status pmg_precond<double, double>(const sem_mesh*, SolveWork&, const double*,
                                                double*, const ChebCg&, hipStream_t, int*);
template sem_status pmg_precond<double, float>(const sem_mesh*, SolveWork&, const double*,
                                               double*, const ChebCg&, hipStream_t, int*);
template sem_status pmg_precond<float, float>(const sem_mesh*, SolveWork&, const float*, float*,
                                              const ChebCg&, hipStream_t, int*);

sem_status schwarz_precond(Pmg& P, int level, const double* r, double* z, const ChebCg& cg,
                           hipStream_t s) {
  PmgLevel& L = P.lv[level];
  const int64_t nf = L.m->n_free;
  sem_status st;
  if (cg.sc && (st = launch_cg_gate(cg.check_in, cg.nblk, cg.sc, cg.hist, s))) return st;
  double* q = P.vec<double>(L, 7);
  if (!q) return fail(SEM_ENOMEM, "multigrid work space");
  if ((st = schwarz_apply<double>(L, r, q, cg.sc ? &cg.sc->done : nullptr, s))) return st;
  return launch_flex_dots<double, double>(nf, q, z, r, static_cast<const double*>(cg.w),
                                          cg.part_out, cg.sc, s);
}

}  // namespace sem
