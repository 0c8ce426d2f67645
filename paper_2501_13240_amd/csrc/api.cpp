// The C entry points of libsem (declared and documented in include/sem.h).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "advection.hpp"
#include "common.hpp"
#include "pmg.hpp"
#include "solver.hpp"

namespace sem {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

sem_status fail(sem_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

sem_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? SEM_ENOMEM : SEM_EDEVICE;
}

sem_status DevBuf::ensure(size_t nbytes) {
  if (nbytes <= bytes && p) return SEM_OK;
  release();
  hipError_t e = hipMalloc(&p, nbytes);
  if (e != hipSuccess) {
    p = nullptr;
    return hip_fail(e, "hipMalloc");
  }
  bytes = nbytes;
  return SEM_OK;
}

template <typename T>
static sem_status upload(DevBuf& d, const std::vector<T>& h, hipStream_t s) {
  sem_status st = d.ensure(std::max<size_t>(h.size(), 1) * sizeof(T));
  if (st) return st;
  if (!h.empty()) SEM_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return SEM_OK;
}

// --------------------------------------------------------- shared pieces

static SolveWork& work_of(const sem_mesh* m) {
  sem_mesh* mm = const_cast<sem_mesh*>(m);
  if (!mm->work) mm->work = new SolveWork();
  return *mm->work;
}

// inverse of the assembled diagonal on the free nodes (FP64 + FP32 copy)
static sem_status prepare_dinv(const sem_mesh* m, SolveWork& W, const double* k, double h2,
                               hipStream_t s) {
  double* dinv = W.vec<double>(W.dinv, m->n_free);
  float* dinv32 = W.vec<float>(W.dinv32, m->n_free);
  double* dL = W.vec<double>(W.wL, m->nL);
  if (!dinv || !dinv32 || !dL) return fail(SEM_ENOMEM, "work space");
  sem_mesh* mm = const_cast<sem_mesh*>(m);
  if (!k && mm->dinv_valid && mm->cached_h2 == h2) return SEM_OK;
  SEM_HIP(launch_local_diag(m, k, h2, dL, s));
  SEM_HIP((launch_free_sum<double, double>(m, dL, dinv, s)));
  SEM_HIP(launch_reciprocal_mask(dinv, dinv32, m->n_free, s));
  mm->dinv_valid = (k == nullptr);
  mm->cached_h2 = h2;
  return SEM_OK;
}

static Op<double> op64_of(const sem_mesh* m, const double* k, double h2) {
  Op<double> o;
  o.G = m->G64.as<double>();
  o.B = m->B64.as<double>();
  o.D = m->D64.as<double>();
  o.k = k;
  o.h2 = h2;
  return o;
}

static sem_status op32_of(const sem_mesh* m, SolveWork& W, const double* k, double h2,
                          hipStream_t s, Op<float>& o) {
  o.G = m->G32.as<float>();
  o.B = m->B32.as<float>();
  o.D = m->D32.as<float>();
  o.h2 = (float)h2;
  o.k = nullptr;
  if (k) {
    float* k32 = W.vec<float>(W.k32, m->nL);
    if (!k32) return fail(SEM_ENOMEM, "work space");
    SEM_HIP((launch_convert<double, float>(k, k32, m->nL, 1.0, s)));
    o.k = k32;
  }
  return SEM_OK;
}

// largest eigenvalue of a symmetric tridiagonal matrix by Sturm-sequence bisection
static double tridiag_lmax(const std::vector<double>& a, const std::vector<double>& b) {
  const int n = (int)a.size();
  if (n == 0) return 0.0;
  double lo = a[0], hi = a[0];
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto count_below = [&](double x) {
    int c = 0;
    double q = 1.0;
    for (int i = 0; i < n; ++i) {
      q = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / q : 0.0);
      if (q == 0.0) q = -1e-300;
      if (q < 0.0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(hi), 1.0); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) == n) hi = mid;
    else lo = mid;
  }
  return hi;
}

static sem_status estimate_lmax(const sem_mesh* m, SolveWork& W, const double* k, double h2,
                                int steps, double* out, hipStream_t s) {
  sem_mesh* mm = const_cast<sem_mesh*>(m);
  if (!k && mm->cached_lmax > 0.0 && mm->cached_lmax_h2 == h2 && steps == 20) {
    *out = mm->cached_lmax;
    return SEM_OK;
  }
  sem_status st = W.init(m, std::max(steps, 1));
  if (st) return st;
  if ((st = prepare_dinv(m, W, k, h2, s))) return st;
  const bool neumann = m->nullspace && h2 == 0.0;
  double* b = W.vec<double>(W.tmpf, m->n_free);
  CgArgs<double, double> a;
  a.op = op64_of(m, k, h2);
  a.b = b;
  a.x = W.vec<double>(W.x, m->n_free);
  a.r = W.vec<double>(W.r, m->n_free);
  a.p = W.vec<double>(W.p, m->n_free);
  a.w = W.vec<double>(W.w, m->n_free);
  a.z = W.vec<double>(W.z, m->n_free);
  a.wL = W.vec<double>(W.wL, m->nL);
  a.dinv = W.dinv.as<double>();
  if (!b || !a.x || !a.r || !a.p || !a.w || !a.z || !a.wL) return fail(SEM_ENOMEM, "work space");
  SEM_HIP(launch_pseudo_random(b, m->n_free, 0x5eed5eedull, s));
  if (neumann && (st = free_remove_mean_f64(m, W, b, s))) return st;
  a.precond = SEM_PRECOND_JACOBI;
  a.rtol = 0.0;
  a.max_it = steps;
  a.fixed = true;
  a.x_zero = true;
  a.neumann = neumann;
  std::vector<double> al, be;
  a.alpha_out = &al;
  a.beta_out = &be;
  CgResult res;
  if ((st = cg_solve<double, double>(m, W, a, res, s))) return st;
  // CG-Lanczos tridiagonal: T_jj = 1/a_j + b_{j-1}/a_{j-1}, T_{j,j+1} = sqrt(b_j)/a_j
  int n = (int)al.size();
  for (int j = 0; j < n; ++j)
    if (!(al[j] > 0.0) || !std::isfinite(al[j])) {
      n = j;
      break;
    }
  if (n == 0) return fail(SEM_EBREAKDOWN, "eigenvalue estimate: CG produced no coefficient");
  std::vector<double> diag(n), off(std::max(n - 1, 0));
  for (int j = 0; j < n; ++j) {
    diag[j] = 1.0 / al[j] + (j > 0 ? be[j - 1] / al[j - 1] : 0.0);
    if (j + 1 < n) off[j] = std::sqrt(std::max(be[j], 0.0)) / al[j];
  }
  *out = tridiag_lmax(diag, off);
  if (!k && steps == 20) {
    mm->cached_lmax = *out;
    mm->cached_lmax_h2 = h2;
  }
  return SEM_OK;
}

// Level operators, Jacobi inverses and Chebyshev bounds of the multigrid
// hierarchy for one solve (k interpolated to every level), and the cycle's
// work space in the precision it runs in, allocated here so that no
// allocation happens inside the iterations (which may be graph-captured).
// Must run before the caller places its own vectors in the fine work space:
// the bound estimate uses it.
static sem_status estimate_lmax_schwarz(Pmg& P, int l, const double* k, double h2, double* out,
                                        hipStream_t s);

static sem_status pmg_prepare(const sem_mesh* m, const double* k, double h2, bool f64,
                              hipStream_t s) {
  Pmg& P = *m->pmg;
  sem_status st;
  for (size_t l = 0; l < P.lv.size(); ++l) {
    PmgLevel& L = P.lv[l];
    const sem_mesh* ml = L.m;
    SolveWork& Wl = work_of(ml);
    if ((st = Wl.init(ml, 20))) return st;
    const double* kl = nullptr;
    if (k && l == 0) {
      kl = k;
    } else if (k) {
      if ((st = L.k64.ensure((size_t)ml->nL * sizeof(double)))) return st;
      SEM_HIP(launch_interp<double>(m->E, m->n1, ml->n1, L.Ik64.as<double>(), 0, k, nullptr,
                                    nullptr, L.k64.as<double>(), nullptr, s));
      kl = L.k64.as<double>();
    }
    if ((st = prepare_dinv(ml, Wl, kl, h2, s))) return st;
    double est = 0.0;
    const bool schwarz = P.smoother == SEM_SMOOTH_SCHWARZ && l + 1 < P.lv.size();
    if (schwarz) {
      if ((st = estimate_lmax_schwarz(P, (int)l, kl, h2, &est, s))) return st;
    } else if ((st = estimate_lmax(ml, Wl, kl, h2, 20, &est, s))) {
      return st;
    }
    L.rho_hat = 1.1 * est;
    L.op64 = op64_of(ml, kl, h2);
    if ((st = op32_of(ml, Wl, kl, h2, s, L.op32))) return st;
    L.dinv64 = Wl.dinv.as<double>();
    L.dinv32 = Wl.dinv32.as<float>();
    bool ok = true;
    for (int v = 0; v < 8; ++v) ok = ok && (f64 ? P.vec<double>(L, v) != nullptr : P.vec<float>(L, v) != nullptr);
    if (f64)
      ok = ok && Wl.vec<double>(Wl.wL, ml->nL) && Wl.vec<double>(Wl.cd, ml->n_free) &&
           Wl.vec<double>(Wl.crk, ml->n_free);
    else
      ok = ok && Wl.vec<float>(Wl.wL32, ml->nL) && Wl.vec<float>(Wl.cd32, ml->n_free) &&
           Wl.vec<float>(Wl.crk32, ml->n_free);
    if (!ok) return fail(SEM_ENOMEM, "multigrid work space");
  }
  SEM_HIP(hipStreamSynchronize(s));
  return SEM_OK;
}

// Schwarz factors of one level on the device (from its host description)
static sem_status setup_schwarz(PmgLevel& L, int N, int64_t E, const int64_t* gid,
                                const uint8_t* dir, const double* xyz, hipStream_t s) {
  HostNumbering hn;
  sem_status st = build_numbering(N, E, gid, dir, hn);
  if (st) return st;
  SchwarzHost H;
  if ((st = build_schwarz(N, E, gid, dir, xyz, hn.lmap.data(), hn.n_free, H))) return st;
  SchwarzDev& X = L.sch;
  X.nx = N + 3;
  std::vector<float> S32(H.S.begin(), H.S.end()), L32(H.lam.begin(), H.lam.end());
  if ((st = upload(X.xmap, H.xmap, s)) || (st = upload(X.xseg, H.xseg, s)) ||
      (st = upload(X.xperm, H.xperm, s)) || (st = upload(X.S64, H.S, s)) ||
      (st = upload(X.S32, S32, s)) || (st = upload(X.L64, H.lam, s)) ||
      (st = upload(X.L32, L32, s)))
    return st;
  const size_t nbox = H.xmap.size();
  if ((st = X.box64.ensure(nbox * sizeof(double))) || (st = X.box32.ensure(nbox * sizeof(float))))
    return st;
  SEM_HIP(hipStreamSynchronize(s));  // host vectors go out of scope
  return SEM_OK;
}

// largest eigenvalue of (Schwarz) A on a level from 20 CG-Lanczos steps with
// the Schwarz smoother as preconditioner (cached per level for k == NULL)
static sem_status estimate_lmax_schwarz(Pmg& P, int l, const double* k, double h2, double* out,
                                        hipStream_t s) {
  PmgLevel& L = P.lv[l];
  const sem_mesh* ml = L.m;
  if (!k && L.sch_rho > 0.0 && L.sch_rho_h2 == h2) {
    *out = L.sch_rho;
    return SEM_OK;
  }
  SolveWork& W = work_of(ml);
  sem_status st = W.init(ml, 20);
  if (st) return st;
  if ((st = prepare_dinv(ml, W, k, h2, s))) return st;
  const bool neumann = ml->nullspace && h2 == 0.0;
  const int64_t nf = ml->n_free;
  double* b = W.vec<double>(W.tmpf, nf);
  CgArgs<double, double> a;
  a.op = op64_of(ml, k, h2);
  a.b = b;
  a.x = W.vec<double>(W.x, nf);
  a.r = W.vec<double>(W.r, nf);
  a.p = W.vec<double>(W.p, nf);
  a.w = W.vec<double>(W.w, nf);
  a.z = W.vec<double>(W.z, nf);
  a.wL = W.vec<double>(W.wL, ml->nL);
  a.dinv = W.dinv.as<double>();
  if (!b || !a.x || !a.r || !a.p || !a.w || !a.z || !a.wL || !P.vec<double>(L, 7))
    return fail(SEM_ENOMEM, "work space");
  SEM_HIP(launch_pseudo_random(b, nf, 0x5eed5eedull, s));
  if (neumann && (st = free_remove_mean_f64(ml, W, b, s))) return st;
  a.precond = SEM_PRECOND_CHEBYSHEV;  // the flexible path, preconditioned by:
  Pmg* pp = &P;
  a.cheb = [pp, l](const sem_mesh*, SolveWork&, const double* r, double* z, const ChebCg& cg,
                   hipStream_t ss, int*) { return schwarz_precond(*pp, l, r, z, cg, ss); };
  a.rtol = 0.0;
  a.max_it = 20;
  a.fixed = true;
  a.x_zero = true;
  a.neumann = neumann;
  std::vector<double> al, be;
  a.alpha_out = &al;
  a.beta_out = &be;
  CgResult res;
  if ((st = cg_solve<double, double>(ml, W, a, res, s))) return st;
  int n = (int)al.size();
  for (int j = 0; j < n; ++j)
    if (!(al[j] > 0.0) || !std::isfinite(al[j])) {
      n = j;
      break;
    }
  if (n == 0) return fail(SEM_EBREAKDOWN, "Schwarz bound: CG produced no coefficient");
  std::vector<double> diag(n), off(std::max(n - 1, 0));
  for (int j = 0; j < n; ++j) {
    diag[j] = 1.0 / al[j] + (j > 0 ? be[j - 1] / al[j - 1] : 0.0);
    if (j + 1 < n) off[j] = std::sqrt(std::max(be[j], 0.0)) / al[j];
  }
  *out = tridiag_lmax(diag, off);
  if (!k) {
    L.sch_rho = *out;
    L.sch_rho_h2 = h2;
  }
  return SEM_OK;
}

// iterations per chunk of a multigrid-preconditioned solve (one iteration is
// a few hundred launches)
constexpr int kPmgMaxChunk = 2;

static bool prec_ok(sem_prec p) {
  return p == SEM_FP64 || p == SEM_FP32 || p == SEM_BF16_MFMA || p == SEM_FP16_MFMA;
}
// 16-bit contraction mode of an FP32-data precision
static int lp_of(sem_prec p) { return p == SEM_BF16_MFMA ? 1 : p == SEM_FP16_MFMA ? 2 : 0; }

static sem_status check_mesh(const sem_mesh* m) {
  if (!m) return fail(SEM_EINVAL, "mesh is NULL");
  return SEM_OK;
}

// The options of a solve, validated (defaults when opts_in is NULL).
static sem_status solve_options(const sem_mesh* m, const sem_solve_opts* opts_in,
                                sem_solve_opts& opts) {
  if (opts_in) opts = *opts_in;
  else sem_solve_opts_default(&opts);
  if (opts.mode != SEM_SOLVE_CG && opts.mode != SEM_SOLVE_MIXED_IR)
    return fail(SEM_EINVAL, "unknown solve mode");
  if (opts.precond != SEM_PRECOND_JACOBI && opts.precond != SEM_PRECOND_CHEBYSHEV &&
      opts.precond != SEM_PRECOND_PMG && opts.precond != SEM_PRECOND_CHEBYSHEV_FIRST)
    return fail(SEM_EINVAL, "unknown preconditioner");
  const bool pmg = opts.precond == SEM_PRECOND_PMG;
  if (pmg && !m->pmg) return fail(SEM_EINVAL, "multigrid preconditioner: call sem_setup_pmg first");
  if (pmg && opts.precond_prec != SEM_FP32 &&
      !(opts.precond_prec == SEM_FP64 && opts.mode == SEM_SOLVE_CG))
    return fail(SEM_EINVAL, "the multigrid cycle runs in SEM_FP32 (or SEM_FP64 in mode CG)");
  if (opts.cheb_order < 1) return fail(SEM_EINVAL, "cheb_order must be >= 1");
  if (opts.max_iter < 0) return fail(SEM_EINVAL, "max_iter must be >= 0");
  if (!(opts.rtol >= 0.0)) return fail(SEM_EINVAL, "rtol must be >= 0");
  if (opts.mode == SEM_SOLVE_MIXED_IR && opts.fixed_iters)
    return fail(SEM_EINVAL, "fixed_iters is only available in mode CG");
  if (opts.mode == SEM_SOLVE_MIXED_IR && !(opts.inner_rtol > 0.0 && opts.inner_rtol < 1.0))
    return fail(SEM_EINVAL, "inner_rtol must be in (0, 1)");
  const bool cheb_any =
      opts.precond == SEM_PRECOND_CHEBYSHEV || opts.precond == SEM_PRECOND_CHEBYSHEV_FIRST;
  if (cheb_any && !prec_ok((sem_prec)opts.precond_prec))
    return fail(SEM_EINVAL, "unknown Chebyshev precision");
  if (opts.mode == SEM_SOLVE_MIXED_IR && cheb_any && opts.precond_prec == SEM_FP64)
    return fail(SEM_EINVAL, "the inner solve of MIXED_IR runs in FP32 data");

  return SEM_OK;
}

// How a solve takes its right-hand side and start on the free nodes
// (`load`: fills bf and xf, tells whether x0 = 0) and what it does with the
// solution there (`store`).  Both enqueue on the solve's stream.
using SolveLoad = std::function<sem_status(double* bf, double* xf, bool* x_zero)>;
using SolveStore = std::function<sem_status(const double* xf)>;

// Everything of a solve between the free-node right-hand side and the
// free-node solution: preconditioner set-up, the CG or the refinement loop,
// the null-space projection, the timing and the statistics.
static sem_status solve_free(const sem_mesh* m, const double* k, double h2,
                             const sem_solve_opts& opts, const SolveLoad& load,
                             const SolveStore& store, sem_solve_stats* stats, hipStream_t s) {
  SolveWork& W = work_of(m);
  const bool pmg = opts.precond == SEM_PRECOND_PMG;
  sem_status st = W.init(m, std::max(opts.max_iter, 1));
  if (st) return st;
  W.ev_used = 0;
  if (m->n_free == 0) {
    // no unknowns (every node Dirichlet): the solution is empty, so the
    // output holds 0 at every copy; no preconditioner is set up
    double* xf = W.vec<double>(W.x, 1);
    if (!xf) return fail(SEM_ENOMEM, "work space");
    if ((st = store(xf))) return st;
    SEM_HIP(hipStreamSynchronize(s));
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->converged = 1;
    }
    return SEM_OK;
  }
  hipEvent_t t0, t1;
  SEM_HIP(hipEventCreate(&t0));
  SEM_HIP(hipEventCreate(&t1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } guard{t0, t1};

  const bool neumann = m->nullspace && h2 == 0.0;
  const bool cheb =
      opts.precond == SEM_PRECOND_CHEBYSHEV || opts.precond == SEM_PRECOND_CHEBYSHEV_FIRST;
  const int kind = opts.precond == SEM_PRECOND_CHEBYSHEV_FIRST ? 1 : 4;
  const bool pmg64 = pmg && opts.precond_prec == SEM_FP64;
  if (pmg && (st = pmg_prepare(m, k, h2, pmg64, s))) return st;
  double lmax = pmg ? m->pmg->lv[0].rho_hat : opts.lmax;
  if (cheb && !(lmax > 0.0)) {
    double est = 0.0;
    if ((st = estimate_lmax(m, W, k, h2, 20, &est, s))) return st;
    lmax = 1.1 * est;
  }
  SEM_HIP(hipEventRecord(t0, s));
  if ((st = prepare_dinv(m, W, k, h2, s))) return st;
  const int64_t nf = m->n_free;
  double* bf = W.vec<double>(W.bf, nf);
  double* xf = W.vec<double>(W.x, nf);
  if (!bf || !xf) return fail(SEM_ENOMEM, "work space");
  bool x_zero = false;
  if ((st = load(bf, xf, &x_zero))) return st;
  if (neumann && (st = free_remove_mean_f64(m, W, bf, s))) return st;

  const Op<double> op64 = op64_of(m, k, h2);
  Op<float> op32;
  if ((st = op32_of(m, W, k, h2, s, op32))) return st;
  Op<float> opc = op32;  // the Chebyshev preconditioner's FP32-data operator
  opc.lp = lp_of((sem_prec)opts.precond_prec);
  const double* dinv = W.dinv.as<double>();
  const float* dinv32 = W.dinv32.as<float>();

  int iters = 0, outer = 0, applies = 0;
  bool converged = false;
  int fail_status = 0;
  double rel = 0.0;

  if (opts.mode == SEM_SOLVE_CG) {
    // A Chebyshev preconditioner of order >= 2 with FP64 or FP32 contractions
    // runs inside the CG's own kernels when the split operator is available
    // (the CG then carries the preconditioner's precision as Tp); z_0 = M r_0
    // still comes from the stand-alone pass.
    const bool fuse = cheb && opts.cheb_order >= 2 && ax_split_available(m) &&
                      (opts.precond_prec == SEM_FP64 || opts.precond_prec == SEM_FP32);
    auto run = [&](auto& a) -> sem_status {
      a.op = op64;
      a.b = bf;
      a.x = xf;
      a.r = W.vec<double>(W.r, nf);
      a.p = W.vec<double>(W.p, nf);
      a.w = W.vec<double>(W.w, nf);
      a.z = W.vec<double>(W.z, nf);
      a.wL = W.vec<double>(W.wL, m->nL);
      if (!a.r || !a.p || !a.w || !a.z || !a.wL) return fail(SEM_ENOMEM, "work space");
      a.dinv = dinv;
      a.precond = opts.precond;
      a.cheb_order = opts.cheb_order;
      if (pmg) {
        if (pmg64)
          a.cheb = [](const sem_mesh* mm, SolveWork& WW, const double* r, double* z,
                      const ChebCg& cg, hipStream_t ss, int* ap) {
            return pmg_precond<double, double>(mm, WW, r, z, cg, ss, ap);
          };
        else
          a.cheb = [](const sem_mesh* mm, SolveWork& WW, const double* r, double* z,
                      const ChebCg& cg, hipStream_t ss, int* ap) {
            return pmg_precond<double, float>(mm, WW, r, z, cg, ss, ap);
          };
      } else if (cheb) {
        const int order = opts.cheb_order;
        if (opts.precond_prec == SEM_FP64) {
          a.cheb = [op64, dinv, order, lmax, kind](const sem_mesh* mm, SolveWork& WW,
                                                   const double* r, double* z, const ChebCg& cg,
                                                   hipStream_t ss, int* ap) {
            return cheb_apply_dev<double, double>(mm, WW, op64, dinv, r, z, order, lmax, cg, ss,
                                                  ap, kind);
          };
        } else {
          a.cheb = [opc, dinv32, order, lmax, kind](const sem_mesh* mm, SolveWork& WW,
                                                    const double* r, double* z, const ChebCg& cg,
                                                    hipStream_t ss, int* ap) {
            return cheb_apply_dev<double, float>(mm, WW, opc, dinv32, r, z, order, lmax, cg, ss,
                                                 ap, kind);
          };
        }
      }
      a.rtol = opts.rtol;
      a.max_it = opts.max_iter;
      a.fixed = opts.fixed_iters != 0;
      a.x_zero = x_zero;
      a.neumann = neumann;
      a.profile = opts.profile != 0;
      a.check_every = opts.check_every;
      if (pmg) a.max_chunk = kPmgMaxChunk;
      a.hist = opts.residual_history;
      CgResult res;
      sem_status sst = cg_solve(m, W, a, res, s);
      if (sst) return sst;
      iters = res.iters;
      applies = res.applies;
      converged = res.converged;
      fail_status = res.status;
      rel = res.bnorm > 0.0 ? res.rnorm / res.bnorm : 0.0;
      return SEM_OK;
    };
    if (fuse && opts.precond_prec == SEM_FP32) {
      CgArgs<double, float> a;
      a.fuse.on = true;
      a.fuse.op = opc;
      a.fuse.dinv = dinv32;
      a.fuse.order = opts.cheb_order;
      a.fuse.lmax = lmax;
      a.fuse.kind = kind;
      if ((st = run(a))) return st;
    } else {
      CgArgs<double, double> a;
      if (fuse) {
        a.fuse.on = true;
        a.fuse.op = op64;
        a.fuse.dinv = dinv;
        a.fuse.order = opts.cheb_order;
        a.fuse.lmax = lmax;
        a.fuse.kind = kind;
      }
      if ((st = run(a))) return st;
    }
  } else {
    // FP64 iterative refinement around an FP32 inner CG
    double* r = W.vec<double>(W.r, nf);
    float* b32 = W.vec<float>(W.r32, nf);
    CgArgs<float, float> a;
    a.op = op32;
    a.b = b32;
    a.x = W.vec<float>(W.x32, nf);
    a.r = W.vec<float>(W.ri32, nf);
    a.p = W.vec<float>(W.p32, nf);
    a.w = W.vec<float>(W.w32, nf);
    a.z = W.vec<float>(W.z32, nf);
    a.wL = W.vec<float>(W.wL32, m->nL);
    if (!r || !b32 || !a.x || !a.r || !a.p || !a.w || !a.z || !a.wL)
      return fail(SEM_ENOMEM, "work space");
    a.dinv = dinv32;
    a.precond = opts.precond;
    a.cheb_order = opts.cheb_order;
    if (pmg) {
      a.cheb = [](const sem_mesh* mm, SolveWork& WW, const float* rr, float* z, const ChebCg& cg,
                  hipStream_t ss, int* ap) {
        return pmg_precond<float, float>(mm, WW, rr, z, cg, ss, ap);
      };
    } else if (cheb) {
      const int order = opts.cheb_order;
      a.cheb = [opc, dinv32, order, lmax, kind](const sem_mesh* mm, SolveWork& WW, const float* rr,
                                          float* z, const ChebCg& cg, hipStream_t ss, int* ap) {
        return cheb_apply_dev<float, float>(mm, WW, opc, dinv32, rr, z, order, lmax, cg, ss, ap,
                                            kind);
      };
      if (order >= 2 && opc.lp == 0 && ax_split_available(m)) {
        a.fuse.on = true;
        a.fuse.op = opc;
        a.fuse.dinv = dinv32;
        a.fuse.order = order;
        a.fuse.lmax = lmax;
        a.fuse.kind = kind;
      }
    }
    a.neumann = neumann;
    a.x_zero = true;
    a.fixed = false;
    a.rtol = opts.inner_rtol;
    a.check_every = opts.check_every;
    if (pmg) a.max_chunk = kPmgMaxChunk;
    double bd[3];
    if ((st = free_dots_f64(m, W, bf, nullptr, bd, s))) return st;
    const double bnorm = std::sqrt(bd[0]);
    double rr_sum[2];
    if (x_zero) {
      SEM_HIP((launch_convert<double, double>(bf, r, nf, 1.0, s)));
      rr_sum[0] = bd[0];
      rr_sum[1] = bd[2];
    } else {
      if ((st = ir_residual(m, W, op64, xf, bf, r, rr_sum, s, opts.profile != 0))) return st;
      ++applies;
    }
    if (bnorm == 0.0) {
      SEM_HIP(launch_fill<double>(xf, nf, 0.0, s));
      converged = true;
    }
    while (!converged) {
      const double rnorm = std::sqrt(rr_sum[0]);
      rel = rnorm / bnorm;
      if (!std::isfinite(rel)) {
        fail_status = 3;
        break;
      }
      if (rel <= opts.rtol) {
        converged = true;
        break;
      }
      if (outer >= opts.max_outer || iters >= opts.max_iter) break;
      const double shift = neumann ? rr_sum[1] / (double)nf : 0.0;
      if ((st = ir_prepare(m, r, b32, shift, 1.0 / rnorm, s))) return st;
      a.max_it = std::max(1, opts.max_iter - iters);
      // inner reduction: inner_rtol, or only what is still missing to reach rtol
      // (with a 0.3 safety factor), so the last refinement step is short
      a.rtol = std::min(0.5, std::max(opts.inner_rtol, 0.3 * opts.rtol / rel));
      CgResult res;
      if ((st = cg_solve<float, float>(m, W, a, res, s))) return st;
      iters += res.iters;
      applies += res.applies;
      if (res.status == 2 || res.status == 3) {
        fail_status = res.status;
        break;
      }
      if ((st = ir_update(m, xf, a.x, rnorm, s))) return st;
      if ((st = ir_residual(m, W, op64, xf, bf, r, rr_sum, s, opts.profile != 0))) return st;
      ++applies;
      ++outer;
    }
  }
  if (neumann && (st = free_remove_mean_f64(m, W, xf, s))) return st;
  if ((st = store(xf))) return st;
  SEM_HIP(hipEventRecord(t1, s));
  SEM_HIP(hipEventSynchronize(t1));
  float ms = 0.f;
  SEM_HIP(hipEventElapsedTime(&ms, t0, t1));
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->iters = iters;
    stats->outer_iters = outer;
    stats->operator_applies = applies;
    stats->converged = converged ? 1 : 0;
    stats->rel_res = rel;
    stats->time_ms = ms;
    stats->lmax = (cheb || pmg) ? lmax : 0.0;
    double ax_ms = 0.0;
    for (int i = 0; i + 1 < W.ev_used; i += 2) {
      float d = 0.f;
      if (hipEventElapsedTime(&d, W.ev[i], W.ev[i + 1]) == hipSuccess) ax_ms += d;
    }
    stats->ax_ms = ax_ms;
    stats->ax_launches = W.ev_used / 2;
  }
  if (fail_status == 2 || fail_status == 3)
    return fail(SEM_EBREAKDOWN, fail_status == 2 ? "CG breakdown: p.Ap <= 0"
                                                 : "CG produced a non-finite value");
  if (!converged && !opts.fixed_iters)
    return fail(SEM_ENOCONV, "iteration limit reached before the tolerance");
  return SEM_OK;
}


}  // namespace sem

sem_mesh::~sem_mesh() {
  pmg_destroy(pmg);
  delete work;
  delete adv[0];
  delete adv[1];
}

using namespace sem;

extern "C" {

void sem_solve_opts_default(sem_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->mode = SEM_SOLVE_CG;
  o->precond = SEM_PRECOND_JACOBI;
  o->precond_prec = SEM_FP64;
  o->cheb_order = 3;
  o->lmax = 0.0;
  o->rtol = 1e-10;
  o->max_iter = 10000;
  o->fixed_iters = 0;
  o->inner_rtol = 1e-5;
  o->max_outer = 30;
  o->check_every = 0;
  o->profile = 0;
  o->residual_history = nullptr;
}

const char* sem_last_error(void) { return g_last_error.c_str(); }

sem_status sem_gll(int32_t N, double* xi, double* rho, double* D) {
  g_last_error.clear();
  return host_gll(N, xi, rho, D);
}

sem_status sem_host_numbering(int32_t N, int64_t E, const int64_t* gid, const uint8_t* dirichlet,
                              int32_t* free_index, int64_t* n_unique, int64_t* n_free,
                              int64_t* n_shared) {
  HostNumbering hn;
  sem_status st = build_numbering(N, E, gid, dirichlet, hn);
  if (st) return st;
  if (free_index) std::memcpy(free_index, hn.lmap.data(), hn.lmap.size() * sizeof(int32_t));
  if (n_unique) *n_unique = hn.n_unique;
  if (n_free) *n_free = hn.n_free;
  if (n_shared) *n_shared = hn.n_shared;
  return SEM_OK;
}

sem_status sem_setup_mesh(const sem_mesh_desc* desc, void* stream, sem_mesh** out) {
  if (!desc || !out) return fail(SEM_EINVAL, "desc and out must not be NULL");
  *out = nullptr;
  const int N = desc->N;
  const int64_t E = desc->E;
  if (N < 1 || N > kMaxOrder) return fail(SEM_EINVAL, "N must be in [1, 10]");
  if (E < 1) return fail(SEM_EINVAL, "E must be >= 1");
  if (!desc->xyz || !desc->gid) return fail(SEM_EINVAL, "xyz and gid must not be NULL");
  const int64_t P = (int64_t)(N + 1) * (N + 1) * (N + 1);
  if (E > (int64_t)0x7fffffff / P) return fail(SEM_EINVAL, "E*(N+1)^3 must be < 2^31");
  const int64_t nL = E * P;
  for (int64_t a = 0; a < 3 * nL; ++a)
    if (!std::isfinite(desc->xyz[a])) return fail(SEM_EINVAL, "xyz holds a non-finite value");

  HostNumbering hn;
  sem_status st = build_numbering(N, E, desc->gid, desc->dirichlet, hn);
  if (st) return st;

  hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<sem_mesh> m(new sem_mesh());
  m->N = N;
  m->n1 = N + 1;
  m->P = (int)P;
  m->E = E;
  m->nL = nL;
  m->n_unique = hn.n_unique;
  m->n_free = hn.n_free;
  m->n_shared = hn.n_shared;
  m->n_dloc = (int64_t)hn.dlist.size();
  m->nullspace = (hn.n_free == hn.n_unique);
  SEM_HIP(hipGetDevice(&m->device));

  const int n1 = N + 1;
  std::vector<double> Dh(n1 * n1 + n1);
  if ((st = host_gll(N, nullptr, Dh.data() + n1 * n1, Dh.data()))) return st;
  std::memcpy(m->h_D, Dh.data(), n1 * n1 * sizeof(double));
  std::vector<float> D32(n1 * n1);
  for (int a = 0; a < n1 * n1; ++a) D32[a] = (float)Dh[a];
  if ((st = upload(m->D64, Dh, s)) || (st = upload(m->D32, D32, s))) return st;

  if ((st = m->G64.ensure((size_t)E * 6 * P * sizeof(double))) ||
      (st = m->B64.ensure((size_t)nL * sizeof(double))) ||
      (st = m->G32.ensure((size_t)E * 6 * P * sizeof(float))) ||
      (st = m->B32.ensure((size_t)nL * sizeof(float))))
    return st;
  {
    DevBuf dxyz, dbad;
    if ((st = dxyz.ensure((size_t)3 * nL * sizeof(double))) || (st = dbad.ensure(sizeof(int))))
      return st;
    SEM_HIP(hipMemcpyAsync(dxyz.p, desc->xyz, (size_t)3 * nL * sizeof(double),
                           hipMemcpyHostToDevice, s));
    SEM_HIP(launch_fill<int>(dbad.as<int>(), 1, 0, s));
    SEM_HIP(launch_geometry(m.get(), dxyz.as<double>(), m->G64.as<double>(), m->B64.as<double>(),
                            m->G32.as<float>(), m->B32.as<float>(), dbad.as<int>(), s));
    int bad = 0;
    SEM_HIP(hipMemcpyAsync(&bad, dbad.p, sizeof(int), hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    if (bad > 0)
      return fail(SEM_EINVAL, "element map is not orientation-preserving (detJ <= 0) at " +
                                  std::to_string(bad) + " points");
  }
  // routing of the in-solve operator: single-copy free nodes are written
  // straight to the free vector, shared ones through the segmented sum (the
  // host array lives until the stream is synchronised below)
  std::vector<int32_t> lmap2(hn.lmap.size()), fperm2(hn.fperm);
  for (size_t q = 0; q < hn.lmap.size(); ++q) {
    const int32_t v = hn.lmap[q];
    lmap2[q] = v < 0 ? -1 : v < hn.n_single ? v : -(v + 2);
  }
  // shared copies are stored at their element's surface slots
  bool surf = true;
  for (int64_t a = hn.fseg[hn.n_single]; a < (int64_t)fperm2.size() && surf; ++a) {
    const int64_t q = fperm2[a];
    const int64_t e = q / P, ql = q - e * P;
    const int r = surface_rank((int)(ql % n1), (int)((ql / n1) % n1), (int)(ql / (n1 * n1)), N);
    if (r < 0) surf = false;
    else fperm2[a] = (int32_t)(e * P + r);
  }
  m->n_single = hn.n_single;
  m->split_ok = surf;
  if (const char* ev = std::getenv("SEM_AX_NT_BYTES")) {
    char* end = nullptr;
    const long long v = std::strtoll(ev, &end, 10);
    if (end != ev && *end == '\0' && v >= 0) m->ax_nt_bytes = (int64_t)v;
  }
  if ((st = upload(m->lmap2, lmap2, s)) || (st = upload(m->fperm2, fperm2, s))) return st;
  if ((st = upload(m->lmap, hn.lmap, s)) || (st = upload(m->fseg, hn.fseg, s)) ||
      (st = upload(m->fperm, hn.fperm, s)) || (st = upload(m->gseg, hn.gseg, s)) ||
      (st = upload(m->gperm, hn.gperm, s)) || (st = upload(m->dlist, hn.dlist, s)))
    return st;
  SEM_HIP(hipStreamSynchronize(s));
  *out = m.release();
  return SEM_OK;
}

sem_status sem_free_mesh(sem_mesh* mesh) {
  if (!mesh) return SEM_OK;
  (void)hipDeviceSynchronize();
  delete mesh;
  return SEM_OK;
}

sem_status sem_get_info(const sem_mesh* m, sem_mesh_info* info) {
  if (sem_status st = check_mesh(m)) return st;
  if (!info) return fail(SEM_EINVAL, "info is NULL");
  info->E = m->E;
  info->n_local = m->nL;
  info->n_unique = m->n_unique;
  info->n_free = m->n_free;
  info->n_shared = m->n_shared;
  info->N = m->N;
  info->has_nullspace = m->nullspace ? 1 : 0;
  return SEM_OK;
}

sem_status sem_get_geometry(const sem_mesh* m, double* G, double* B, void* stream) {
  if (sem_status st = check_mesh(m)) return st;
  hipStream_t s = (hipStream_t)stream;
  if (G)
    SEM_HIP(hipMemcpyAsync(G, m->G64.p, (size_t)m->E * 6 * m->P * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
  if (B)
    SEM_HIP(hipMemcpyAsync(B, m->B64.p, (size_t)m->nL * sizeof(double), hipMemcpyDeviceToDevice, s));
  return SEM_OK;
}

sem_status sem_ax(const sem_mesh* m, const void* u, void* w, const void* k, double h2,
                  sem_prec prec, void* stream) {
  if (sem_status st = check_mesh(m)) return st;
  if (!u || !w) return fail(SEM_EINVAL, "u and w must not be NULL");
  if (u == w) return fail(SEM_EINVAL, "w must not alias u");
  if (!(h2 >= 0.0) || !std::isfinite(h2)) return fail(SEM_EINVAL, "h2 must be finite and >= 0");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (prec == SEM_FP64) {
    e = launch_ax<double>(m, (const double*)u, nullptr, (double*)w, (const double*)k, h2,
                          m->G64.as<double>(), m->B64.as<double>(), m->D64.as<double>(), s);
  } else if (prec == SEM_FP32) {
    e = launch_ax<float>(m, (const float*)u, nullptr, (float*)w, (const float*)k, (float)h2,
                         m->G32.as<float>(), m->B32.as<float>(), m->D32.as<float>(), s);
  } else if (prec == SEM_BF16_MFMA || prec == SEM_FP16_MFMA) {
    e = launch_ax<float>(m, (const float*)u, nullptr, (float*)w, (const float*)k, (float)h2,
                         m->G32.as<float>(), m->B32.as<float>(), m->D32.as<float>(), s, nullptr,
                         lp_of(prec));
  } else {
    return fail(SEM_EINVAL, "unknown precision");
  }
  if (e != hipSuccess) return hip_fail(e, "sem_ax");
  return SEM_OK;
}

sem_status sem_mass(const sem_mesh* m, const void* u, void* w, sem_prec prec, void* stream) {
  if (sem_status st = check_mesh(m)) return st;
  if (!u || !w) return fail(SEM_EINVAL, "u and w must not be NULL");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (prec == SEM_FP64)
    e = launch_mass<double>(m->nL, m->B64.as<double>(), (const double*)u, (double*)w, s);
  else if (prec == SEM_FP32)
    e = launch_mass<float>(m->nL, m->B32.as<float>(), (const float*)u, (float*)w, s);
  else
    return fail(SEM_EINVAL, "sem_mass supports SEM_FP64 and SEM_FP32");
  if (e != hipSuccess) return hip_fail(e, "sem_mass");
  return SEM_OK;
}

sem_status sem_gs(const sem_mesh* m, void* v, sem_prec prec, void* stream) {
  if (sem_status st = check_mesh(m)) return st;
  if (!v) return fail(SEM_EINVAL, "v must not be NULL");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (prec == SEM_FP64) e = launch_gs_local<double>(m, (double*)v, s);
  else if (prec == SEM_FP32) e = launch_gs_local<float>(m, (float*)v, s);
  else return fail(SEM_EINVAL, "sem_gs supports SEM_FP64 and SEM_FP32");
  if (e != hipSuccess) return hip_fail(e, "sem_gs");
  return SEM_OK;
}

sem_status sem_mask(const sem_mesh* m, void* v, sem_prec prec, void* stream) {
  if (sem_status st = check_mesh(m)) return st;
  if (!v) return fail(SEM_EINVAL, "v must not be NULL");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (prec == SEM_FP64) e = launch_mask_local<double>(m, (double*)v, s);
  else if (prec == SEM_FP32) e = launch_mask_local<float>(m, (float*)v, s);
  else return fail(SEM_EINVAL, "sem_mask supports SEM_FP64 and SEM_FP32");
  if (e != hipSuccess) return hip_fail(e, "sem_mask");
  return SEM_OK;
}

sem_status sem_jacobi_inverse(const sem_mesh* m, const double* k, double h2, double* dinv,
                              void* stream) {
  if (sem_status st = check_mesh(m)) return st;
  if (!dinv) return fail(SEM_EINVAL, "dinv must not be NULL");
  if (!(h2 >= 0.0) || !std::isfinite(h2)) return fail(SEM_EINVAL, "h2 must be finite and >= 0");
  hipStream_t s = (hipStream_t)stream;
  SolveWork& W = work_of(m);
  sem_status st = prepare_dinv(m, W, k, h2, s);
  if (st) return st;
  SEM_HIP((launch_free_to_local<double, double>(m, W.dinv.as<double>(), dinv, s)));
  return SEM_OK;
}

sem_status sem_cheb_apply(const sem_mesh* m, const double* r, double* z, const double* k,
                          double h2, int32_t order, double lmax, sem_prec prec, void* stream) {
  if (sem_status st = check_mesh(m)) return st;
  if (!r || !z) return fail(SEM_EINVAL, "r and z must not be NULL");
  if (order < 1) return fail(SEM_EINVAL, "order must be >= 1");
  if (!(lmax > 0.0) || !std::isfinite(lmax)) return fail(SEM_EINVAL, "lmax must be > 0");
  if (!(h2 >= 0.0) || !std::isfinite(h2)) return fail(SEM_EINVAL, "h2 must be finite and >= 0");
  if (!prec_ok(prec)) return fail(SEM_EINVAL, "unknown precision");
  hipStream_t s = (hipStream_t)stream;
  SolveWork& W = work_of(m);
  sem_status st = W.init(m, 1);
  if (st) return st;
  if ((st = prepare_dinv(m, W, k, h2, s))) return st;
  double* rf = W.vec<double>(W.tmpf, m->n_free);
  double* zf = W.vec<double>(W.z, m->n_free);
  if (!rf || !zf) return fail(SEM_ENOMEM, "work space");
  SEM_HIP((launch_local_to_free_avg<double, double>(m, r, rf, s)));
  if (prec == SEM_FP64) {
    st = cheb_apply_dev<double, double>(m, W, op64_of(m, k, h2), W.dinv.as<double>(), rf, zf, order,
                                        lmax, ChebCg(), s, nullptr);
  } else {
    Op<float> o32;
    if ((st = op32_of(m, W, k, h2, s, o32))) return st;
    o32.lp = lp_of(prec);
    st = cheb_apply_dev<double, float>(m, W, o32, W.dinv32.as<float>(), rf, zf, order, lmax,
                                       ChebCg(), s, nullptr);
  }
  if (st) return st;
  SEM_HIP((launch_free_to_local<double, double>(m, zf, z, s)));
  return SEM_OK;
}

void sem_pmg_opts_default(sem_pmg_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->smooth_order = 4;
  o->coarse_iters = 30;
  o->smoother = SEM_SMOOTH_SCHWARZ;
}

sem_status sem_setup_pmg(sem_mesh* m, const sem_mesh_desc* desc, const sem_pmg_opts* opts_in,
                         void* stream) {
  if (sem_status st = check_mesh(m)) return st;
  if (!desc || !desc->xyz || !desc->gid) return fail(SEM_EINVAL, "desc, xyz and gid are required");
  if (desc->N != m->N || desc->E != m->E)
    return fail(SEM_EINVAL, "the description differs from the one the mesh was set up with");
  sem_pmg_opts opts;
  if (opts_in) opts = *opts_in;
  else sem_pmg_opts_default(&opts);
  if (opts.smooth_order < 1) return fail(SEM_EINVAL, "smooth_order must be >= 1");
  if (opts.coarse_iters < 1) return fail(SEM_EINVAL, "coarse_iters must be >= 1");
  if (opts.smoother != SEM_SMOOTH_JACOBI && opts.smoother != SEM_SMOOTH_SCHWARZ)
    return fail(SEM_EINVAL, "unknown smoother");
  std::vector<int> orders;
  if (opts.n_levels == 0) {
    for (int n = m->N; ; n /= 2) {
      orders.push_back(n);
      if (n <= 1) break;
    }
  } else {
    if (opts.n_levels < 1 || opts.n_levels > SEM_PMG_MAX_LEVELS)
      return fail(SEM_EINVAL, "n_levels must be in [0, 8]");
    for (int l = 0; l < opts.n_levels; ++l) orders.push_back(opts.orders[l]);
    if (orders[0] != m->N) return fail(SEM_EINVAL, "orders[0] must be the mesh order");
    for (size_t l = 1; l < orders.size(); ++l)
      if (!(orders[l] >= 1 && orders[l] < orders[l - 1]))
        return fail(SEM_EINVAL, "level orders must decrease strictly and stay >= 1");
  }
  hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<Pmg, void (*)(Pmg*)> P(new Pmg(), pmg_destroy);
  P->smooth_order = opts.smooth_order;
  P->coarse_iters = opts.coarse_iters;
  P->smoother = opts.smoother;
  P->lv.resize(orders.size());
  const int64_t E = m->E;
  sem_status st;
  for (size_t l = 0; l < orders.size(); ++l) {
    PmgLevel& L = P->lv[l];
    L.N = orders[l];
    const bool smooths = l + 1 < orders.size();
    if (l == 0) {
      L.m = m;
      if (smooths && opts.smoother == SEM_SMOOTH_SCHWARZ &&
          (st = setup_schwarz(L, desc->N, E, desc->gid, desc->dirichlet, desc->xyz, s)))
        return st;
      continue;
    }
    const int Nc = orders[l];
    const int64_t Pc = (int64_t)(Nc + 1) * (Nc + 1) * (Nc + 1);
    std::vector<int64_t> gid_c((size_t)(E * Pc));
    std::vector<uint8_t> dir_c(desc->dirichlet ? (size_t)(E * Pc) : 0);
    std::vector<double> xyz_c((size_t)(3 * E * Pc));
    if ((st = host_coarse_mesh(m->N, E, desc->gid, desc->dirichlet, desc->xyz, Nc, gid_c.data(),
                               desc->dirichlet ? dir_c.data() : nullptr, xyz_c.data())))
      return st;
    sem_mesh_desc dc{Nc, E, xyz_c.data(), gid_c.data(), desc->dirichlet ? dir_c.data() : nullptr};
    sem_mesh* mc = nullptr;
    if ((st = sem_setup_mesh(&dc, stream, &mc))) return st;
    L.m = mc;
    L.owned = true;
    if (smooths && opts.smoother == SEM_SMOOTH_SCHWARZ &&
        (st = setup_schwarz(L, Nc, E, gid_c.data(), desc->dirichlet ? dir_c.data() : nullptr,
                            xyz_c.data(), s)))
      return st;
    std::vector<double> Ik((size_t)(Nc + 1) * (m->N + 1));
    if ((st = host_interp_matrix(m->N, Nc, Ik.data())) || (st = upload(L.Ik64, Ik, s))) return st;
  }
  for (size_t l = 0; l + 1 < orders.size(); ++l) {
    PmgLevel& L = P->lv[l];
    const int nf = orders[l] + 1, nc = orders[l + 1] + 1;
    std::vector<double> J((size_t)nf * nc), JT((size_t)nc * nf);
    if ((st = host_interp_matrix(orders[l + 1], orders[l], J.data()))) return st;
    for (int i = 0; i < nf; ++i)
      for (int j = 0; j < nc; ++j) JT[(size_t)j * nf + i] = J[(size_t)i * nc + j];
    std::vector<float> J32(J.begin(), J.end()), JT32(JT.begin(), JT.end());
    if ((st = upload(L.J64, J, s)) || (st = upload(L.JT64, JT, s)) || (st = upload(L.J32, J32, s)) ||
        (st = upload(L.JT32, JT32, s)))
      return st;
  }
  SEM_HIP(hipStreamSynchronize(s));
  pmg_destroy(m->pmg);
  m->pmg = P.release();
  return SEM_OK;
}

sem_status sem_pmg_info(const sem_mesh* m, int32_t* n_levels, int32_t* orders, double* rho_hat) {
  if (sem_status st = check_mesh(m)) return st;
  if (!m->pmg) return fail(SEM_EINVAL, "no multigrid hierarchy: call sem_setup_pmg first");
  const auto& lv = m->pmg->lv;
  if (n_levels) *n_levels = (int32_t)lv.size();
  for (size_t l = 0; l < SEM_PMG_MAX_LEVELS; ++l) {
    if (orders) orders[l] = l < lv.size() ? lv[l].N : 0;
    if (rho_hat) rho_hat[l] = l < lv.size() ? lv[l].rho_hat : 0.0;
  }
  return SEM_OK;
}

sem_status sem_pmg_apply(const sem_mesh* m, const double* r, double* z, const double* k,
                         double h2, sem_prec prec, void* stream) {
  if (sem_status st = check_mesh(m)) return st;
  if (!r || !z) return fail(SEM_EINVAL, "r and z must not be NULL");
  if (!(h2 >= 0.0) || !std::isfinite(h2)) return fail(SEM_EINVAL, "h2 must be finite and >= 0");
  if (prec != SEM_FP64 && prec != SEM_FP32) return fail(SEM_EINVAL, "prec must be FP64 or FP32");
  if (!m->pmg) return fail(SEM_EINVAL, "no multigrid hierarchy: call sem_setup_pmg first");
  hipStream_t s = (hipStream_t)stream;
  sem_status st;
  if (m->n_free == 0) {  // no unknowns: z = 0 at every copy
    SEM_HIP(launch_fill<double>(z, m->nL, 0.0, s));
    return SEM_OK;
  }
  if ((st = pmg_prepare(m, k, h2, prec == SEM_FP64, s))) return st;
  SolveWork& W = work_of(m);
  double* rf = W.vec<double>(W.tmpf, m->n_free);
  double* zf = W.vec<double>(W.z, m->n_free);
  if (!rf || !zf) return fail(SEM_ENOMEM, "work space");
  SEM_HIP((launch_local_to_free_avg<double, double>(m, r, rf, s)));
  if (prec == SEM_FP64) st = pmg_precond<double, double>(m, W, rf, zf, ChebCg(), s, nullptr);
  else st = pmg_precond<double, float>(m, W, rf, zf, ChebCg(), s, nullptr);
  if (st) return st;
  SEM_HIP((launch_free_to_local<double, double>(m, zf, z, s)));
  return SEM_OK;
}

sem_status sem_host_schwarz(int32_t N, int64_t E, const int64_t* gid, const uint8_t* dirichlet,
                            const double* xyz, int32_t* xmap, double* S, double* lam) {
  if (!gid || !xyz || !xmap) return fail(SEM_EINVAL, "gid, xyz and xmap are required");
  HostNumbering hn;
  sem_status st = build_numbering(N, E, gid, dirichlet, hn);
  if (st) return st;
  SchwarzHost H;
  if ((st = build_schwarz(N, E, gid, dirichlet, xyz, hn.lmap.data(), hn.n_free, H))) return st;
  std::memcpy(xmap, H.xmap.data(), H.xmap.size() * sizeof(int32_t));
  if (S) std::memcpy(S, H.S.data(), H.S.size() * sizeof(double));
  if (lam) std::memcpy(lam, H.lam.data(), H.lam.size() * sizeof(double));
  return SEM_OK;
}

sem_status sem_host_coarse_mesh(int32_t N, int64_t E, const int64_t* gid,
                                const uint8_t* dirichlet, const double* xyz, int32_t Nc,
                                int64_t* gid_c, uint8_t* dirichlet_c, double* xyz_c) {
  if ((xyz == nullptr) != (xyz_c == nullptr))
    return fail(SEM_EINVAL, "xyz and xyz_c must both be given or both be NULL");
  return host_coarse_mesh(N, E, gid, dirichlet, xyz, Nc, gid_c, dirichlet_c, xyz_c);
}

sem_status sem_advection_rule(int32_t N, int32_t rule, int32_t* q1, double* x, double* w,
                              double* J) {
  if (sem_status st = host_adv_rule(N, rule, x, w, J)) return st;
  if (q1) *q1 = adv_points(N, rule);
  return SEM_OK;
}

sem_status sem_setup_advection(sem_mesh* m, const sem_mesh_desc* desc, int32_t rule,
                               void* stream) {
  if (sem_status st = check_mesh(m)) return st;
  if (!desc || !desc->xyz) return fail(SEM_EINVAL, "desc and xyz are required");
  if (desc->N != m->N || desc->E != m->E)
    return fail(SEM_EINVAL, "the description differs from the one the mesh was set up with");
  if (rule != SEM_ADV_COLLOCATION && rule != SEM_ADV_DEALIAS)
    return fail(SEM_EINVAL, "unknown quadrature rule");
  for (int64_t a = 0; a < 3 * m->nL; ++a)
    if (!std::isfinite(desc->xyz[a])) return fail(SEM_EINVAL, "xyz holds a non-finite value");
  hipStream_t s = (hipStream_t)stream;
  const int n = m->n1, q1 = adv_points(m->N, rule);
  const int64_t Q = (int64_t)q1 * q1 * q1;
  std::vector<double> x(q1), w(q1), J((size_t)q1 * n);
  sem_status st;
  if ((st = host_adv_rule(m->N, rule, x.data(), w.data(), J.data()))) return st;
  // J, JD = J D, J^T
  std::vector<double> mats((size_t)3 * q1 * n);
  double* JD = mats.data() + q1 * n;
  double* JT = JD + q1 * n;
  for (int i = 0; i < q1; ++i)
    for (int j = 0; j < n; ++j) {
      double acc = 0.0;
      for (int l = 0; l < n; ++l) acc += J[i * n + l] * m->h_D[l * n + j];
      mats[i * n + j] = J[i * n + j];
      JD[i * n + j] = acc;
      JT[j * q1 + i] = J[i * n + j];
    }
  std::vector<float> mats32(mats.begin(), mats.end());
  std::unique_ptr<AdvRule> R(new AdvRule());
  R->q1 = q1;
  if ((st = upload(R->mats64, mats, s)) || (st = upload(R->mats32, mats32, s)) ||
      (st = R->G64.ensure((size_t)m->E * 9 * Q * sizeof(double))) ||
      (st = R->G32.ensure((size_t)m->E * 9 * Q * sizeof(float))))
    return st;
  DevBuf dxyz, dw, dbad;
  if ((st = dxyz.ensure((size_t)3 * m->nL * sizeof(double))) || (st = upload(dw, w, s)) ||
      (st = dbad.ensure(sizeof(int))))
    return st;
  SEM_HIP(hipMemcpyAsync(dxyz.p, desc->xyz, (size_t)3 * m->nL * sizeof(double),
                         hipMemcpyHostToDevice, s));
  SEM_HIP(launch_fill<int>(dbad.as<int>(), 1, 0, s));
  SEM_HIP(launch_adv_geometry(m, q1, R->mats64.as<double>(), dw.as<double>(),
                              dxyz.as<double>(), R->G64.as<double>(), R->G32.as<float>(),
                              dbad.as<int>(), s));
  int bad = 0;
  SEM_HIP(hipMemcpyAsync(&bad, dbad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  if (bad > 0)
    return fail(SEM_EINVAL, "element map is not orientation-preserving (detJ <= 0) at " +
                                std::to_string(bad) + " quadrature points");
  delete m->adv[rule];
  m->adv[rule] = R.release();
  return SEM_OK;
}

sem_status sem_get_advection_factors(const sem_mesh* m, int32_t rule, double* G, void* stream) {
  if (sem_status st = check_mesh(m)) return st;
  if (rule != SEM_ADV_COLLOCATION && rule != SEM_ADV_DEALIAS)
    return fail(SEM_EINVAL, "unknown quadrature rule");
  const AdvRule* R = m->adv[rule];
  if (!R) return fail(SEM_EINVAL, "rule not set up: call sem_setup_advection first");
  if (!G) return fail(SEM_EINVAL, "G must not be NULL");
  const size_t nb = (size_t)m->E * 9 * R->q1 * R->q1 * R->q1 * sizeof(double);
  SEM_HIP(hipMemcpyAsync(G, R->G64.p, nb, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return SEM_OK;
}

static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char *pa = (const char*)a, *pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

sem_status sem_advect_fields(const sem_mesh* m, int32_t rule, const void* u, int32_t nf,
                             const void* f, void* out, sem_prec prec, void* stream) {
  if (sem_status st = check_mesh(m)) return st;
  if (rule != SEM_ADV_COLLOCATION && rule != SEM_ADV_DEALIAS)
    return fail(SEM_EINVAL, "unknown quadrature rule");
  const AdvRule* R = m->adv[rule];
  if (!R) return fail(SEM_EINVAL, "rule not set up: call sem_setup_advection first");
  if (nf < 0) return fail(SEM_EINVAL, "nf must be >= 0");
  if (nf == 0) return SEM_OK;
  if (!u || !f || !out) return fail(SEM_EINVAL, "u, f and out must not be NULL");
  if (prec != SEM_FP64 && prec != SEM_FP32) return fail(SEM_EINVAL, "prec must be FP64 or FP32");
  const size_t sz = prec == SEM_FP64 ? sizeof(double) : sizeof(float), nb = (size_t)m->nL * sz;
  if (overlaps(out, nf * nb, u, 3 * nb) || overlaps(out, nf * nb, f, nf * nb))
    return fail(SEM_EINVAL, "out must not overlap u or f");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (prec == SEM_FP64)
    e = launch_advect<double>(m, rule, nf, R->mats64.as<double>(), m->D64.as<double>(),
                              R->G64.as<double>(), (const double*)u, (const double*)f,
                              (double*)out, s);
  else
    e = launch_advect<float>(m, rule, nf, R->mats32.as<float>(), m->D32.as<float>(),
                             R->G32.as<float>(), (const float*)u, (const float*)f, (float*)out,
                             s);
  if (e != hipSuccess) return hip_fail(e, "advect");
  return SEM_OK;
}

sem_status sem_advect(const sem_mesh* m, int32_t rule, const void* u, const void* f, void* out,
                      sem_prec prec, void* stream) {
  return sem_advect_fields(m, rule, u, 1, f, out, prec, stream);
}

sem_status sem_lmax_estimate(const sem_mesh* m, const double* k, double h2, int32_t steps,
                             double* lmax, void* stream) {
  if (sem_status st = check_mesh(m)) return st;
  if (!lmax) return fail(SEM_EINVAL, "lmax must not be NULL");
  if (steps < 1) return fail(SEM_EINVAL, "steps must be >= 1");
  if (!(h2 >= 0.0) || !std::isfinite(h2)) return fail(SEM_EINVAL, "h2 must be finite and >= 0");
  if (m->n_free == 0) return fail(SEM_EINVAL, "the mesh has no free node (every node Dirichlet)");
  return estimate_lmax(m, work_of(m), k, h2, steps, lmax, (hipStream_t)stream);
}

sem_status sem_pcg_solve(const sem_mesh* m, const double* b, double* x, const double* k,
                         double h2, const sem_solve_opts* opts_in, sem_solve_stats* stats,
                         void* stream) {
  if (sem_status st = check_mesh(m)) return st;
  if (!b || !x) return fail(SEM_EINVAL, "b and x must not be NULL");
  if (!(h2 >= 0.0) || !std::isfinite(h2)) return fail(SEM_EINVAL, "h2 must be finite and >= 0");
  sem_solve_opts opts;
  if (sem_status st = solve_options(m, opts_in, opts)) return st;
  hipStream_t s = (hipStream_t)stream;
  // b and x0 are read as the mean of their copies
  const SolveLoad load = [&](double* bf, double* xf, bool* x_zero) -> sem_status {
    SEM_HIP((launch_local_to_free_avg<double, double>(m, b, bf, s)));
    SEM_HIP((launch_local_to_free_avg<double, double>(m, x, xf, s)));
    double xd[3];
    if (sem_status st = free_dots_f64(m, work_of(m), xf, nullptr, xd, s)) return st;
    if (!std::isfinite(xd[0])) return fail(SEM_EINVAL, "x0 is not finite");
    *x_zero = xd[0] == 0.0;
    return SEM_OK;
  };
  const SolveStore store = [&](const double* xf) -> sem_status {
    SEM_HIP((launch_free_to_local<double, double>(m, xf, x, s)));
    return SEM_OK;
  };
  return solve_free(m, k, h2, opts, load, store, stats, s);
}

sem_status sem_solve_backward(const sem_mesh* m, const double* x, const double* xbar,
                              const double* k, double h2, const sem_solve_opts* opts_in,
                              double* kbar, double* bbar, sem_solve_stats* stats, void* stream) {
  if (sem_status st = check_mesh(m)) return st;
  if (!xbar) return fail(SEM_EINVAL, "xbar must not be NULL");
  if (!kbar && !bbar) return fail(SEM_EINVAL, "kbar and bbar are both NULL");
  if (kbar && !x) return fail(SEM_EINVAL, "kbar needs the forward solution x");
  if (kbar && (kbar == x || kbar == bbar))
    return fail(SEM_EINVAL, "kbar must not alias x or bbar");
  if (bbar && bbar == x) return fail(SEM_EINVAL, "bbar must not alias x");
  if (!(h2 >= 0.0) || !std::isfinite(h2)) return fail(SEM_EINVAL, "h2 must be finite and >= 0");
  sem_solve_opts opts;
  if (sem_status st = solve_options(m, opts_in, opts)) return st;
  hipStream_t s = (hipStream_t)stream;
  // adjoint right-hand side R Q^T xbar (the transpose of copying the free
  // solution to every local copy), adjoint solve from zero
  const SolveLoad load = [&](double* bf, double* xf, bool* x_zero) -> sem_status {
    SEM_HIP((launch_free_sum<double, double>(m, xbar, bf, s)));
    SEM_HIP(launch_fill<double>(xf, m->n_free, 0.0, s));
    *x_zero = true;
    return SEM_OK;
  };
  // lambda = the adjoint solution: dL/dk = -kbar(lambda_L, x_L); dL/db at a
  // copy = lambda / (copies of its node), the transpose of reading b as the
  // mean of its copies
  const SolveStore store = [&](const double* lam) -> sem_status {
    if (kbar) {
      SolveWork& W = work_of(m);
      double* lamL = W.vec<double>(W.wL, m->nL);
      if (!lamL) return fail(SEM_ENOMEM, "work space");
      SEM_HIP((launch_free_to_local<double, double>(m, lam, lamL, s)));
      SEM_HIP(launch_ax_kbar(m, x, lamL, kbar, -1.0, s));
    }
    if (bbar) SEM_HIP(launch_free_to_local_per_copy(m, lam, bbar, s));
    return SEM_OK;
  };
  return solve_free(m, k, h2, opts, load, store, stats, s);
}

sem_status sem_ax_backward(const sem_mesh* m, const double* u, const double* wbar, const double* k,
                           double h2, double* ubar, double* kbar, void* stream) {
  if (sem_status st = check_mesh(m)) return st;
  if (!u || !wbar) return fail(SEM_EINVAL, "u and wbar must not be NULL");
  if (!(h2 >= 0.0) || !std::isfinite(h2)) return fail(SEM_EINVAL, "h2 must be finite and >= 0");
  if (ubar == wbar) return fail(SEM_EINVAL, "ubar must not alias wbar");
  hipStream_t s = (hipStream_t)stream;
  if (ubar) {
    hipError_t e = launch_ax<double>(m, wbar, nullptr, ubar, k, h2, m->G64.as<double>(),
                                     m->B64.as<double>(), m->D64.as<double>(), s);
    if (e != hipSuccess) return hip_fail(e, "sem_ax_backward (ubar)");
  }
  if (kbar) {
    hipError_t e = launch_ax_kbar(m, u, wbar, kbar, 1.0, s);
    if (e != hipSuccess) return hip_fail(e, "sem_ax_backward (kbar)");
  }
  return SEM_OK;
}

}  // extern "C"
