// Internal interface of the solver drivers.
#pragma once

#include <functional>
#include <vector>

#include "common.hpp"

namespace sem {

// Per-mesh work space of the solve entry points (grown on demand, kept until
// sem_free_mesh).
struct SolveWork {
  DevBuf bf, x, r, p, w, z, wL, dinv, tmpf;          // FP64
  DevBuf x32, r32, ri32, p32, w32, z32, wL32, dinv32, k32; // FP32
  DevBuf cd, crk, cd32, crk32;                       // Chebyshev d and r_k
  DevBuf cwf, cza, cz;                               // fused Chebyshev: A d at single-copy
                                                     // nodes, running z, output z
  DevBuf part, sc, red, hist, ahist, bhist, epart;
  CgScalars* h_sc = nullptr;  // pinned: [0..1] polling slots, [3] upload
  double* h_red = nullptr;    // pinned reduction results
  std::vector<hipEvent_t> ev; // profiling events
  int ev_used = 0;
  hipStream_t cap = nullptr;  // stream used only to capture iteration graphs
  ~SolveWork();
  sem_status capture_stream(hipStream_t* out);
  sem_status init(const sem_mesh* m, int max_iter);
  template <typename T> T* vec(DevBuf& b, int64_t n);
};

// operator data in one precision
template <typename T>
struct Op {
  const T* G = nullptr;
  const T* B = nullptr;
  const T* k = nullptr;
  const T* D = nullptr;
  T h2 = T(0);
  const int32_t* skip = nullptr;  // device flag: nonzero = skip the launch's work
  int lp = 0;                     // FP32 only: 16-bit contraction operands (1 bf16, 2 half)
};

struct CgResult {
  int iters = 0;
  int applies = 0;
  int status = 0;  // 0 running/limit, 1 converged, 2 breakdown, 3 non-finite
  bool converged = false;
  double bnorm = 0.0, rnorm = 0.0;
};

// Coupling of a Chebyshev pass to an enclosing flexible CG iteration (all
// null/zero for a stand-alone apply): the first pass takes the convergence
// decision from the update's r.r partials `check_in`, the last one writes the
// z.r and z.(w - mean_w) partials for beta into `part_out`.
struct ChebCg {
  CgScalars* sc = nullptr;
  const void* w = nullptr;          // w = A p of the CG iteration (CG vector type)
  const double* check_in = nullptr;
  int nblk = 0;
  double* part_out = nullptr;
  double* hist = nullptr;
  // without `sc`: a solve's scalars whose `done` flag makes the pass return at
  // once (a preconditioner pass inside a V-cycle of a flexible CG)
  const CgScalars* skip_sc = nullptr;
};

template <typename T>
using ChebFn = std::function<sem_status(const sem_mesh*, SolveWork&, const T* r, T* z,
                                        const ChebCg& cg, hipStream_t s, int* applies)>;

// Chebyshev preconditioner of order >= 2 run inside the flexible CG's own
// kernels on the split operator in precision Tp (see k_update_cheb0); when
// `on`, the iterations use it and `cheb` only forms z_0 = M r_0
template <typename Tp>
struct ChebFuse {
  bool on = false;
  Op<Tp> op;
  const Tp* dinv = nullptr;
  int order = 3;
  double lmax = 0.0;
  int kind = 4;  // 4: fourth kind, 1: first kind on [lmax / 10, lmax]
};

// coefficients of a Chebyshev pass: d_0 = c0 S r, d_k = ca[k] d_{k-1} + cb[k] S r_k
void cheb_coeffs(int order, double lmax, int kind, double* c0, std::vector<double>& ca,
                 std::vector<double>& cb);

template <typename T, typename Tp>
struct CgArgs {
  Op<T> op;
  const T* b = nullptr;  // free rhs
  T *x = nullptr, *r = nullptr, *p = nullptr, *w = nullptr, *z = nullptr, *wL = nullptr;
  const T* dinv = nullptr;
  int precond = SEM_PRECOND_JACOBI;
  int cheb_order = 3;
  ChebFn<T> cheb;
  ChebFuse<Tp> fuse;
  double rtol = 1e-10;
  int max_it = 1000;
  bool fixed = false;
  bool x_zero = true;
  bool neumann = false;
  bool profile = false;
  int check_every = 0;
  // most iterations per chunk (graph capture and read-back interval); a
  // preconditioner of many launches (multigrid) asks for short chunks so
  // that neither the capture nor the overshoot past convergence replays
  // hundreds of launches
  int max_chunk = 16;
  double* hist = nullptr;                      // host, max_it + 1
  std::vector<double>* alpha_out = nullptr;    // CG coefficients (Lanczos)
  std::vector<double>* beta_out = nullptr;
};

template <typename T>
sem_status apply_op(const sem_mesh* m, SolveWork& W, const Op<T>& op, const T* xf, T* wL,
                    hipStream_t s, bool timed, T* wf = nullptr, double* epart = nullptr,
                    bool mean_sums = true);

// work vectors of one Chebyshev pass: d, r_k (free, n_free) and w_L (local, n_L)
template <typename Tp>
struct ChebBufs {
  Tp* d = nullptr;
  Tp* rk = nullptr;
  Tp* wL = nullptr;
};

// z = p_m(S A) S r with the work vectors taken from the mesh's work space
template <typename Tr, typename Tp>
sem_status cheb_apply_dev(const sem_mesh* m, SolveWork& W, const Op<Tp>& op, const Tp* dinv,
                          const Tr* r, Tr* z, int order, double lmax, const ChebCg& cg,
                          hipStream_t s, int* applies, int kind = 4);
// the same with caller-provided work vectors (no allocation)
template <typename Tr, typename Tp>
sem_status cheb_apply_bufs(const sem_mesh* m, const Op<Tp>& op, const Tp* dinv, const Tr* r,
                           Tr* z, int order, double lmax, const ChebCg& cg, hipStream_t s,
                           int* applies, int kind, const ChebBufs<Tp>& b);

template <typename T, typename Tp>
sem_status cg_solve(const sem_mesh* m, SolveWork& W, const CgArgs<T, Tp>& a, CgResult& res,
                    hipStream_t s);

sem_status free_remove_mean_f64(const sem_mesh* m, SolveWork& W, double* a, hipStream_t s);
sem_status free_dots_f64(const sem_mesh* m, SolveWork& W, const double* a, const double* b,
                         double out[3], hipStream_t s);
sem_status ir_residual(const sem_mesh* m, SolveWork& W, const Op<double>& op, const double* x,
                       const double* b, double* r, double out[2], hipStream_t s, bool timed);
sem_status ir_prepare(const sem_mesh* m, const double* r, float* r32, double shift, double scale,
                      hipStream_t s);
sem_status ir_update(const sem_mesh* m, double* x, const float* e, double sc, hipStream_t s);

// grid of the reducing vector kernels for n elements (= number of partials)
unsigned vec_grid(int64_t n);

// `iters` Jacobi-PCG iterations from x = 0 entirely on the device (W.sc holds
// the scalars; r, p, w free scratch, wL local scratch); the constant mode is
// projected out when `neumann`.  Every launch returns at once when `outer`
// (nullable) has finished.
template <typename T>
sem_status cg_fixed_device(const sem_mesh* m, SolveWork& W, const Op<T>& op, const T* dinv,
                           const T* b, T* x, T* r, T* p, T* w, T* wL, int iters, bool neumann,
                           const CgScalars* outer, hipStream_t s);
// convergence decision of a flexible CG iteration from the update's r.r partials
sem_status launch_cg_gate(const double* check_in, int nblk, CgScalars* sc, double* hist,
                          hipStream_t s);
// z = x in the CG's type; with sc: partials of z.r and z.(w - mean_w) into part
template <typename Tr, typename Tp>
sem_status launch_flex_dots(int64_t nf, const Tp* x, Tr* z, const Tr* r, const Tr* w,
                            double* part, const CgScalars* sc, hipStream_t s);
template <typename Tin, typename Tout>
sem_status launch_convert_skip(int64_t n, const Tin* a, Tout* b, const CgScalars* sc,
                               hipStream_t s);

}  // namespace sem
