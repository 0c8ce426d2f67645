/*
 * sem.h -- C ABI of libsem: a matrix-free spectral-element Poisson/Helmholtz
 * solve for AMD MI355X (gfx950).
 *
 * The discretisation is the one of the paper's solver (Sec. 2.2): N_e
 * hexahedral elements of polynomial order N, Gauss-Lobatto-Legendre (GLL)
 * nodes and quadrature, unknowns ordered as tensors (ijk, i fastest) on the
 * reference cube [-1,1]^3, operators applied matrix-free as dense
 * (N+1)x(N+1) contractions identical for all elements and carried to deformed
 * elements by the chain rule.  The pressure Poisson solve is the hardest part
 * of each time step and is solved by preconditioned conjugate gradients
 * (Sec. 2.2), with fourth-kind Chebyshev acceleration and preconditioner work
 * in FP32, which halves its memory traffic (Sec. 2.2).
 *
 * Notation used below:
 *   P   = (N+1)^3 local points per element, local index q = i + (N+1)(j + (N+1)k)
 *   n_L = E * P local points; "local vector" = array [E][P] (C order)
 *   copy-consistent local vector = all local copies of a global node hold the
 *   same value.
 *   G   = six geometric factors per local point, order (rr, rs, rt, ss, st, tt),
 *         G_ab = rho_i rho_j rho_k detJ (grad a . grad b); B = rho_i rho_j rho_k detJ.
 *   A_L = element (unassembled) operator:
 *         A_L(k) u = sum_ab D_a^T diag(k G_ab) D_b u + h2 B u
 *         (weak form of -div(k grad u) + h2 u);
 *   Q^T = sum of local copies into global nodes, Q = copy back; R = drop the
 *         Dirichlet nodes.  The assembled operator is A = R Q^T A_L Q R^T.
 *
 * Conventions for every entry point:
 *   - Pointers documented as DEVICE must point to device memory of the device
 *     that was current at sem_setup_mesh; HOST pointers to host memory.
 *   - The caller owns every vector it passes.  The library owns the mesh
 *     handle and everything inside it (geometry, numbering, work space) and
 *     releases it in sem_free_mesh.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *     work on it and return without waiting unless documented as blocking.
 *     A mesh handle is used from one stream at a time (its work space is
 *     per handle).
 *   - Errors: every call returns a sem_status; on SEM_EINVAL nothing was
 *     written.  sem_last_error() returns a thread-local message describing
 *     the last non-OK status of the calling thread.  HIP runtime failures
 *     map to SEM_EDEVICE with the HIP error string in the message.
 */
#ifndef SEM_H
#define SEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SEM_OK = 0,
  SEM_EINVAL = -1,     /* invalid argument, mesh or option */
  SEM_ENOMEM = -2,     /* device allocation failed */
  SEM_EDEVICE = -3,    /* HIP runtime error */
  SEM_ENOCONV = -4,    /* solve hit its iteration limit; x holds the last iterate */
  SEM_EBREAKDOWN = -5, /* CG breakdown (p.Ap <= 0 or not finite); x holds the last iterate */
  SEM_ENOTSUP = -6     /* valid request that the library does not implement */
} sem_status;

/* Arithmetic of an operator apply or of a preconditioner.
 * SEM_FP64: data and arithmetic in double.
 * SEM_FP32: data and arithmetic in float (vectors passed as float).
 * SEM_BF16_MFMA / SEM_FP16_MFMA: float data; the (N+1)x(N+1) derivative
 *   contractions run on the matrix cores with bfloat16 / IEEE-half operands
 *   (D, the element block of u, each metric-weighted derivative block; round
 *   to nearest even) and FP32 accumulation; metric, k and mass terms in FP32.
 *   For half every block is first scaled by a power of two that puts its
 *   largest magnitude in [2^14, 2^15) and the result scaled back, so small
 *   inputs (residuals) keep their bits.  Relative error about 4e-3 (bf16) and
 *   3e-4 (half) of the operator: meant for the preconditioner (Sec. 2.2 runs
 *   most preconditioner work in reduced precision). */
typedef enum { SEM_FP64 = 0, SEM_FP32 = 1, SEM_BF16_MFMA = 2, SEM_FP16_MFMA = 3 } sem_prec;

typedef struct sem_mesh sem_mesh; /* opaque, library-owned */

/* Mesh description (Sec. 2.2: N_e hexahedra of order N, ijk ordering). */
typedef struct {
  int32_t N;                /* polynomial order, 1 <= N <= 10 (the solver family uses p <= 10, Sec. 4.1) */
  int64_t E;                /* number of elements, >= 1, E*(N+1)^3 < 2^31 */
  const double* xyz;        /* HOST [E][P][3]: physical coordinates of every local node */
  const int64_t* gid;       /* HOST [E][P]: global node id >= 0; equal ids = one unknown
                               (periodicity is expressed by equal ids) */
  const uint8_t* dirichlet; /* HOST [E][P] or NULL (no Dirichlet nodes): nonzero = homogeneous
                               Dirichlet node; must agree between all copies of a node */
} sem_mesh_desc;

typedef struct {
  int64_t E, n_local, n_unique, n_free, n_shared; /* n_shared: unique nodes with >1 copy */
  int32_t N;
  int32_t has_nullspace; /* 1 if no Dirichlet node: the constant is in the kernel for h2 = 0 */
} sem_mesh_info;

/* Preconditioner of the CG.  SEM_PRECOND_CHEBYSHEV: fourth-kind Chebyshev-
 * Jacobi of order cheb_order (the acceleration Sec. 2.2 names).
 * SEM_PRECOND_PMG: one p-multigrid V-cycle per iteration (Sec. 2.2: the
 * default pressure preconditioner, p-multigrid with fourth-kind Chebyshev-
 * accelerated smoothing); needs sem_setup_pmg first.
 * SEM_PRECOND_CHEBYSHEV_FIRST: the classical first-kind Chebyshev semi-
 * iteration of order cheb_order on [rho_hat/10, rho_hat] (a comparison
 * variant; same cost per call as the fourth kind). */
typedef enum {
  SEM_PRECOND_JACOBI = 0,
  SEM_PRECOND_CHEBYSHEV = 1,
  SEM_PRECOND_PMG = 2,
  SEM_PRECOND_CHEBYSHEV_FIRST = 3
} sem_precond;
typedef enum { SEM_SOLVE_CG = 0, SEM_SOLVE_MIXED_IR = 1 } sem_solve_mode;

typedef struct {
  int32_t mode;         /* sem_solve_mode.  CG: FP64 (flexible when preconditioned by Chebyshev)
                           conjugate gradients on the assembled system.  MIXED_IR: FP64 iterative
                           refinement (true residual, update and norms in FP64) around an inner
                           FP32 preconditioned CG. */
  int32_t precond;      /* sem_precond of the CG (mode CG) or of the inner CG (MIXED_IR) */
  int32_t precond_prec; /* sem_prec of the Chebyshev preconditioner.  Mode CG: any (FP64 CG with
                           a lower-precision preconditioner); MIXED_IR: SEM_FP32, SEM_BF16_MFMA
                           or SEM_FP16_MFMA (the inner CG's own operator stays FP32).
                           Multigrid: SEM_FP32 (the cycle in float) or, in mode CG, SEM_FP64 */
  int32_t cheb_order;   /* Chebyshev order m >= 1 (m-1 operator applies per call); default 3 */
  double lmax;          /* Chebyshev bound rho_hat >= lambda_max(D^-1 A); <= 0: 1.1 x a
                           20-step CG-Lanczos estimate (cached per mesh for k == NULL) */
  double rtol;          /* stop when ||b - A x||_2 <= rtol ||b||_2 over the free unique nodes */
  int32_t max_iter;     /* CG iteration limit (mode CG) or total inner-iteration limit (MIXED_IR) */
  int32_t fixed_iters;  /* mode CG only: 1 = run exactly max_iter iterations (no early exit) */
  double inner_rtol;    /* MIXED_IR: relative residual reduction of each inner solve (default 1e-5);
                           the last steps only reduce by what is still missing to reach rtol */
  int32_t max_outer;    /* MIXED_IR: refinement step limit (default 30) */
  int32_t check_every;  /* iterations between convergence read-backs (0 = automatic) */
  int32_t profile;      /* 1: time every FP64 operator-apply kernel with HIP events into stats */
  double* residual_history; /* HOST, nullable, length max_iter + 1: ||r_i||_2 of the CG
                               recurrence (mode CG) */
} sem_solve_opts;

typedef struct {
  int32_t iters;        /* CG iterations (mode CG) or total inner iterations (MIXED_IR) */
  int32_t outer_iters;  /* MIXED_IR refinement steps (0 in mode CG) */
  int32_t operator_applies;  /* FP64 + low-precision operator applies */
  int32_t converged;    /* 1 if the tolerance was met */
  double rel_res;       /* final ||r|| / ||b|| of the recurrence (mode CG) or of the FP64 true
                           residual (MIXED_IR) */
  double time_ms;       /* wall time of the solve on the stream (HIP events) */
  double lmax;          /* Chebyshev bound used (0 for Jacobi) */
  double ax_ms;         /* profile = 1: summed duration of FP64 operator kernels */
  int32_t ax_launches;  /* profile = 1: number of FP64 operator kernels timed */
  int32_t pad_;
} sem_solve_stats;

/* Fill `opts` with defaults: mode CG, Jacobi, FP64, order 3, rtol 1e-10,
 * max_iter 10000, inner_rtol 1e-5, max_outer 30. */
void sem_solve_opts_default(sem_solve_opts* opts);

/* HOST-only.  GLL nodes xi[N+1] (ascending), weights rho[N+1] and derivative
 * matrix D[(N+1)*(N+1)] with D[i*(N+1)+j] = l_j'(xi_i) for 1 <= N <= 10 (the
 * nodal basis and quadrature of Sec. 2.2).  Any output may be NULL. */
sem_status sem_gll(int32_t N, double* xi, double* rho, double* D);

/* HOST-only.  The numbering sem_setup_mesh builds from gid/dirichlet:
 * free_index[E*P] (HOST, caller-allocated) receives for each local point the
 * index of its free unique node, or -1 for Dirichlet nodes: the free nodes
 * with a single local copy come first, then those with several, each class
 * in first-touch order (the order of first appearance in the local points);
 * n_unique / n_free / n_shared receive the counts.  Validates as
 * sem_setup_mesh does (gid >= 0, consistent Dirichlet flags). */
sem_status sem_host_numbering(int32_t N, int64_t E, const int64_t* gid, const uint8_t* dirichlet,
                              int32_t* free_index, int64_t* n_unique, int64_t* n_free,
                              int64_t* n_shared);

/* Build a mesh handle on the current HIP device: uploads the nodes,
 * computes G and B on the device (chain rule, Sec. 2.2), builds the
 * gather-scatter tables and checks detJ > 0 at every point (SEM_EINVAL
 * otherwise).  Blocks until done.  *out receives the handle. */
sem_status sem_setup_mesh(const sem_mesh_desc* desc, void* stream, sem_mesh** out);

/* Release a handle (NULL is allowed).  Waits for the device. */
sem_status sem_free_mesh(sem_mesh* mesh);

sem_status sem_get_info(const sem_mesh* mesh, sem_mesh_info* info);

/* Copy the geometric factors to caller buffers: G DEVICE double [E][6][P],
 * B DEVICE double [E][P] (either may be NULL).  Stream-ordered. */
sem_status sem_get_geometry(const sem_mesh* mesh, double* G, double* B, void* stream);

/* w = A_L(k) u, the element operator of Sec. 2.2 applied to every element
 * (unassembled).  u, w: DEVICE [E][P] of double (SEM_FP64) or float
 * (SEM_FP32, SEM_BF16_MFMA, SEM_FP16_MFMA); k: DEVICE [E][P] of the same type
 * or NULL (k = 1); h2 >= 0.  w must not alias u. */
sem_status sem_ax(const sem_mesh* mesh, const void* u, void* w, const void* k, double h2,
                  sem_prec prec, void* stream);

/* w = B u (the diagonal GLL mass matrix), DEVICE [E][P], FP64 or FP32. */
sem_status sem_mass(const sem_mesh* mesh, const void* u, void* w, sem_prec prec, void* stream);

/* Direct-stiffness summation v <- Q Q^T v in place: every local copy of a
 * global node receives the sum over its copies, summed in ascending local
 * index order (deterministic).  v: DEVICE [E][P], FP64 or FP32. */
sem_status sem_gs(const sem_mesh* mesh, void* v, sem_prec prec, void* stream);

/* Zero every local copy of a Dirichlet node, in place (R^T R on copies). */
sem_status sem_mask(const sem_mesh* mesh, void* v, sem_prec prec, void* stream);

/* dinv = inverse of the assembled diagonal of A(k) = R Q^T A_L(k) Q R^T at
 * every local copy (0 at Dirichlet nodes): the Jacobi preconditioner.
 * k: DEVICE double [E][P] or NULL; dinv: DEVICE double [E][P]. */
sem_status sem_jacobi_inverse(const sem_mesh* mesh, const double* k, double h2, double* dinv,
                              void* stream);

/* z = p_m(S A) S r: the fourth-kind Chebyshev preconditioner of order m for
 * the assembled operator, S = Jacobi (Sec. 2.2 names this acceleration;
 * recurrence of Lottes 2022).  r, z: DEVICE double [E][P] copy-consistent
 * (values at Dirichlet copies ignored / returned 0).  lmax > 0 is the bound
 * rho_hat.  prec: SEM_FP64 (internal vectors and operator in double) or
 * SEM_FP32 / SEM_BF16_MFMA / SEM_FP16_MFMA (float vectors; the operator's
 * contractions per that precision).  Stream-ordered. */
sem_status sem_cheb_apply(const sem_mesh* mesh, const double* r, double* z, const double* k,
                          double h2, int32_t order, double lmax, sem_prec prec, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation, arguments, result and errors as sem_cheb_apply, with every work
 * vector in one fixed library-owned device array instead of the mesh's
 * lazily allocated work space.  No device memory is allocated or freed, and
 * nothing is read back to the host: the call only enqueues kernels on
 * `stream`.  The array holds 64 MiB (67108864 bytes) on every device the
 * call runs on, from the first call for a mesh of that device until the
 * process ends.  A call needs, with each part rounded up to 256 bytes,
 *   prec SEM_FP64:  8 n_local + 40 n_free bytes,
 *   otherwise:      8 n_local + 36 n_free (+ 4 n_local when k != NULL) bytes
 * (n_local = E (N+1)^3, n_free from sem_get_info; each at least 1) and returns
 * SEM_EINVAL, with nothing written, when that exceeds the array.  The Jacobi
 * inverse is formed again on every call.  All calls on one device share the
 * array: calls ordered on one stream are safe, calls that overlap in time on
 * one device (several streams or host threads) race and give wrong results. */
sem_status sem_cheb_apply_noalloc(const sem_mesh* mesh, const double* r, double* z,
                                  const double* k, double h2, int32_t order, double lmax,
                                  sem_prec prec, void* stream);

/* *lmax = largest eigenvalue estimate of D^-1 A from `steps` Jacobi-CG
 * iterations (CG-Lanczos tridiagonal), started from a fixed pseudo-random
 * vector.  Blocks.  SEM_EINVAL for a mesh with no free node. */
sem_status sem_lmax_estimate(const sem_mesh* mesh, const double* k, double h2, int32_t steps,
                             double* lmax, void* stream);

/* Solve A(k) x = b with A = R Q^T A_L(k) Q R^T (the pressure-Poisson /
 * Helmholtz solve of Sec. 2.2).  b, x: DEVICE double [E][P] copy-consistent
 * (b is read as the mean of its copies; Dirichlet entries ignored); x holds
 * x0 on entry (NULL-free: pass zeros for x0 = 0) and the copy-consistent
 * solution on return (0 at Dirichlet nodes).  With no Dirichlet node and
 * h2 = 0 the constant mode is removed from b and from x (zero mean over the
 * unique nodes), and every residual update subtracts the mean of A p, so
 * the residual stays free of it.  k: DEVICE double [E][P] or NULL.  Blocks the host (it reads
 * residual norms).  stats may be NULL.  Returns SEM_ENOCONV / SEM_EBREAKDOWN
 * with x = last iterate and stats filled.  A mesh with no free node (every
 * node Dirichlet) returns SEM_OK at once with x = 0 and 0 iterations. */
sem_status sem_pcg_solve(const sem_mesh* mesh, const double* b, double* x, const double* k,
                         double h2, const sem_solve_opts* opts, sem_solve_stats* stats,
                         void* stream);

/* Backward of the solve x = A(k)^-1 b of sem_pcg_solve (the pressure /
 * Helmholtz solve of Sec. 2.2) for a cotangent xbar of its copy-consistent
 * local output x.  With lambda the solution of the adjoint system
 * A(k) lambda = R Q^T xbar (A is symmetric: the same solve, run with `opts`
 * from zero; with no Dirichlet node and h2 = 0 the constant mode is removed
 * from the adjoint right-hand side and from lambda, as in the forward solve):
 *   kbar_q = dL/dk_q = -sum_ab (D_a lambda_L)_q G_ab,q (D_b x)_q   if kbar != NULL
 *   bbar_q = dL/db_q = lambda_L,q / (copies of q's node)          if bbar != NULL
 * (lambda_L = lambda at every local copy, 0 at Dirichlet copies; the second
 * line is the transpose of reading b as the mean of its copies).  x: the
 * forward solution (DEVICE double [E][P], needed for kbar, else nullable);
 * xbar, kbar, bbar: DEVICE double [E][P]; kbar and bbar must not alias x or
 * each other; k, h2 as in the forward solve.  At least one of kbar, bbar.
 * Blocks like sem_pcg_solve; stats (nullable) describe the adjoint solve.
 * SEM_ENOCONV / SEM_EBREAKDOWN: the outputs are formed from the last
 * adjoint iterate. */
sem_status sem_solve_backward(const sem_mesh* mesh, const double* x, const double* xbar,
                              const double* k, double h2, const sem_solve_opts* opts,
                              double* kbar, double* bbar, sem_solve_stats* stats, void* stream);

/* Backward of w = A_L(k) u for a cotangent wbar (all DEVICE double [E][P]):
 *   ubar = A_L(k) wbar                (A_L is symmetric)           if ubar != NULL
 *   kbar_q = sum_ab (D_a wbar)_q G_ab,q (D_b u)_q                   if kbar != NULL
 * so that <wbar, A_L(dk) u> = <kbar, dk>.  Stream-ordered. */
sem_status sem_ax_backward(const sem_mesh* mesh, const double* u, const double* wbar,
                           const double* k, double h2, double* ubar, double* kbar, void* stream);

/* ---------------------------------------------------------- p-multigrid
 * Levels of polynomial order N_0 = N > N_1 > ... > N_L on the same hexahedra
 * (default N, floor(N/2), ..., 1).  Level l >= 1 is a mesh of its own: its
 * element maps interpolate the fine ones at the order-N_l GLL points and its
 * unknowns are identified through the fine global ids (a coarse node is a
 * mesh vertex, a position on a mesh edge or face, or an element-interior
 * position), so every level has the spectral-element operator of its order.
 * One V-cycle: pre-smoothing x = C_l(r), coarse correction
 * x += P_l V_{l+1}(P_l^T (r - A_l x)), post-smoothing x += C_l(r - A_l x),
 * with C_l the fourth-kind Chebyshev polynomial of order smooth_order in
 * S_l A_l (S_l the smoother below: Jacobi or overlapping Schwarz; bound
 * 1.1 x a 20-step Lanczos estimate per level, per solve), P_l the
 * element-wise tensor-product Lagrange interpolation (averaged over the copies
 * of a fine node), P_l^T its transpose, and coarse_iters Jacobi-PCG
 * iterations from zero on the coarsest level (constant mode projected out on
 * a singular level).  Sec. 2.2 names this preconditioner: p-multigrid with
 * Chebyshev-accelerated overlapping Schwarz smoothing. */
#define SEM_PMG_MAX_LEVELS 8
typedef struct {
  int32_t n_levels;                    /* 0: default orders; else the number of entries used */
  int32_t orders[SEM_PMG_MAX_LEVELS];  /* strictly decreasing, orders[0] = N, all >= 1 */
  int32_t smooth_order;                /* Chebyshev order m >= 1 (m-1 applies per smoothing) */
  int32_t coarse_iters;                /* Jacobi-PCG iterations on the coarsest level, >= 1 */
  int32_t smoother;                    /* SEM_SMOOTH_JACOBI or SEM_SMOOTH_SCHWARZ */
} sem_pmg_opts;

/* The operator S the Chebyshev smoothing of a level accelerates.
 * SEM_SMOOTH_SCHWARZ: additive overlapping Schwarz, Sec. 2.2's smoother.  The
 * subdomain of an element is its nodes plus, across each face, the
 * neighbour's node layer one GLL step inside; the local problem on that
 * (N+3)^3 box is the separable approximation built from three 1-D GLL
 * elements (the element and its two neighbours along each direction, at
 * their mean lengths), solved exactly by fast diagonalisation; the box's
 * edge and corner points are left out.  The local operator is that of the
 * constant-coefficient Laplacian whatever k and h2 (the Chebyshev bound, a
 * Lanczos estimate of the Schwarz-preconditioned operator, absorbs the
 * scale). */
typedef enum { SEM_SMOOTH_JACOBI = 0, SEM_SMOOTH_SCHWARZ = 1 } sem_smoother;

/* Defaults: n_levels 0, smooth_order 4, coarse_iters 30, Schwarz smoother
 * (fastest to a 1e-10 residual of the settings measured on the benchmark
 * meshes, within 10 % on both). */
void sem_pmg_opts_default(sem_pmg_opts* opts);

/* Build (or rebuild) the hierarchy of `mesh` from the description it was set
 * up with (same N and E; HOST arrays, read during the call only).  The coarse
 * meshes are owned by `mesh` and freed with it.  Blocks.  SEM_EINVAL for bad
 * options, a different description, or a mesh whose edge or face has corners
 * sharing a global id (one element across a periodic direction). */
sem_status sem_setup_pmg(sem_mesh* mesh, const sem_mesh_desc* desc, const sem_pmg_opts* opts,
                         void* stream);

/* Level orders (HOST int32[SEM_PMG_MAX_LEVELS], nullable) and the Chebyshev
 * bounds of the last solve or apply (HOST double[SEM_PMG_MAX_LEVELS],
 * nullable; 0 before the first). */
sem_status sem_pmg_info(const sem_mesh* mesh, int32_t* n_levels, int32_t* orders,
                        double* rho_hat);

/* z = V(r): one V-cycle for A(k) (+ h2 B).  r, z: DEVICE double [E][P]
 * copy-consistent (values at Dirichlet copies ignored / returned 0); k DEVICE
 * double [E][P] or NULL.  prec: SEM_FP64 or SEM_FP32 (arithmetic of the
 * cycle).  Blocks on the first call for given k, h2 (level bounds).  With no
 * free node z = 0. */
sem_status sem_pmg_apply(const sem_mesh* mesh, const double* r, double* z, const double* k,
                         double h2, sem_prec prec, void* stream);

/* HOST-only.  The Schwarz subdomains sem_setup_pmg builds for an order-N
 * mesh (1 <= N <= 10; same validation as sem_setup_mesh), with the free
 * numbering of sem_host_numbering: xmap [E][(N+3)^3] receives the free index
 * of each box point or -1; S [E][3][(N+3)^2] (row-major per direction r, s,
 * t) and lam [E][3][N+3] the fast-diagonalisation factors (nullable). */
sem_status sem_host_schwarz(int32_t N, int64_t E, const int64_t* gid, const uint8_t* dirichlet,
                            const double* xyz, int32_t* xmap, double* S, double* lam);

/* HOST-only.  The order-Nc mesh sem_setup_pmg builds from an order-N one
 * (2 <= N <= 10, 1 <= Nc < N): xyz_c [E][Pc][3] (nullable together with
 * xyz), gid_c [E][Pc] (ids 0.., numbered per coarse node), dirichlet_c
 * [E][Pc] (NULL together with dirichlet), all caller-allocated. */
sem_status sem_host_coarse_mesh(int32_t N, int64_t E, const int64_t* gid,
                                const uint8_t* dirichlet, const double* xyz, int32_t Nc,
                                int64_t* gid_c, uint8_t* dirichlet_c, double* xyz_c);

/* ------------------------------------------------------ convective term
 * The advection term u . grad f of the Boussinesq equations (Sec. 4.1: the
 * temperature and each velocity component are advected by the velocity), in
 * weak form per element:
 *   C_e(u) f |_i = sum_q phi_i(x_q) w_q detJ_q u(x_q) . grad f(x_q),
 * with u and f interpolated from the element's GLL nodes.  The paper prints
 * no discretisation of this term; two quadratures are offered:
 *   SEM_ADV_COLLOCATION  the GLL nodes themselves (N+1 per direction;
 *                        aliased: the integrand has degree 3N - 1 per
 *                        direction, the rule is exact to 2N - 1);
 *   SEM_ADV_DEALIAS      M = floor(3(N+1)/2) Gauss-Legendre points per
 *                        direction (over-integration by the 3/2 rule, exact
 *                        on affine elements).
 * The nine factors w detJ dr_a/dx_d per point are precomputed by
 * sem_setup_advection. */
typedef enum { SEM_ADV_COLLOCATION = 0, SEM_ADV_DEALIAS = 1 } sem_adv_rule;

/* HOST-only.  The rule's points per direction (q1, nullable), points x and
 * weights w on [-1, 1] (ascending, q1 each, nullable) and the interpolation
 * J [q1][N+1] (row-major, nullable) from the GLL nodes to them (the identity
 * for collocation).  1 <= N <= 10. */
sem_status sem_advection_rule(int32_t N, int32_t rule, int32_t* q1, double* x, double* w,
                              double* J);

/* Compute the factors of `rule` for `mesh` from the description it was set
 * up with (same N and E; HOST arrays, read during the call only).  Device
 * memory: 9 q1^3 E values in FP64 and FP32.  Blocks.  SEM_EINVAL for a
 * different description, an unknown rule or detJ <= 0 at a point. */
sem_status sem_setup_advection(sem_mesh* mesh, const sem_mesh_desc* desc, int32_t rule,
                               void* stream);

/* Copy the factors of `rule` to G: DEVICE double [E][9][q1^3], slot 3 a + d
 * holding w detJ dr_a/dx_d (a = r, s, t; d = x, y, z), points in [k][j][i]
 * order.  Stream-ordered. */
sem_status sem_get_advection_factors(const sem_mesh* mesh, int32_t rule, double* G,
                                     void* stream);

/* out = C_L(u) f: every element's contribution (unassembled; sem_gs sums
 * them).  u: DEVICE [3][E][P] (x, y and z components of the velocity at the
 * local nodes), f, out: DEVICE [E][P]; double (SEM_FP64) or float (SEM_FP32:
 * FP32 factors and arithmetic).  out must not overlap u or f.
 * Stream-ordered. */
sem_status sem_advect(const sem_mesh* mesh, int32_t rule, const void* u, const void* f,
                      void* out, sem_prec prec, void* stream);

/* out[k] = C_L(u) f[k] for nf >= 0 fields advected by one velocity (the
 * temperature and the three velocity components of a Boussinesq step): f,
 * out DEVICE [nf][E][P], the rest as sem_advect.  The velocity and the
 * factors are read once per element for all fields; each out[k] equals
 * sem_advect's for f[k].  nf = 0 does nothing.  Stream-ordered. */
sem_status sem_advect_fields(const sem_mesh* mesh, int32_t rule, const void* u, int32_t nf,
                             const void* f, void* out, sem_prec prec, void* stream);

/* Environment variables (read once per process; for comparisons, not needed
 * in normal use):
 *   SEM_AX_KERNEL=scalar|mfma   force the thread-per-point or the matrix-core
 *                               element operator (default: matrix cores from
 *                               N = 5 on);
 *   SEM_AX_SPLIT=0              inside sem_pcg_solve, keep the gather form of
 *                               the operator followed by a segmented sum over
 *                               all free nodes (default from N = 5: single-copy
 *                               nodes written by the operator directly);
 *   SEM_GRAPH_MAX_FREE=n        largest solve (free nodes) that replays
 *                               captured iteration graphs (default 262144);
 *   SEM_AX_NT_BYTES=n           read at sem_setup_mesh: inside sem_pcg_solve
 *                               the operator stores shared-copy results with
 *                               nontemporal stores when the local array
 *                               (E (N+1)^3 values) is larger than n bytes
 *                               (default 134217728; 0 = always). */

/* Thread-local description of the last non-OK status ("" if none). */
const char* sem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SEM_H */
