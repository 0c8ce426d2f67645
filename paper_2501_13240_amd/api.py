"""Python binding of libsem (same names as the C ABI in include/sem.h).

PyTorch supplies device memory (tensors) and the stream (torch's current HIP
stream); every step of the computation runs in libsem's HIP kernels.  Local
vectors are CUDA tensors of shape (E, (N+1)^3) (or any shape with that many
elements), float64 unless a precision says otherwise.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L


class SemError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        self.name = L.STATUS_NAMES.get(status, str(status))
        super().__init__(f"{where}: {self.name}: {message}")


def _check(status: int, where: str):
    if status != L.SEM_OK:
        msg = L.load().sem_last_error().decode(errors="replace")
        raise SemError(status, where, msg)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def gll(N: int):
    """GLL nodes, weights and derivative matrix computed by the library (host)."""
    lib = L.load()
    xi, rho, D = np.zeros(N + 1), np.zeros(N + 1), np.zeros((N + 1) * (N + 1))
    _check(lib.sem_gll(N, _np_ptr(xi), _np_ptr(rho), _np_ptr(D)), "sem_gll")
    return xi, rho, D.reshape(N + 1, N + 1)


def host_numbering(N: int, gid: np.ndarray, dirichlet: np.ndarray | None = None):
    """The library's free-node numbering (host only)."""
    lib = L.load()
    gid = np.ascontiguousarray(gid, dtype=np.int64)
    E = gid.shape[0]
    d = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8)
    fi = np.empty(gid.size, dtype=np.int32)
    nu, nf, ns = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib.sem_host_numbering(N, E, _np_ptr(gid), _np_ptr(d), _np_ptr(fi), ctypes.byref(nu),
                                  ctypes.byref(nf), ctypes.byref(ns)), "sem_host_numbering")
    return fi.reshape(gid.shape), nu.value, nf.value, ns.value


class Mesh:
    """A mesh handle on the current HIP device (sem_setup_mesh)."""

    def __init__(self, xyz: np.ndarray, gid: np.ndarray, dirichlet: np.ndarray | None, N: int):
        self._lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("libsem needs a HIP device")
        self.N = int(N)
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        gid = np.ascontiguousarray(gid, dtype=np.int64)
        self.E = gid.shape[0]
        self.P = (self.N + 1) ** 3
        if gid.size != self.E * self.P or xyz.size != 3 * gid.size:
            raise ValueError("xyz must be (E, P, 3) and gid (E, P) with P = (N+1)^3")
        d = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8)
        # kept for a later sem_setup_pmg (it re-reads the description)
        self._desc_arrays = (xyz, gid, d)
        self._pmg = False
        self._adv = set()
        desc = L.MeshDesc(self.N, self.E, _np_ptr(xyz), _np_ptr(gid), _np_ptr(d))
        h = ctypes.c_void_p()
        self.device = torch.cuda.current_device()
        _check(self._lib.sem_setup_mesh(ctypes.byref(desc), _stream(), ctypes.byref(h)),
               "sem_setup_mesh")
        self._h = h
        info = L.MeshInfo()
        _check(self._lib.sem_get_info(self._h, ctypes.byref(info)), "sem_get_info")
        self.info = {f: getattr(info, f) for f, _ in L.MeshInfo._fields_}
        self._mult = None

    @property
    def handle(self):
        return self._h

    def setup_pmg(self, orders=None, smooth_order: int = 4, coarse_iters: int = 30,
                  smoother: str = "schwarz"):
        """Build the p-multigrid hierarchy (sem_setup_pmg); orders default to
        N, N//2, ..., 1; smoother 'jacobi' or 'schwarz'."""
        opts = L.PmgOpts()
        self._lib.sem_pmg_opts_default(ctypes.byref(opts))
        if orders is not None:
            orders = [int(o) for o in orders]
            opts.n_levels = len(orders)
            for i, o in enumerate(orders):
                opts.orders[i] = o
        opts.smooth_order = int(smooth_order)
        opts.coarse_iters = int(coarse_iters)
        opts.smoother = L.SMOOTHER[smoother]
        xyz, gid, d = self._desc_arrays
        desc = L.MeshDesc(self.N, self.E, _np_ptr(xyz), _np_ptr(gid), _np_ptr(d))
        _check(self._lib.sem_setup_pmg(self._h, ctypes.byref(desc), ctypes.byref(opts), _stream()),
               "sem_setup_pmg")
        self._pmg = True

    def pmg_info(self):
        """(level orders, Chebyshev bounds of the last solve or apply)."""
        n = ctypes.c_int32()
        orders = (ctypes.c_int32 * L.PMG_MAX_LEVELS)()
        rho = (ctypes.c_double * L.PMG_MAX_LEVELS)()
        _check(self._lib.sem_pmg_info(self._h, ctypes.byref(n), orders, rho), "sem_pmg_info")
        return list(orders[:n.value]), list(rho[:n.value])

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.sem_free_mesh(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def zeros(self, dtype=torch.float64):
        return torch.zeros(self.E, self.P, dtype=dtype, device=f"cuda:{self.device}")

    def check_local(self, t, dtype=torch.float64, name="vector"):
        if t is None:
            return None
        if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()
                and t.numel() == self.E * self.P):
            raise ValueError(f"{name} must be a contiguous CUDA {dtype} tensor with "
                             f"E*(N+1)^3 = {self.E * self.P} elements")
        return t

    def multiplicity(self):
        """Copies of each local point's global node (Q Q^T 1), float64 local."""
        if self._mult is None:
            m = torch.ones(self.E, self.P, dtype=torch.float64, device=f"cuda:{self.device}")
            self._mult = gs(self, m)
        return self._mult

    def setup_advection(self, rule: str = "dealias"):
        """Precompute the convective term's factors for `rule` ('dealias':
        the 3/2 Gauss rule, 'collocation': the GLL nodes)."""
        xyz, _, _ = self._desc_arrays
        desc = L.MeshDesc(self.N, self.E, _np_ptr(xyz), None, None)
        _check(self._lib.sem_setup_advection(self._h, ctypes.byref(desc), L.ADV_RULE[rule],
                                             _stream()), "sem_setup_advection")
        self._adv.add(rule)

    def advection_factors(self, rule: str = "dealias"):
        """(E, 9, q1^3) float64: w detJ dr_a/dx_d in slot 3 a + d."""
        q1 = advection_rule(self.N, rule)[0].size
        G = torch.empty(self.E, 9, q1 ** 3, dtype=torch.float64, device=f"cuda:{self.device}")
        _check(self._lib.sem_get_advection_factors(self._h, L.ADV_RULE[rule], _ptr(G), _stream()),
               "sem_get_advection_factors")
        return G

    def geometry(self):
        G = torch.empty(self.E, 6, self.P, dtype=torch.float64, device=f"cuda:{self.device}")
        B = self.zeros()
        _check(self._lib.sem_get_geometry(self._h, _ptr(G), _ptr(B), _stream()), "sem_get_geometry")
        return G, B


def _prec_of(t):
    return L.PREC["fp64"] if t.dtype == torch.float64 else L.PREC["fp32"]


def ax(mesh: Mesh, u, k=None, h2: float = 0.0, out=None, prec: str | None = None):
    """w = A_L(k) u on every element (sem_ax).  prec: None (from u's dtype),
    or 'bf16_mfma' / 'fp16_mfma' for float32 u (16-bit contraction operands)."""
    mesh.check_local(u, u.dtype, "u")
    if k is not None:
        mesh.check_local(k, u.dtype, "k")
    if prec is None:
        code = _prec_of(u)
    else:
        code = L.PREC[prec]
        want = torch.float64 if prec == "fp64" else torch.float32
        if u.dtype != want:
            raise TypeError(f"precision {prec} takes {want} data, got {u.dtype}")
    w = torch.empty_like(u) if out is None else mesh.check_local(out, u.dtype, "out")
    _check(mesh._lib.sem_ax(mesh.handle, _ptr(u), _ptr(w), _ptr(k), float(h2), code,
                            _stream()), "sem_ax")
    return w


def mass(mesh: Mesh, u, out=None):
    mesh.check_local(u, u.dtype, "u")
    w = torch.empty_like(u) if out is None else out
    _check(mesh._lib.sem_mass(mesh.handle, _ptr(u), _ptr(w), _prec_of(u), _stream()), "sem_mass")
    return w


def gs(mesh: Mesh, v):
    """In place v <- Q Q^T v (sem_gs); returns v."""
    mesh.check_local(v, v.dtype, "v")
    _check(mesh._lib.sem_gs(mesh.handle, _ptr(v), _prec_of(v), _stream()), "sem_gs")
    return v


def mask(mesh: Mesh, v):
    mesh.check_local(v, v.dtype, "v")
    _check(mesh._lib.sem_mask(mesh.handle, _ptr(v), _prec_of(v), _stream()), "sem_mask")
    return v


def jacobi_inverse(mesh: Mesh, k=None, h2: float = 0.0):
    mesh.check_local(k, torch.float64, "k")
    d = mesh.zeros()
    _check(mesh._lib.sem_jacobi_inverse(mesh.handle, _ptr(k), float(h2), _ptr(d), _stream()),
           "sem_jacobi_inverse")
    return d


def cheb_apply(mesh: Mesh, r, lmax: float, k=None, h2: float = 0.0, order: int = 3,
               prec: str = "fp64"):
    mesh.check_local(r, torch.float64, "r")
    mesh.check_local(k, torch.float64, "k")
    z = torch.empty_like(r)
    _check(mesh._lib.sem_cheb_apply(mesh.handle, _ptr(r), _ptr(z), _ptr(k), float(h2), int(order),
                                    float(lmax), L.PREC[prec], _stream()), "sem_cheb_apply")
    return z


def cheb_apply_noalloc(mesh: Mesh, r, lmax: float, k=None, h2: float = 0.0, order: int = 3,
                       prec: str = "fp64", out=None):
    """cheb_apply through sem_cheb_apply_noalloc (work space in the library's
    fixed device array; `out`, when given, receives z)."""
    mesh.check_local(r, torch.float64, "r")
    mesh.check_local(k, torch.float64, "k")
    z = torch.empty_like(r) if out is None else out
    mesh.check_local(z, torch.float64, "out")
    _check(mesh._lib.sem_cheb_apply_noalloc(mesh.handle, _ptr(r), _ptr(z), _ptr(k), float(h2),
                                            int(order), float(lmax), L.PREC[prec], _stream()),
           "sem_cheb_apply_noalloc")
    return z


def pmg_apply(mesh: Mesh, r, k=None, h2: float = 0.0, prec: str = "fp32"):
    """z = V(r), one p-multigrid V-cycle (sem_pmg_apply); sets up the default
    hierarchy on first use."""
    mesh.check_local(r, torch.float64, "r")
    mesh.check_local(k, torch.float64, "k")
    if not mesh._pmg:
        mesh.setup_pmg()
    z = torch.empty_like(r)
    _check(mesh._lib.sem_pmg_apply(mesh.handle, _ptr(r), _ptr(z), _ptr(k), float(h2),
                                   L.PREC[prec], _stream()), "sem_pmg_apply")
    return z


def advection_rule(N: int, rule: str = "dealias"):
    """(points, weights, J) of the convective term's rule (host): J
    interpolates from the GLL nodes to the points."""
    lib = L.load()
    q1 = ctypes.c_int32()
    _check(lib.sem_advection_rule(N, L.ADV_RULE[rule], ctypes.byref(q1), None, None, None),
           "sem_advection_rule")
    x, w, J = np.zeros(q1.value), np.zeros(q1.value), np.zeros((q1.value, N + 1))
    _check(lib.sem_advection_rule(N, L.ADV_RULE[rule], None, _np_ptr(x), _np_ptr(w), _np_ptr(J)),
           "sem_advection_rule")
    return x, w, J


def advect(mesh: Mesh, u, f, rule: str = "dealias", out=None):
    """out = C_L(u) f, the unassembled convective term: u (3, E, P) and f
    (E, P) for one field (sem_advect) or (nf, E, P) for nf fields advected by
    the same velocity (sem_advect_fields), one dtype (float64 or float32);
    sets up the rule's factors on first use."""
    dt = f.dtype
    shape = (mesh.E, mesh.P)
    if not (f.is_cuda and f.is_contiguous() and tuple(f.shape[-2:]) == shape
            and f.dim() in (2, 3)):
        raise ValueError(f"f must be a contiguous CUDA tensor of shape (E, P) or (nf, E, P)")
    if not (u.is_cuda and u.dtype == dt and u.is_contiguous()
            and tuple(u.shape) == (3,) + shape):
        raise ValueError(f"u must be a contiguous CUDA {dt} tensor of shape (3, E, P)")
    if dt not in (torch.float64, torch.float32):
        raise TypeError("advect takes float64 or float32 data")
    if rule not in mesh._adv:
        mesh.setup_advection(rule)
    if out is None:
        w = torch.empty_like(f)
    else:
        if not (out.is_cuda and out.dtype == dt and out.is_contiguous() and out.shape == f.shape):
            raise ValueError("out must be a contiguous CUDA tensor like f")
        w = out
    nf = 1 if f.dim() == 2 else f.shape[0]
    _check(mesh._lib.sem_advect_fields(mesh.handle, L.ADV_RULE[rule], _ptr(u), nf, _ptr(f),
                                       _ptr(w), _prec_of(f), _stream()), "sem_advect_fields")
    return w


def host_coarse_mesh(N: int, gid: np.ndarray, dirichlet, xyz, Nc: int):
    """The library's order-Nc mesh on the hexahedra of an order-N mesh (host)."""
    lib = L.load()
    gid = np.ascontiguousarray(gid, dtype=np.int64)
    E = gid.shape[0]
    Pc = (Nc + 1) ** 3
    d = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8)
    x = None if xyz is None else np.ascontiguousarray(xyz, dtype=np.float64)
    gid_c = np.empty((E, Pc), dtype=np.int64)
    d_c = None if d is None else np.empty((E, Pc), dtype=np.uint8)
    x_c = None if x is None else np.empty((E, Pc, 3), dtype=np.float64)
    _check(lib.sem_host_coarse_mesh(N, E, _np_ptr(gid), _np_ptr(d), _np_ptr(x), Nc,
                                    _np_ptr(gid_c), _np_ptr(d_c), _np_ptr(x_c)),
           "sem_host_coarse_mesh")
    return x_c, gid_c, d_c


def host_schwarz(N: int, gid: np.ndarray, dirichlet, xyz):
    """The library's Schwarz subdomain map and fast-diagonalisation factors
    (host): xmap (E, (N+3)^3), S (E, 3, N+3, N+3), lam (E, 3, N+3)."""
    lib = L.load()
    gid = np.ascontiguousarray(gid, dtype=np.int64)
    E = gid.shape[0]
    nx = N + 3
    d = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8)
    x = np.ascontiguousarray(xyz, dtype=np.float64)
    xmap = np.empty((E, nx ** 3), dtype=np.int32)
    S = np.empty((E, 3, nx, nx))
    lam = np.empty((E, 3, nx))
    _check(lib.sem_host_schwarz(N, E, _np_ptr(gid), _np_ptr(d), _np_ptr(x), _np_ptr(xmap),
                                _np_ptr(S), _np_ptr(lam)), "sem_host_schwarz")
    return xmap, S, lam


def lmax_estimate(mesh: Mesh, k=None, h2: float = 0.0, steps: int = 20) -> float:
    mesh.check_local(k, torch.float64, "k")
    out = ctypes.c_double()
    _check(mesh._lib.sem_lmax_estimate(mesh.handle, _ptr(k), float(h2), int(steps),
                                       ctypes.byref(out), _stream()), "sem_lmax_estimate")
    return out.value


def _solve_opts(mesh, mode, precond, precond_prec, cheb_order, lmax, rtol, max_iter,
                fixed_iters, inner_rtol, max_outer, check_every, profile, history):
    """sem_solve_opts from keyword arguments (and the residual-history buffer)."""
    if precond_prec is None:  # the multigrid cycle and the inner solve of refinement: FP32
        precond_prec = "fp32" if (precond == "pmg" or mode == "mixed_ir") else "fp64"
    if precond == "pmg" and not mesh._pmg:
        mesh.setup_pmg()
    opts = L.SolveOpts()
    mesh._lib.sem_solve_opts_default(ctypes.byref(opts))
    opts.mode = L.MODE[mode]
    opts.precond = L.PRECOND[precond]
    opts.precond_prec = L.PREC[precond_prec]
    opts.cheb_order = int(cheb_order)
    opts.lmax = float(lmax)
    opts.rtol = float(rtol)
    opts.max_iter = int(max_iter)
    opts.fixed_iters = 1 if fixed_iters else 0
    opts.inner_rtol = float(inner_rtol)
    opts.max_outer = int(max_outer)
    opts.check_every = int(check_every)
    opts.profile = 1 if profile else 0
    hist = None
    if history:
        hist = np.zeros(max_iter + 1)
        opts.residual_history = _np_ptr(hist)
    return opts, hist


def _stats_dict(st, status, hist):
    stats = {f: getattr(st, f) for f, _ in L.SolveStats._fields_ if f != "pad_"}
    stats["status"] = L.STATUS_NAMES.get(status, str(status))
    if hist is not None:
        stats["history"] = hist[: (stats["iters"] + 1)]
    return stats


def solve(mesh: Mesh, b, x0=None, k=None, h2: float = 0.0, *, mode: str = "cg",
          precond: str = "jacobi", precond_prec: str | None = None, cheb_order: int = 3,
          lmax: float = 0.0, rtol: float = 1e-10, max_iter: int = 10000,
          fixed_iters: bool = False, inner_rtol: float = 1e-5, max_outer: int = 30,
          check_every: int = 0, profile: bool = False, history: bool = False,
          raise_on_noconv: bool = True, out=None):
    """Solve A(k) x = b (sem_pcg_solve).  Returns (x, stats dict)."""
    mesh.check_local(b, torch.float64, "b")
    mesh.check_local(k, torch.float64, "k")
    if out is None:
        x = torch.zeros_like(b) if x0 is None else x0.clone()
    else:
        x = mesh.check_local(out, torch.float64, "out")
        if x0 is None:
            x.zero_()
        else:
            x.copy_(x0)
    opts, hist = _solve_opts(mesh, mode, precond, precond_prec, cheb_order, lmax, rtol, max_iter,
                             fixed_iters, inner_rtol, max_outer, check_every, profile, history)
    st = L.SolveStats()
    status = mesh._lib.sem_pcg_solve(mesh.handle, _ptr(b), _ptr(x), _ptr(k), float(h2),
                                     ctypes.byref(opts), ctypes.byref(st), _stream())
    stats = _stats_dict(st, status, hist)
    if status == L.SEM_ENOCONV and not raise_on_noconv:
        return x, stats
    _check(status, "sem_pcg_solve")
    return x, stats


def solve_backward(mesh: Mesh, x, xbar, k=None, h2: float = 0.0, *, need_kbar: bool = True,
                   need_bbar: bool = True, mode: str = "cg", precond: str = "jacobi",
                   precond_prec: str | None = None, cheb_order: int = 3, lmax: float = 0.0,
                   rtol: float = 1e-10, max_iter: int = 10000, inner_rtol: float = 1e-5,
                   max_outer: int = 30, check_every: int = 0):
    """(kbar, bbar, stats): the gradients dL/dk and dL/db of the solve
    x = A(k)^-1 b for the cotangent xbar = dL/dx (sem_solve_backward; the
    adjoint solve takes the same options as sem_pcg_solve)."""
    mesh.check_local(x, torch.float64, "x")
    mesh.check_local(xbar, torch.float64, "xbar")
    mesh.check_local(k, torch.float64, "k")
    if not (need_kbar or need_bbar):
        raise ValueError("nothing to compute: need_kbar and need_bbar are both False")
    kbar = torch.empty_like(xbar) if need_kbar else None
    bbar = torch.empty_like(xbar) if need_bbar else None
    opts, hist = _solve_opts(mesh, mode, precond, precond_prec, cheb_order, lmax, rtol, max_iter,
                             False, inner_rtol, max_outer, check_every, False, False)
    st = L.SolveStats()
    status = mesh._lib.sem_solve_backward(mesh.handle, _ptr(x), _ptr(xbar), _ptr(k), float(h2),
                                          ctypes.byref(opts), _ptr(kbar), _ptr(bbar),
                                          ctypes.byref(st), _stream())
    _check(status, "sem_solve_backward")
    return kbar, bbar, _stats_dict(st, status, hist)


def ax_backward(mesh: Mesh, u, wbar, k=None, h2: float = 0.0, need_ubar: bool = True,
                need_kbar: bool = True):
    """(ubar, kbar) of w = A_L(k) u for the cotangent wbar (sem_ax_backward)."""
    mesh.check_local(u, torch.float64, "u")
    mesh.check_local(wbar, torch.float64, "wbar")
    mesh.check_local(k, torch.float64, "k")
    ubar = torch.empty_like(u) if need_ubar else None
    kbar = torch.empty_like(u) if need_kbar else None
    _check(mesh._lib.sem_ax_backward(mesh.handle, _ptr(u), _ptr(wbar), _ptr(k), float(h2),
                                     _ptr(ubar), _ptr(kbar), _stream()), "sem_ax_backward")
    return ubar, kbar
