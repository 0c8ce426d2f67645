"""Benchmark: FP64 Jacobi-PCG on one GPU's share of the convection box.

Workload: [0,4]x[0,4]x[0,1], 32x32x16 hexahedra at N = 7 (5,669,888 unique
nodes, 8,388,608 local points), periodic in x and y, Dirichlet plates,
tanh clustering to both plates (largest/smallest layer 20), smooth seeded
deformation, random normal right-hand side.  One step = one solve of exactly
100 Jacobi-PCG iterations (operator apply + gather-scatter + fused vector
updates and reductions), inputs resident in device memory.

value = unique DOF x iterations / second of the timed steps (GDOF/s).
roofline: the element-operator kernel (the dominant kernel), 64 algorithmic
bytes per local point (u, six geometric factors, w in FP64) per launch,
divided by its average duration measured with HIP events on the solve's
stream inside the timed region: each operator launch of the last timed step
is made with a start and a stop event that the runtime stamps with the
kernel's own start and end (the other steps run without events).
CPU leg (after every GPU measurement): cpu_baseline, the CPU oracle's PCG
iteration on a 32x8x16-element sample of the same recipe timed on this host;
and the error of every solve result against the FP64 oracle: the GPU
solutions are copied to the host after their timed solves, and the oracle's
own operator gives their true residual ||b - A x|| / ||b|| (oracle_rel_res),
with ||x - x_FP64|| / ||x_FP64|| against the FP64 Jacobi-CG solution of the
same mesh (x_rel_diff_vs_fp64; on the 4^3 cubes against the oracle's own
solution, x_rel_diff_vs_oracle) and, for the gradient workload, the oracle's
residual of the adjoint solve and its k-gradient formed from the GPU's x and
adjoint solution.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=150)
    ap.add_argument("--ax-reps", type=int, default=50)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for counter calibration)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-vs-FP64 solve comparison on the 32^3, N=9 Neumann box")
    ap.add_argument("--mixed-variants", default="",
                    help="comma-separated subset of the mixed-vs-FP64 variants (default: all)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the small-case solves and the forward/backward timing")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


class OracleChecks:
    """GPU results kept on the host for the oracle's checks in the CPU leg:
    per mesh (workload number, order, shape) the right-hand side and the
    solution of every variant, and where each number goes in the JSON."""

    def __init__(self):
        self.meshes = {}

    def add(self, key, spec, b_local, name, x_local, target):
        ent = self.meshes.setdefault(key, dict(spec=spec, b=b_local, sols={}))
        ent["sols"][name] = (x_local, target)


CHECKS = OracleChecks()
GRAD_CHECK = {}


def cpu_baseline(iters):
    """The oracle as it stands: PCG iterations on a sample of the recipe."""
    import oracle
    from sem_inputs import config_mesh

    m, fld = config_mesh(2, shape=(32, 8, 16))
    P = oracle.Problem(m.xyz, m.gid, m.dirichlet, m.N)
    b = P.num.from_local_consistent(fld["b"])
    t0 = time.perf_counter()
    res = P.solve(b, rtol=1e-30, max_iter=iters, fixed_iters=True)
    dt = time.perf_counter() - t0
    gdofs = P.num.n * res["iters"] / dt / 1e9
    cpu = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return dict(value=gdofs, unit="GDOF/s", cores=1, kind="oracle",
                sample=(f"{res['iters']} Jacobi-PCG iterations of the NumPy oracle on a "
                        f"32x8x16-element slice of the same recipe ({P.num.n} unique nodes), "
                        f"{dt:.1f} s; its einsum/bincount kernels run on one thread "
                        f"({avail} cores available, {cpu})"),
                seconds=dt)


def oracle_errors(out):
    """The FP64 oracle's verdict on every GPU solve result (CPU, untimed):
    the true residual by the oracle's own assembled operator, the difference
    to the FP64 Jacobi-CG solution of the same mesh (or, on the small cubes,
    to the oracle's own solution at 1e-12), and for the gradient workload the
    adjoint solve's residual and the k-gradient formed by the oracle from the
    GPU's solution and adjoint solution."""
    import oracle
    from sem_inputs import config_mesh

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    for key, ent in CHECKS.meshes.items():
        spec = ent["spec"]
        t = time.time()
        m, fld = config_mesh(spec["cfg"], N=spec.get("N"))
        P = oracle.Problem(m.xyz, m.gid, m.dirichlet, m.N, k=fld["k"], h2=fld["h2"])
        if fld["f"] is not None:  # manufactured source: b = R Q^T (B f), f = 3 pi^2 u
            b = P.rhs_from_source(fld["f"] * 3 * np.pi ** 2)
        else:
            b = P.num.from_local_consistent(ent["b"])
        if P.neumann:
            b = b - b.mean()
        ref, ref_kind = None, None
        if spec["cfg"] == 1:
            ref, ref_kind = P.solve(b, rtol=1e-12)["x"], "x_rel_diff_vs_oracle"
        elif "fp64_jacobi_cg" in ent["sols"]:
            ref = P.num.from_local_consistent(ent["sols"]["fp64_jacobi_cg"][0])
            ref_kind = "x_rel_diff_vs_fp64"
        for name, (xl, target) in ent["sols"].items():
            xf = P.num.from_local_consistent(xl)
            target["oracle_rel_res"] = float(np.linalg.norm(b - P.apply(xf)) / np.linalg.norm(b))
            if ref is not None and not (ref_kind == "x_rel_diff_vs_fp64"
                                        and name == "fp64_jacobi_cg"):
                target[ref_kind] = rel(xf, ref)
        log(f"  {key}: {len(ent['sols'])} results checked in {time.time() - t:.1f}s")
        del P, m, fld
    if GRAD_CHECK:
        g = GRAD_CHECK
        m, fld = config_mesh(4)
        P = oracle.Problem(m.xyz, m.gid, m.dirichlet, m.N, k=fld["k"], h2=fld["h2"])
        b = P.rhs_from_source(fld["f"])
        xf = P.num.from_local_consistent(g["x"])
        lf = P.num.from_local_consistent(g["lam"])
        adj_b = P.num.R(P.num.Qt(g["xbar"]))
        kb = -oracle.kgrad_contraction(P.num.to_local(xf), P.num.to_local(lf), P.G, m.N)
        r = g["result"]
        r["oracle_rel_res_forward"] = float(np.linalg.norm(b - P.apply(xf)) / np.linalg.norm(b))
        r["oracle_rel_res_adjoint"] = float(np.linalg.norm(adj_b - P.apply(lf))
                                            / np.linalg.norm(adj_b))
        r["kbar_rel_diff_vs_oracle"] = rel(g["kbar"], kb)
        r["kbar_autograd_rel_diff_vs_oracle"] = rel(g["kbar_autograd"], kb)
        if "pmg_fp32" in r:
            xpf = P.num.from_local_consistent(g["x_pmg"])
            r["pmg_fp32"]["oracle_rel_res_forward"] = float(np.linalg.norm(b - P.apply(xpf))
                                                            / np.linalg.norm(b))
            # against the oracle's gradient at the Jacobi-CG solutions (both at 1e-12)
            r["pmg_fp32"]["kbar_rel_diff_vs_oracle"] = rel(g["kbar_pmg"], kb)
        log(f"  gradient: forward res {r['oracle_rel_res_forward']:.2e}, adjoint res "
            f"{r['oracle_rel_res_adjoint']:.2e}, kbar {r['kbar_rel_diff_vs_oracle']:.2e}")


def ax_kernel_name(N):
    """Which operator kernel the library launches at order N (the matrix-core
    one from N = 5 on unless SEM_AX_KERNEL overrides)."""
    if N < 5 or os.environ.get("SEM_AX_KERNEL", "") == "scalar":
        return "ax_kernel"
    return "ax_mfma_kernel"


# the operator kernel's sources: the counter summary holds for them only
OPERATOR_SOURCES = ("kernels_ax.hip", "common.hpp", "mfma_16x16x4.hpp")


def operator_sources_sha256():
    """sha256 over the operator kernel's source files, in OPERATOR_SOURCES order."""
    import hashlib

    h = hashlib.sha256()
    for name in OPERATOR_SOURCES:
        with open(os.path.join(ROOT, "paper_2501_13240_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_traffic():
    """HBM bytes per operator launch from the committed rocprofv3 counter summary,
    or None when the operator's sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "ax_N7_convection_box_traffic.txt")
    try:
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith(("|", "#", " ")):
                key, val = line.split(":", 1)
                kv[key.strip()] = val.strip()
        if kv.get("operator sources sha256") != operator_sources_sha256():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def true_rel_residual(sem, M, b, x, k=None, h2=0.0):
    """||b - A x|| / ||b|| over the free unique nodes with the FP64 operator."""
    import torch

    w = sem.gs(M, sem.ax(M, x, k=k, h2=h2))
    r = sem.mask(M, (b - w).contiguous())
    bb = sem.mask(M, b.clone())
    if M.info["has_nullspace"] and h2 == 0.0:
        mult = M.multiplicity()
        n = M.info["n_unique"]
        r = r - torch.sum(r / mult) / n
        bb = bb - torch.sum(bb / mult) / n
    mult = M.multiplicity()
    return float(torch.sqrt(torch.sum(r * r / mult) / torch.sum(bb * bb / mult)))


def ax_rate(sem, M, dtype, reps, k=None, h2=0.0):
    """Stand-alone sem_ax on a mesh: median of individually event-timed applies
    after 5 warm-ups; algorithmic bytes per local point 64 (FP64) or 32 (FP32)
    for u, G and w, plus one value each for k and, with h2 != 0, for B."""
    import torch
    u = torch.randn(M.E, M.P, dtype=dtype, device="cuda")
    w = torch.empty_like(u)
    for _ in range(5):
        sem.ax(M, u, k=k, h2=h2, out=w)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for e0, e1 in evs:
        e0.record()
        sem.ax(M, u, k=k, h2=h2, out=w)
        e1.record()
    torch.cuda.synchronize()
    ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in evs]))
    vb = 8.0 if dtype == torch.float64 else 4.0
    nbytes = (8 * vb + (vb if k is not None else 0.0) + (vb if h2 != 0.0 else 0.0)) \
        * M.info["n_local"]
    return {"us": ms * 1e3, "gdof_s": M.info["n_unique"] / (ms * 1e-3) / 1e9,
            "algorithmic_bytes": nbytes, "gb_s": nbytes / (ms * 1e-3) / 1e9,
            "hbm_frac": nbytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}


def mixed_vs_fp64(sem, only="", reps=20):
    """Time to ||b - A x|| <= 1e-10 ||b|| on the 32^3-element, N = 9,
    all-Neumann box: FP64 Jacobi CG against the mixed-precision variants; and
    the stand-alone operator's rate on that mesh."""
    import torch
    from sem_inputs import config_mesh

    m, fld = config_mesh(5)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, m.N)
    b_host = fld["b"]
    b = torch.tensor(b_host, device="cuda")
    del fld, m
    variants = {
        "fp64_jacobi_cg": dict(mode="cg", precond="jacobi"),
        "fp64_cheb3_fcg": dict(mode="cg", precond="chebyshev", precond_prec="fp64"),
        "fp64_cg_fp32_cheb3": dict(mode="cg", precond="chebyshev", precond_prec="fp32"),
        "fp64_cg_bf16_cheb3": dict(mode="cg", precond="chebyshev", precond_prec="bf16_mfma"),
        "mixed_ir_fp32_cg": dict(mode="mixed_ir", precond="jacobi", precond_prec="fp32"),
        "fp64_pmg_jacobi_fcg": dict(mode="cg", precond="pmg", precond_prec="fp64"),
        "fp64_cg_fp32_pmg_jacobi": dict(mode="cg", precond="pmg", precond_prec="fp32"),
        "fp64_pmg_fcg": dict(mode="cg", precond="pmg", precond_prec="fp64"),
        "fp64_cg_fp32_pmg": dict(mode="cg", precond="pmg", precond_prec="fp32"),
        "mixed_ir_fp32_pmg": dict(mode="mixed_ir", precond="pmg", precond_prec="fp32"),
    }
    if only:
        keep = set(only.split(","))
        unknown = keep - set(variants)
        if unknown:
            raise SystemExit(f"unknown mixed variants: {sorted(unknown)}")
        variants = {k: v for k, v in variants.items() if k in keep}
    out = {"workload": "32x32x32 hexahedra, N=9, tanh 1:20 z-clustering, seeded wall-preserving "
                       "deformation, all-Neumann (constant mode removed), zero-mean random rhs",
           "n_unique": M.info["n_unique"], "rtol": 1e-10}
    out["ax_fp64"] = ax_rate(sem, M, torch.float64, reps)
    out["ax_fp32"] = ax_rate(sem, M, torch.float32, reps)
    log(f"  sem_ax N = 9: FP64 {out['ax_fp64']['us']:.1f} us ({out['ax_fp64']['hbm_frac']:.3f}), "
        f"FP32 {out['ax_fp32']['us']:.1f} us ({out['ax_fp32']['hbm_frac']:.3f})")
    sem.lmax_estimate(M)  # bound estimate shared by the Chebyshev variants (cached)
    for name, v in variants.items():
        pmg_setup(sem, M, b, name)
        x, st = sem.solve(M, b, rtol=1e-10, max_iter=30000, **v)
        res = true_rel_residual(sem, M, b, x)
        out[name] = {"ms": st["time_ms"], "iters": st["iters"], "outer": st["outer_iters"],
                     "true_rel_res": res,
                     "gdof_s": M.info["n_unique"] * st["iters"] / (st["time_ms"] * 1e-3) / 1e9}
        CHECKS.add("cube5", dict(cfg=5), b_host, name, x.cpu().numpy(), out[name])
        log(f"  {name}: {st['time_ms']:.1f} ms, {st['iters']} it, true rel res {res:.2e}")
    fp64 = ("fp64_jacobi_cg", "fp64_cheb3_fcg", "fp64_pmg_fcg", "fp64_pmg_jacobi_fcg")
    best = min((k for k in variants if k not in fp64
                and out[k]["true_rel_res"] <= 1e-10), key=lambda k: out[k]["ms"], default=None)
    out["fastest_mixed"] = best
    if best and "fp64_jacobi_cg" in out:
        out["speedup_vs_fp64"] = out["fp64_jacobi_cg"]["ms"] / out[best]["ms"]
    if "fp64_cg_fp32_pmg" in out:
        # whole-iteration roofline of the FP32-cycle p-multigrid solve
        total, parts = pmg_cube_iteration_bytes()
        v = out["fp64_cg_fp32_pmg"]
        ms_it = v["ms"] / v["iters"]
        out["pmg_roofline"] = {
            "variant": "fp64_cg_fp32_pmg", "bound": "hbm",
            "ms_per_iteration": ms_it,
            "algorithmic_bytes_per_iteration": total,
            "achieved": total / (ms_it * 1e-3) / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": total / (ms_it * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "timing": "solve time / iterations (the first V-cycle, z_0 = M r_0, included)",
            "bytes_by_kernel": parts,
        }
    if "fp64_pmg_fcg" in out and "fp64_cg_fp32_pmg" in out:
        # the same preconditioner in FP64 and with the FP32 cycle
        out["pmg_fp32_cycle_speedup_vs_fp64_pmg"] = (out["fp64_pmg_fcg"]["ms"]
                                                     / out["fp64_cg_fp32_pmg"]["ms"])
    M.close()
    return out


def pmg_cube_iteration_bytes(nel=32, orders=(9, 4, 2, 1), smooth_order=4, coarse_iters=30):
    """Algorithmic HBM bytes of one iteration of FP64 flexible CG preconditioned
    by one FP32 Schwarz-smoothed V-cycle on the all-Neumann nel^3 cube (every
    kernel the iteration launches, each array counted once per access; index
    arrays 4 B, FP32 values 4 B, FP64 values 8 B).  Returns (total, per-kernel
    dict of bytes per iteration).  Counts of the structured mesh:
    local points E (N+1)^3, free nodes (nel N + 1)^3, single-copy nodes the
    element interiors and the boundary-face interiors, box copies E ((N+1)^3 +
    6 (N+1)^2) minus the (N+1)^2 layer missing behind each boundary face."""
    E = nel ** 3
    faces_b = 6 * nel * nel

    def sizes(N):
        nL = E * (N + 1) ** 3
        nf = (nel * N + 1) ** 3
        n1 = E * (N - 1) ** 3 + faces_b * (N - 1) ** 2
        box_pts = (N + 3) ** 3
        box_copies = E * ((N + 1) ** 3 + 6 * (N + 1) ** 2) - faces_b * (N + 1) ** 2
        return nL, nf, n1, box_pts, box_copies

    out = {}

    def add(name, b):
        out[name] = out.get(name, 0.0) + b

    # outer FP64 flexible CG
    nL, nf, n1, _, _ = sizes(orders[0])
    add("ax FP64 in-solve (64 B per local point)", 64.0 * nL)
    add("shared-node sum (12 B per shared copy, 12 B per shared node)",
        12.0 * (nL - n1) + 12.0 * (nf - n1))
    add("CG update (24 B per free node)", 24.0 * nf)
    add("residual to FP32 (12 B per free node)", 12.0 * nf)
    add("z and dots (28 B per free node)", 28.0 * nf)
    add("x and p update (40 B per free node)", 40.0 * nf)
    # V-cycle (FP32)
    for lev, N in enumerate(orders):
        nL, nf, n1, bp, bc = sizes(N)
        if lev == len(orders) - 1:
            # coarsest: fixed Jacobi-PCG iterations (operator 32 B per local point,
            # sum 8 B per copy + 12 per node, update 20 B and p update 16 B per node)
            add("coarse CG", coarse_iters * (32.0 * nL + 8.0 * nL + 12.0 * nf + 36.0 * nf))
            break
        m = smooth_order
        add("ax FP32 (32 B per local point)", (2 * (m - 1) + 2) * 32.0 * nL)
        add("Schwarz local solves (12 B per box point + factors)",
            2 * m * E * (12.0 * bp + 4.0 * (3 * (N + 3) ** 2 + 3 * (N + 3))))
        add("Schwarz sums with the recurrence (8 B per box copy + 12 / 20 B per node)",
            2 * (8.0 * bc + 12.0 * nf) + 2 * (m - 1) * (8.0 * bc + 20.0 * nf))
        if N >= 5:
            # split-form residual: wf and r (or b) at single-copy nodes, 8 B per
            # shared copy, 8 B per shared node, r written
            add("residual, split form (8 B per single-copy node, 8 B per shared copy and "
                "shared node, 4 B written per node)",
                (2 * (m - 1) + 2) * (8.0 * n1 + 8.0 * (nL - n1) + 8.0 * (nf - n1) + 4.0 * nf))
        else:
            add("residual sums (8 B per local copy + 12 B per node)",
                (2 * (m - 1) + 2) * (8.0 * nL + 12.0 * nf))
        nLc, nfc = sizes(orders[lev + 1])[:2]
        add("restriction (4 B per fine point, 8 per fine node, 4 per coarse point; then 8 B "
            "per coarse copy + 8 per coarse node)",
            4.0 * nL + 8.0 * nf + 4.0 * nLc + 8.0 * nLc + 8.0 * nfc)
        add("prolongation (4 B per coarse point and node, 4 per fine point; then 8 B per "
            "copy + 12 per node)",
            4.0 * nLc + 4.0 * nfc + 4.0 * nL + 8.0 * nL + 12.0 * nf)
        add("post-smoothing add (12 B per node)", 12.0 * nf)
    return sum(out.values()), out


def pmg_setup(sem, M, b, name):
    """Variants named *_pmg_jacobi* use Jacobi-smoothed p-multigrid (order-5
    smoothing, 20 coarse iterations), the other *_pmg* ones the library
    default (Schwarz smoothing); the hierarchy is rebuilt when that changes
    and its level bounds are formed before the timed solve."""
    if "pmg" not in name:
        return
    kind = "jacobi" if "pmg_jacobi" in name else "schwarz"
    if getattr(M, "_bench_pmg_kind", None) == kind:
        return
    if kind == "jacobi":
        M.setup_pmg(smoother="jacobi", smooth_order=5, coarse_iters=20)
    else:
        M.setup_pmg()
    for prec in ("fp32", "fp64"):
        sem.solve(M, b, rtol=1e-10, max_iter=2, precond="pmg", precond_prec=prec,
                  raise_on_noconv=False)
    M._bench_pmg_kind = kind


def to_tolerance(sem, M, b, b_host):
    """Time to ||b - A x|| <= 1e-10 ||b|| on the benchmark mesh: FP64 Jacobi
    CG against p-multigrid-preconditioned flexible CG (FP64 and FP32 cycles)
    and refinement around it."""
    variants = {
        "fp64_jacobi_cg": dict(mode="cg", precond="jacobi"),
        "fp64_pmg_jacobi_fcg": dict(mode="cg", precond="pmg", precond_prec="fp64"),
        "fp64_cg_fp32_pmg_jacobi": dict(mode="cg", precond="pmg", precond_prec="fp32"),
        "fp64_pmg_fcg": dict(mode="cg", precond="pmg", precond_prec="fp64"),
        "fp64_cg_fp32_pmg": dict(mode="cg", precond="pmg", precond_prec="fp32"),
        "mixed_ir_fp32_pmg": dict(mode="mixed_ir", precond="pmg", precond_prec="fp32"),
    }
    out = {"rtol": 1e-10}
    for name, v in variants.items():
        pmg_setup(sem, M, b, name)
        x, st = sem.solve(M, b, rtol=1e-10, max_iter=30000, **v)
        out[name] = {"ms": st["time_ms"], "iters": st["iters"], "outer": st["outer_iters"],
                     "true_rel_res": true_rel_residual(sem, M, b, x)}
        CHECKS.add("box2", dict(cfg=2), b_host, name, x.cpu().numpy(), out[name])
        log(f"  {name}: {st['time_ms']:.1f} ms, {st['iters']} it, "
            f"true rel res {out[name]['true_rel_res']:.2e}")
    return out


def gs_rate(sem, M, reps):
    """sem_gs on the benchmark mesh: 20 B per local copy of a shared node
    (index 4, read 8, write 8) + 4 B per shared node (segment offset).
    sector_floor_bytes: what any gather-scatter on the [E][P] FP64 layout must
    move, since memory is read and written in 32-byte sectors: every sector that
    holds a shared copy, read and written once, plus the index arrays."""
    import torch

    mult = M.multiplicity()
    shared = mult > 1
    copies = int(shared.sum())
    nodes = float((1.0 / mult[shared]).sum())
    alg = 20.0 * copies + 4.0 * nodes
    sectors = int(shared.reshape(-1, 4).any(dim=1).sum())
    floor = 2.0 * 32.0 * sectors + 4.0 * copies + 4.0 * nodes
    v = torch.randn(M.E, M.P, dtype=torch.float64, device="cuda")
    for _ in range(3):
        sem.gs(M, v)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        sem.gs(M, v)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) / reps * 1e3
    return {"us": us, "algorithmic_bytes": alg, "gb_s": alg / us / 1e3,
            "shared_copies": copies, "sector_floor_bytes": floor,
            "sector_floor_gb_s": floor / us / 1e3,
            "sector_floor_frac": floor / us / 1e3 / PEAK_HBM_GBS}


PEAK_MFMA_TFLOPS = {8: 78.6, 4: 157.3}  # MI355X dense matrix cores, FP64 / FP32


def dealias_mfma_per_element(N, nf):
    """16x16x4 MFMA products the dealiased convective-term kernel executes per
    element: per velocity component the three interpolation stages, per field
    the derivative stages (2 i-, 3 j- and 3 k-stage products) and the three
    projection stages; each stage is ceil(columns / 16) tiles of ceil(K / 4)
    products (padded rows and columns included)."""
    n, M = N + 1, (3 * (N + 1)) // 2
    nt = lambda c: (c + 15) // 16
    kn, km = (n + 3) // 4, (M + 3) // 4
    i0, i1, i2 = nt(n * n), nt(n * M), nt(M * M)
    u_pass = (i0 + i1 + i2) * kn
    f_pass = (2 * i0 + 3 * i1 + 3 * i2) * kn
    back = (nt(M * M) + nt(n * M) + nt(n * n)) * km
    return 3 * u_pass + nf * (f_pass + back)


def advection_rate(sem, M, m, reps):
    """sem_advect on the benchmark mesh (smooth seeded velocity and scalar),
    and sem_advect_fields on the four fields of a Boussinesq step (the scalar
    and the three velocity components, advected by the velocity): median of
    individually event-timed launches after warm-ups.  Algorithmic bytes per
    element: u (3 P values) and the nine factors per quadrature point (9 q1^3)
    once, plus f and out (P values each) per field, in the arithmetic's
    width."""
    import torch
    from sem_inputs import random_fourier_field, velocity_field

    t = time.time()
    u64 = torch.tensor(velocity_field(m.xyz, seed=11, M=8), device="cuda")
    f64 = torch.tensor(random_fourier_field(m.xyz, M=16, seed=7), device="cuda")
    log(f"advection inputs in {time.time() - t:.1f}s")
    out = {}

    def timed(fn):
        for _ in range(3):
            fn()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(reps)]
        for e0, e1 in evs:
            e0.record()
            fn()
            e1.record()
        torch.cuda.synchronize()
        return float(np.median([e0.elapsed_time(e1) for e0, e1 in evs]))

    for rule in ("dealias", "collocation"):
        t = time.time()
        M.setup_advection(rule)
        setup_s = time.time() - t
        q1 = sem.advection_rule(M.N, rule)[0].size
        for dt, width in ((torch.float64, 8), (torch.float32, 4)):
            u, f = u64.to(dt), f64.to(dt)
            fields = torch.cat([f[None], u]).contiguous()
            w, w4 = torch.empty_like(f), torch.empty_like(fields)
            name = f"{rule}_{'fp64' if width == 8 else 'fp32'}"
            for nf, fin, fout in ((1, f, w), (4, fields, w4)):
                ms = timed(lambda: sem.advect(M, u, fin, rule=rule, out=fout))
                alg = float(M.E) * (3 * M.P + 9 * q1 ** 3 + 2 * nf * M.P) * width
                key = name if nf == 1 else name + "_4fields"
                out[key] = {"us": ms * 1e3, "points_per_dir": q1, "fields": nf,
                            "algorithmic_bytes": alg, "gb_s": alg / ms / 1e6,
                            "hbm_frac": alg / ms / 1e6 / PEAK_HBM_GBS,
                            "glocal_points_s": nf * M.E * M.P / (ms * 1e-3) / 1e9,
                            "setup_s": setup_s}
                if rule == "dealias":
                    # the matrix-core side of the same launch (executed products)
                    fl = 2048.0 * dealias_mfma_per_element(M.N, nf) * M.E
                    out[key]["mfma_tflops"] = fl / (ms * 1e-3) / 1e12
                    out[key]["mfma_frac"] = fl / (ms * 1e-3) / 1e12 / PEAK_MFMA_TFLOPS[width]
                log(f"  advect {key}: {ms * 1e3:.1f} us, {out[key]['gb_s']:.0f} GB/s")
    return out


def small_solves(sem):
    """Time to ||b - A x|| <= 1e-10 ||b|| on the 4^3-element unit cube at
    N = 7 and 9 (manufactured right-hand side): launch-bound cases, the
    variants differ by iteration counts, not bandwidth."""
    import torch
    from sem_inputs import config_mesh

    variants = {
        "fp64_jacobi_cg": dict(mode="cg", precond="jacobi"),
        "fp64_cheb3_fcg": dict(mode="cg", precond="chebyshev", precond_prec="fp64"),
        "fp64_cg_fp32_cheb3": dict(mode="cg", precond="chebyshev", precond_prec="fp32"),
        "fp64_cg_bf16_cheb3": dict(mode="cg", precond="chebyshev", precond_prec="bf16_mfma"),
        "fp64_cg_fp16_cheb3": dict(mode="cg", precond="chebyshev", precond_prec="fp16_mfma"),
        "mixed_ir_fp32_cg": dict(mode="mixed_ir", precond="jacobi", precond_prec="fp32"),
        "mixed_ir_fp32_cheb3": dict(mode="mixed_ir", precond="chebyshev", precond_prec="fp32"),
        "fp64_cg_fp32_pmg_jacobi": dict(mode="cg", precond="pmg", precond_prec="fp32"),
        "fp64_cg_fp32_pmg": dict(mode="cg", precond="pmg", precond_prec="fp32"),
    }
    out = {}
    for N in (7, 9):
        m, fld = config_mesh(1, N=N)
        M = sem.Mesh(m.xyz, m.gid, m.dirichlet, m.N)
        u_exact = fld["f"]  # the manufactured solution at the local points
        f = torch.tensor(u_exact * 3 * np.pi ** 2, device="cuda")
        b = sem.gs(M, sem.mass(M, f))
        sem.lmax_estimate(M)
        res = {"n_unique": M.info["n_unique"],
               "ax_fp64": ax_rate(sem, M, torch.float64, 20)}
        for name, v in variants.items():
            pmg_setup(sem, M, b, name)
            sem.solve(M, b, rtol=1e-10, **v)  # warm (graph capture, work space)
            best = None
            for _ in range(3):
                x, st = sem.solve(M, b, rtol=1e-10, **v)
                if best is None or st["time_ms"] < best[1]["time_ms"]:
                    best = (x, st)
            x, st = best
            res[name] = {"ms": st["time_ms"], "iters": st["iters"], "outer": st["outer_iters"],
                         "true_rel_res": true_rel_residual(sem, M, b, x),
                         "gdof_it_s": M.info["n_unique"] * st["iters"] / (st["time_ms"] * 1e-3)
                         / 1e9,
                         "max_err_vs_u_exact": float(np.max(np.abs(x.cpu().numpy() - u_exact)))}
            CHECKS.add(f"cube1_N{N}", dict(cfg=1, N=N), None, name, x.cpu().numpy(), res[name])
        out[f"N{N}"] = res
        M.close()
    return out


def gradient_timing(sem):
    """Forward solve and backward (adjoint solve + k-contraction) on the
    16^3-element, N = 7 variable-coefficient Helmholtz cube, both to 1e-12."""
    import torch
    from sem_inputs import config_mesh

    m, fld = config_mesh(4)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, m.N)
    f = torch.tensor(fld["f"], device="cuda")
    b = sem.gs(M, sem.mass(M, f))
    target = f / (3 * np.pi ** 2 + 1.0)
    free = M.multiplicity()
    w = torch.where(sem.mask(M, torch.ones_like(f)) > 0, 1.0 / free, torch.zeros_like(f))
    k0 = torch.tensor(fld["k"], device="cuda")
    out = {}

    def timed_pass(opts):
        k = k0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = sem.sem_solve(M, b, k=k, h2=fld["h2"], rtol=1e-12, **opts)
        loss = torch.sum(w * (x - target) ** 2)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return x, k, (t1 - t0) * 1e3, (t2 - t1) * 1e3

    for rep in range(2):
        x, k, fwd, bwd = timed_pass({})
        out = {"forward_ms": fwd, "backward_ms": bwd, "n_unique": M.info["n_unique"]}
    # the operator with k and the h2 mass term (80 B per local point); its
    # 168 MB stream fits in the memory-side cache, so this is no HBM figure
    out["ax_fp64_k_h2"] = ax_rate(sem, M, torch.float64, 20, k=k0, h2=fld["h2"])
    out["ax_fp64_k_h2"]["cache_resident"] = True
    # the same forward and backward with FP64 flexible CG preconditioned by the
    # FP32 p-multigrid cycle (k interpolated to every level); the hierarchy is
    # built and the level bounds formed outside the timing
    M.setup_pmg()
    pmg = dict(precond="pmg", precond_prec="fp32")
    for rep in range(2):
        xp, kp, fwd, bwd = timed_pass(pmg)
    out["pmg_fp32"] = {"forward_ms": fwd, "backward_ms": bwd,
                       "x_rel_diff_vs_jacobi": float(torch.linalg.norm(xp.detach() - x.detach())
                                                     / torch.linalg.norm(x.detach())),
                       "kbar_rel_diff_vs_jacobi": float(torch.linalg.norm(kp.grad - k.grad)
                                                        / torch.linalg.norm(k.grad))}
    # for the oracle's checks (untimed): the cotangent autograd passes,
    # dL/dx = 2 w (x - target), and the adjoint solution lam = bbar x copies
    xd = x.detach()
    xbar = (2.0 * w * (xd - target)).contiguous()
    kbar, bbar, _ = sem.solve_backward(M, xd, xbar, k=k0, h2=fld["h2"], rtol=1e-12,
                                       max_iter=20000)
    GRAD_CHECK.update(x=xd.cpu().numpy(), xbar=xbar.cpu().numpy(),
                      lam=(bbar * free).cpu().numpy(), kbar=kbar.cpu().numpy(),
                      kbar_autograd=k.grad.detach().cpu().numpy(), result=out,
                      x_pmg=xp.detach().cpu().numpy(),
                      kbar_pmg=kp.grad.detach().cpu().numpy())
    M.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs the single-GPU path only; the "
                                   "multi-GPU decomposition is a design, not code: --gpus "
                                   "must be 1"}))
        sys.exit(2)

    import torch

    import paper_2501_13240_amd as sem
    from sem_inputs import config_mesh

    torch.cuda.set_device(0)
    t = time.time()
    m, fld = config_mesh(2)
    log(f"mesh built in {time.time() - t:.1f}s: E={m.E} N={m.N} n_unique={m.n_unique}")
    t = time.time()
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, m.N)
    log(f"setup in {time.time() - t:.1f}s: {M.info}")
    b_host = fld["b"]
    b = torch.tensor(b_host, device="cuda")
    del fld
    x = torch.zeros_like(b)
    n_unique = M.info["n_unique"]
    nL = M.info["n_local"]

    def step(profile):
        return sem.solve(M, b, max_iter=args.iters, fixed_iters=True, profile=profile, out=x)[1]

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    log("warmup done")

    # The last timed step records a HIP event pair around each of its operator
    # launches (the roofline's launch time); the others run without them.
    ax_ms, ax_n = 0.0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        st = step(i == args.steps - 1)
        ax_ms += st.get("ax_ms", 0.0)
        ax_n += st.get("ax_launches", 0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n_unique * args.iters / (ms_per_step * 1e-3) / 1e9
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, {value:.2f} GDOF/s")

    ax_avg_ms = ax_ms / max(ax_n, 1)
    alg_bytes = 64.0 * nL
    achieved = alg_bytes / (ax_avg_ms * 1e-3) / 1e9

    # standalone operator apply (sem_ax) rate
    # median of individually event-timed applies after 5 warm-ups
    u = torch.randn(M.E, M.P, dtype=torch.float64, device="cuda")
    w = torch.empty_like(u)
    for _ in range(5):
        sem.ax(M, u, out=w)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.ax_reps)]
    for e0, e1 in evs:
        e0.record()
        sem.ax(M, u, out=w)
        e1.record()
    torch.cuda.synchronize()
    sem_ax_ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in evs]))
    log(f"sem_ax: {sem_ax_ms * 1e3:.1f} us, {64.0 * nL / sem_ax_ms / 1e6:.0f} GB/s")

    gs = gs_rate(sem, M, args.ax_reps)
    log(f"sem_gs: {gs['us']:.1f} us, {gs['gb_s']:.0f} GB/s")

    log("convective term (sem_advect) on the benchmark mesh ...")
    adv = advection_rate(sem, M, m, args.ax_reps)

    # what a plain device copy sustains on this HBM (context for the fractions
    # of the 8 TB/s peak above): 1 GiB read and 1 GiB written per copy
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    cev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(5)]
    for e0, e1 in cev:
        e0.record()
        dst.copy_(src)
        e1.record()
    torch.cuda.synchronize()
    copy_ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in cev]))
    copy_gb_s = 2.0 * src.numel() * 8 / (copy_ms * 1e-3) / 1e9
    log(f"1 GiB device copy: {copy_ms * 1e3:.0f} us, {copy_gb_s:.0f} GB/s")
    if args.copy_calibration:
        # three more dispatches, so the counter runs see the copy kernel at
        # least three times whatever else the run launches
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 1 GiB device copies done")
    del src, dst

    out = {
        "metric": "GDOF/s of SEM Ax and PCG solve (N=7, 1 GPU); mixed vs FP64 at 1e-10 residual",
        "value": value,
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": ("convection box share: 32x32x16 hexahedra, N=7, periodic x/y, "
                         "Dirichlet plates, tanh 1:20 z-clustering, seeded deformation, "
                         "random normal rhs; 100 Jacobi-PCG iterations per step"),
            "E": M.E, "N": M.N, "n_unique": n_unique, "n_local": nL,
            "iterations_per_step": args.iters,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": counter_traffic(),
            "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "kernel": (f"{ax_kernel_name(M.N)}<{M.N},double,in-solve> (element operator: p gathered, "
                       "w to the free vector at single-copy nodes and to the local vector at "
                       "shared ones; 64 B/local point)"),
            "avg_launch_us": ax_avg_ms * 1e3,
            "launches_timed": ax_n,
        },
        "ax_gdof_s": n_unique / (sem_ax_ms * 1e-3) / 1e9,
        "ax_us": sem_ax_ms * 1e3,
        "ax_hbm_frac": 64.0 * nL / (sem_ax_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
        "hbm_copy": {"gb_s": copy_gb_s, "frac_of_peak": copy_gb_s / PEAK_HBM_GBS,
                     "what": "torch copy_ of 1 GiB FP64, device to device, median of 5"},
        "gs": gs,
        "advection": adv,
    }
    if not args.no_extras:
        log("to 1e-10 on the benchmark mesh ...")
        out["to_tolerance"] = to_tolerance(sem, M, b, b_host)
        M.close()
        log("small solves (4^3 unit cube, N = 7 and 9) ...")
        out["small_solves"] = small_solves(sem)
        log("forward/backward on the 16^3 Helmholtz cube ...")
        out["gradient"] = gradient_timing(sem)
    if not args.no_mixed:
        log("mixed vs FP64 on the 32^3, N=9 Neumann box ...")
        M.close()
        out["mixed_vs_fp64"] = mixed_vs_fp64(sem, args.mixed_variants, args.ax_reps)
    M.close()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cb = cpu_baseline(args.cpu_sample_iters)
        cb.pop("seconds", None)
        out["cpu_baseline"] = cb
        log("oracle errors of the solve results ...")
        t = time.time()
        oracle_errors(out)
        log(f"oracle errors in {time.time() - t:.1f}s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
