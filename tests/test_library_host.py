"""Host-side checks of libsem (no device work): exported symbols, the
library's GLL quadrature, its numbering, and argument validation that fails
before any device call."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_2501_13240_amd as sem
from paper_2501_13240_amd import _lib as L
from sem_inputs import box_mesh, config_mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(sem_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = L.load()
    declared = _declared_symbols()
    assert len(declared) >= 17
    for name in declared:
        assert hasattr(lib, name), name
    assert set(L.SIGNATURES) == declared


def test_struct_layouts_match_header():
    # field offsets a C compiler gives these structs on x86-64
    assert ctypes.sizeof(L.MeshDesc) == 40
    assert ctypes.sizeof(L.SolveOpts) == 72
    assert ctypes.sizeof(L.SolveStats) == 56
    assert ctypes.sizeof(L.MeshInfo) == 48
    assert ctypes.sizeof(L.PmgOpts) == 48


_STRUCTS = {"sem_mesh_desc": L.MeshDesc, "sem_mesh_info": L.MeshInfo,
            "sem_solve_opts": L.SolveOpts, "sem_solve_stats": L.SolveStats,
            "sem_pmg_opts": L.PmgOpts}


def test_struct_layouts_match_a_c_compiler(tmp_path):
    """sizeof/offsetof of every public struct as gcc lays it out from the
    header, against the binding's ctypes declarations."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "sem.h"', "int main(void) {"]
    for cname, py in _STRUCTS.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}
    for cname, py in _STRUCTS.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


CLOSED = {
    1: ([-1.0, 1.0], [1.0, 1.0]),
    2: ([-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    3: ([-1.0, -1 / np.sqrt(5), 1 / np.sqrt(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    4: ([-1.0, -np.sqrt(3 / 7), 0.0, np.sqrt(3 / 7), 1.0],
        [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
}


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_library_gll_closed_forms(N):
    xi, rho, D = sem.gll(N)
    np.testing.assert_allclose(xi, CLOSED[N][0], atol=1e-15)
    np.testing.assert_allclose(rho, CLOSED[N][1], rtol=1e-14)


@pytest.mark.parametrize("N", range(1, 11))
def test_library_gll_exactness(N):
    xi, rho, D = sem.gll(N)
    for m in range(2 * N):
        assert abs(rho @ xi ** m - (0.0 if m % 2 else 2.0 / (m + 1))) < 1e-13
    for m in range(N + 1):
        d = m * xi ** (m - 1) if m else 0 * xi
        np.testing.assert_allclose(D @ xi ** m, d, atol=1e-12 * N * N)


@pytest.mark.parametrize("N", [0, 11, -3])
def test_library_gll_rejects_bad_order(N):
    assert L.load().sem_gll(N, None, None, None) == L.SEM_EINVAL


@pytest.mark.parametrize("cfg", [1, 3])
def test_numbering_counts_and_first_touch(cfg):
    m, _ = config_mesh(cfg)
    fi, nu, nf, ns = sem.host_numbering(m.N, m.gid, m.dirichlet)
    assert nu == (4 * m.N + 1) ** 3 and nf == (4 * m.N - 1) ** 3
    # copies of one global node share one free index; Dirichlet copies get -1
    d = m.dirichlet.astype(bool)
    assert np.all(fi[d] == -1) and np.all(fi[~d] >= 0)
    first = {}
    for g, f in zip(m.gid.ravel(), fi.ravel()):
        if f >= 0:
            assert first.setdefault(g, f) == f
    # single-copy nodes first, then shared ones, each class in first-touch
    # order: within a class, free indices increase with the first visit
    seen = fi.ravel()[fi.ravel() >= 0]
    _, first_visit = np.unique(seen, return_index=True)  # per free index
    copies = np.bincount(seen, minlength=nf)
    n1 = int(np.sum(copies == 1))
    assert np.all(copies[:n1] == 1) and np.all(copies[n1:] > 1)
    assert np.all(np.diff(first_visit[:n1]) > 0) and np.all(np.diff(first_visit[n1:]) > 0)
    # element interiors at N = 7 on a 4^3 mesh: 64 elements x 6^3 nodes
    assert n1 == 64 * (m.N - 1) ** 3


def test_numbering_periodic_and_shared_counts():
    N = 3
    m = box_mesh(N, (4, 3, 2), (4.0, 4.0, 1.0), periodic=(True, True, False), dirichlet="z")
    fi, nu, nf, ns = sem.host_numbering(N, m.gid, m.dirichlet)
    assert nu == 12 * 9 * 7 and nf == 12 * 9 * 5
    mult = np.bincount(m.gid.ravel())
    assert ns == np.sum(mult > 1)


def test_numbering_sparse_gids_use_sort_path():
    m = box_mesh(2, (2, 2, 2), dirichlet="none")
    gid = m.gid * 1_000_003 + 7  # far beyond the direct-table range
    fi, nu, nf, ns = sem.host_numbering(2, gid, None)
    fi2, nu2, nf2, ns2 = sem.host_numbering(2, m.gid, None)
    assert (nu, nf, ns) == (nu2, nf2, ns2)
    np.testing.assert_array_equal(fi, fi2)


def test_numbering_rejects_inconsistent_dirichlet_and_negative_gid():
    m = box_mesh(2, (2, 2, 2))
    d = m.dirichlet.copy()
    # flag one copy of an interior shared node only
    g = m.gid[0, -1]
    idx = np.argwhere(m.gid == g)
    d[tuple(idx[0])] = 1
    with pytest.raises(sem.SemError, match="EINVAL"):
        sem.host_numbering(2, m.gid, d)
    with pytest.raises(sem.SemError, match="EINVAL"):
        sem.host_numbering(2, m.gid - 1, None)


def _setup_status(N, E, xyz, gid, d):
    lib = L.load()
    desc = L.MeshDesc(N, E, None if xyz is None else xyz.ctypes.data_as(ctypes.c_void_p),
                      None if gid is None else gid.ctypes.data_as(ctypes.c_void_p),
                      None if d is None else d.ctypes.data_as(ctypes.c_void_p))
    h = ctypes.c_void_p()
    return lib.sem_setup_mesh(ctypes.byref(desc), None, ctypes.byref(h)), lib.sem_last_error()


def test_setup_validation_fails_before_device_work():
    m = box_mesh(2, (2, 2, 2))
    xyz, gid, d = m.xyz.copy(), m.gid.copy(), m.dirichlet.copy()
    assert _setup_status(0, m.E, xyz, gid, d)[0] == L.SEM_EINVAL
    assert _setup_status(11, m.E, xyz, gid, d)[0] == L.SEM_EINVAL
    assert _setup_status(2, 0, xyz, gid, d)[0] == L.SEM_EINVAL
    assert _setup_status(2, m.E, None, gid, d)[0] == L.SEM_EINVAL
    bad = xyz.copy()
    bad[3, 5, 1] = np.nan
    st, msg = _setup_status(2, m.E, bad, gid, d)
    assert st == L.SEM_EINVAL and b"finite" in msg
    d2 = d.copy()
    g = gid[0, -1]
    d2[tuple(np.argwhere(gid == g)[0])] = 1
    st, msg = _setup_status(2, m.E, xyz, gid, d2)
    assert st == L.SEM_EINVAL and b"Dirichlet" in msg


def test_null_handles_are_rejected():
    lib = L.load()
    assert lib.sem_ax(None, None, None, None, 0.0, 0, None) == L.SEM_EINVAL
    assert lib.sem_gs(None, None, 0, None) == L.SEM_EINVAL
    assert lib.sem_pcg_solve(None, None, None, None, 0.0, None, None, None) == L.SEM_EINVAL
    assert lib.sem_solve_backward(None, None, None, None, 0.0, None, None, None, None,
                                  None) == L.SEM_EINVAL
    assert lib.sem_free_mesh(None) == L.SEM_OK
    opts = L.SolveOpts()
    lib.sem_solve_opts_default(ctypes.byref(opts))
    assert opts.rtol == 1e-10 and opts.cheb_order == 3 and opts.max_iter == 10000


def _same_partition(a, b):
    a, b = a.ravel(), b.ravel()
    pairs = np.unique(np.stack([a, b], 1), axis=0)
    return len(pairs) == len(np.unique(a)) == len(np.unique(b))


@pytest.mark.parametrize("N,Nc", [(7, 3), (3, 1), (9, 4), (4, 2)])
@pytest.mark.parametrize("kw", [
    dict(periodic=(False, False, False), dirichlet="all", jitter=0.05),
    dict(periodic=(True, True, False), dirichlet="z", z_ratio=4.0,
         deform=dict(a=0.15, seed=1, kind="periodic")),
    dict(periodic=(False, True, True), dirichlet="none", jitter=0.05),
])
def test_host_coarse_mesh_matches_oracle(N, Nc, kw):
    """The library's coarse-order mesh (multigrid levels) against the oracle's:
    coordinates, the partition of local points into unknowns, Dirichlet flags."""
    import oracle
    m = box_mesh(N, (3, 3, 4), (1.0, 1.2, 0.9), **kw)
    xo, go, do = oracle.coarse_mesh(m.xyz, m.gid, m.dirichlet, N, Nc)
    xc, gc, dc = sem.host_coarse_mesh(N, m.gid, m.dirichlet, m.xyz, Nc)
    np.testing.assert_allclose(xc, xo, atol=1e-13)
    assert _same_partition(gc, go)
    if do is None:
        assert dc is None
    else:
        np.testing.assert_array_equal(dc, do)


def test_host_coarse_mesh_rejects_bad_input():
    m = box_mesh(3, (2, 2, 2), dirichlet="all")
    with pytest.raises(sem.SemError, match="EINVAL"):
        sem.host_coarse_mesh(3, m.gid, m.dirichlet, m.xyz, 3)
    # one element across a periodic direction: a face's corners share ids
    p = box_mesh(4, (1, 2, 2), periodic=(True, False, False), dirichlet="none")
    with pytest.raises(sem.SemError, match="share a global id"):
        sem.host_coarse_mesh(4, p.gid, None, p.xyz, 2)


@pytest.mark.parametrize("N", [2, 4, 7])
@pytest.mark.parametrize("kw", [
    dict(periodic=(False, False, False), dirichlet="all", jitter=0.05),
    dict(periodic=(True, True, False), dirichlet="z", z_ratio=4.0,
         deform=dict(a=0.15, seed=1, kind="periodic")),
    dict(periodic=(False, True, False), dirichlet="none", jitter=0.05),
])
def test_host_schwarz_matches_oracle(N, kw):
    """The library's Schwarz subdomains (as global ids of the box points) and
    its 1-D local inverses S diag(1/lam) S^T against the oracle's."""
    import oracle
    m = box_mesh(N, (3, 3, 4), (1.0, 1.2, 0.9), **kw)
    xmap, S, lam = sem.host_schwarz(N, m.gid, m.dirichlet, m.xyz)
    fi, _, nf, _ = sem.host_numbering(N, m.gid, m.dirichlet)
    lib_gid = np.empty(nf, dtype=np.int64)
    lib_gid[fi[fi >= 0]] = m.gid[fi >= 0]
    P = oracle.Problem(m.xyz, m.gid, m.dirichlet, N)
    Sch = oracle.Schwarz(m.xyz, m.gid, m.dirichlet, N, P.num)
    or_gid = P.num.gids[P.num.free]
    got = np.where(xmap >= 0, lib_gid[np.maximum(xmap, 0)], -1)
    want = np.where(Sch.ext >= 0, or_gid[np.maximum(Sch.ext, 0)], -1)
    np.testing.assert_array_equal(got, want)
    inv = lambda S_, L_: np.einsum("edij,edj,edkj->edik", S_, 1.0 / L_, S_)
    a, b = inv(S, lam), inv(Sch.S, Sch.lam)
    assert np.max(np.abs(a - b)) <= 1e-10 * np.max(np.abs(b))


@pytest.mark.parametrize("N", range(1, 11))
def test_advection_rules_match_oracle_and_integrate_exactly(N):
    from oracle.advection import quadrature
    for rule, de in (("dealias", True), ("collocation", False)):
        x, w, J = sem.advection_rule(N, rule)
        xo, wo, Jo, _ = quadrature(N, de)
        assert np.abs(x - xo).max() <= 1e-14 and np.abs(w - wo).max() <= 1e-14
        assert np.abs(J - Jo).max() <= 1e-13
        # exact for monomials up to degree 2 q1 - 1 (Gauss) or 2 q1 - 3 (GLL)
        top = 2 * x.size - 1 if de else 2 * x.size - 3
        for p in range(top + 1):
            exact = 0.0 if p % 2 else 2.0 / (p + 1)
            assert abs(w @ x ** p - exact) <= 1e-13
        # J reproduces degree-N polynomials at the points
        xg, _, _ = sem.gll(N)
        c = np.random.default_rng(N).standard_normal(N + 1)
        assert np.abs(J @ np.polyval(c, xg) - np.polyval(c, x)).max() <= 1e-12


def test_advection_rule_rejects_bad_arguments():
    lib = L.load()
    assert lib.sem_advection_rule(0, 1, None, None, None, None) == L.SEM_EINVAL
    assert lib.sem_advection_rule(11, 1, None, None, None, None) == L.SEM_EINVAL
    assert lib.sem_advection_rule(5, 2, None, None, None, None) == L.SEM_EINVAL
    q1 = ctypes.c_int32()
    assert lib.sem_advection_rule(7, 1, ctypes.byref(q1), None, None, None) == L.SEM_OK
    assert q1.value == 12
