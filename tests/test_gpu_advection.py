"""GPU parity of the convective term (sem_setup_advection, sem_advect,
sem_advect_fields) with the oracle's convect().

Tolerances (max-norm error relative to the largest reference value):
  factors w detJ dr_a/dx_d, FP64      <= 1e-12
  C_L(u) f, FP64                      <= 1e-12 (the FP64 apply bound)
  C_L(u) f, FP32                      <= 2e-5: inputs and factors rounded to
      FP32 (relative 6e-8 each) and sums of about 3 (N+1) + 3 M products per
      stage over four stages, with cancellation in u . grad f
"""

import ctypes

import numpy as np
import pytest
import torch

from oracle.advection import convect, dealias_points, geometric_factors_q
from sem_inputs import (box_mesh, config_mesh, random_fourier_field, reference_node_placement,
                        velocity_field)

pytestmark = pytest.mark.gpu

sem = pytest.importorskip("paper_2501_13240_amd")
from paper_2501_13240_amd import _lib as L  # noqa: E402

RULES = {"dealias": True, "collocation": False}


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def relmax(a, b):
    return np.abs(np.asarray(a) - b).max() / np.abs(b).max()


def _case(N, shape=(2, 2, 4), cfg=2):
    m, _ = config_mesh(cfg, N=N, shape=shape)
    u = velocity_field(m.xyz, seed=11)
    f = random_fourier_field(m.xyz, seed=7)
    return m, u, f


@pytest.mark.parametrize("rule", list(RULES))
@pytest.mark.parametrize("N", [1, 4, 7, 10])
def test_factors_match_oracle(N, rule):
    m, _, _ = _case(N)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, N)
    M.setup_advection(rule)
    G = M.advection_factors(rule).cpu().numpy()
    ref = geometric_factors_q(m.xyz, N, RULES[rule]).reshape(m.E, 9, -1)
    q1 = dealias_points(N) if RULES[rule] else N + 1
    assert G.shape == (m.E, 9, q1 ** 3)
    assert relmax(G, ref) <= 1e-12


@pytest.mark.parametrize("rule", list(RULES))
@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 8, 9, 10])
def test_advect_fp64_matches_oracle(N, rule):
    m, u, f = _case(N, shape=(3, 2, 4))  # 24 elements
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, N)
    out = sem.advect(M, dev(u), dev(f), rule=rule).cpu().numpy()
    ref = convect(np.moveaxis(u, 0, 2), f, m.xyz, N, dealias=RULES[rule])
    assert relmax(out, ref) <= 1e-12


@pytest.mark.parametrize("rule", list(RULES))
@pytest.mark.parametrize("N", [3, 6, 7, 9])
def test_advect_fp32_matches_oracle(N, rule):
    m, u, f = _case(N)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, N)
    out = sem.advect(M, dev(u, torch.float32), dev(f, torch.float32), rule=rule)
    ref = convect(np.moveaxis(u, 0, 2), f, m.xyz, N, dealias=RULES[rule])
    assert relmax(out.double().cpu().numpy(), ref) <= 2e-5


def test_advect_degenerate_fields():
    N = 7
    m, u, f = _case(N)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, N)
    for rule in RULES:
        zero = sem.advect(M, torch.zeros(3, m.E, (N + 1) ** 3, dtype=torch.float64,
                                         device="cuda"), dev(f), rule=rule)
        assert torch.count_nonzero(zero).item() == 0
        full = sem.advect(M, dev(u), dev(f), rule=rule).abs().max().item()
        const = sem.advect(M, dev(u), torch.full_like(dev(f), 2.5), rule=rule)
        assert const.abs().max().item() <= 1e-12 * full


@pytest.mark.parametrize("rule", list(RULES))
def test_assembled_constant_velocity_term_is_skew(rule):
    # periodic brick mesh: T . Q^T C_L(u) Q T = (Q T) . C_L(u) (Q T) = 0
    N = 7
    m = box_mesh(N, (8, 8, 4), (1.0, 1.0, 0.5), periodic=(True, True, True), dirichlet="none")
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, N)
    # one value per global node: copy-consistent across the periodic seams
    T = dev(np.random.default_rng(5).standard_normal(int(m.gid.max()) + 1)[m.gid])
    u = torch.empty(3, m.E, (N + 1) ** 3, dtype=torch.float64, device="cuda")
    for d, c in enumerate((0.7, -0.4, 1.3)):
        u[d] = c
    out = sem.advect(M, u, T, rule=rule)
    assert abs(torch.dot(T.flatten(), out.flatten()).item()) <= \
        1e-12 * T.norm().item() * out.norm().item()


def test_full_size_convection_box_sampled():
    # 32 x 32 x 16 elements at N = 7, the launch the benchmark times
    N = 7
    m, _ = config_mesh(2)
    u = velocity_field(m.xyz, seed=11)
    f = random_fourier_field(m.xyz, seed=7)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, N)
    idx = np.sort(np.random.default_rng(4).choice(m.E, 48, replace=False))
    idx[-1] = m.E - 1
    sel = torch.as_tensor(idx, device="cuda")
    for rule, de in RULES.items():
        out = sem.advect(M, dev(u), dev(f), rule=rule)[sel]
        ref = convect(np.moveaxis(u[:, idx], 0, 2), f[idx], m.xyz[idx], N, dealias=de)
        assert relmax(out.cpu().numpy(), ref) <= 1e-12
        # the four fields of a Boussinesq step in one call
        many = sem.advect(M, dev(u), dev(np.concatenate([f[None], u])), rule=rule)[:, sel]
        for k in range(1, 4):
            ref = convect(np.moveaxis(u[:, idx], 0, 2), u[k - 1, idx], m.xyz[idx], N, dealias=de)
            assert relmax(many[k].cpu().numpy(), ref) <= 1e-12


@pytest.mark.parametrize("N", [5, 6, 8, 9, 10])
def test_dealias_persistent_grid_sampled(N):
    # 1280 elements: more than the persistent grid, so workgroups walk
    # several elements and prefetch the next one's factors (the small meshes
    # above give every workgroup a single element)
    m, _ = config_mesh(2, N=N, shape=(16, 16, 5))
    u = velocity_field(m.xyz, seed=11, M=8)
    f = random_fourier_field(m.xyz, seed=7, M=8)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, N)
    idx = np.sort(np.random.default_rng(N).choice(m.E, 12, replace=False))
    idx[-1] = m.E - 1
    sel = torch.as_tensor(idx, device="cuda")
    ref = convect(np.moveaxis(u[:, idx], 0, 2), f[idx], m.xyz[idx], N, dealias=True)
    fields = np.concatenate([f[None], u])
    for dt, tol in ((torch.float64, 1e-12), (torch.float32, 2e-5)):
        out = sem.advect(M, dev(u, dt), dev(f, dt), rule="dealias")[sel]
        assert relmax(out.double().cpu().numpy(), ref) <= tol, dt
        many = sem.advect(M, dev(u, dt), dev(fields, dt), rule="dealias")[:, sel]
        assert relmax(many[0].double().cpu().numpy(), ref) <= tol, dt
        ref3 = convect(np.moveaxis(u[:, idx], 0, 2), u[2, idx], m.xyz[idx], N, dealias=True)
        assert relmax(many[3].double().cpu().numpy(), ref3) <= tol, dt


def test_errors():
    N = 3
    m, u, f = _case(N)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, N)
    lib = L.load()
    ud, fd = dev(u), dev(f)
    out = torch.empty_like(fd)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # rule not set up yet
    assert lib.sem_advect(M.handle, 1, ptr(ud), ptr(fd), ptr(out), 0, s) == L.SEM_EINVAL
    M.setup_advection("dealias")
    assert lib.sem_advect(M.handle, 1, ptr(ud), ptr(fd), ptr(out), 0, s) == L.SEM_OK
    assert lib.sem_advect(M.handle, 0, ptr(ud), ptr(fd), ptr(out), 0, s) == L.SEM_EINVAL
    assert lib.sem_advect(M.handle, 2, ptr(ud), ptr(fd), ptr(out), 0, s) == L.SEM_EINVAL
    assert lib.sem_advect(M.handle, 1, ptr(ud), ptr(fd), ptr(fd), 0, s) == L.SEM_EINVAL
    assert lib.sem_advect(M.handle, 1, ptr(ud), ptr(fd), ptr(ud[1]), 0, s) == L.SEM_EINVAL
    assert lib.sem_advect(M.handle, 1, ptr(ud), ptr(fd), ptr(out), 2, s) == L.SEM_EINVAL
    assert lib.sem_advect(M.handle, 1, None, ptr(fd), ptr(out), 0, s) == L.SEM_EINVAL
    # a different description, and a mirrored (orientation-reversing) map
    xyz = np.ascontiguousarray(m.xyz)
    bad = L.MeshDesc(N, m.E - 1, xyz.ctypes.data_as(ctypes.c_void_p), None, None)
    assert lib.sem_setup_advection(M.handle, ctypes.byref(bad), 1, s) == L.SEM_EINVAL
    mir = np.ascontiguousarray(xyz * np.array([-1.0, 1.0, 1.0]))
    desc = L.MeshDesc(N, m.E, mir.ctypes.data_as(ctypes.c_void_p), None, None)
    assert lib.sem_setup_advection(M.handle, ctypes.byref(desc), 1, s) == L.SEM_EINVAL
    assert b"detJ" in lib.sem_last_error()
    # the rule set up before is still in place
    again = sem.advect(M, ud, fd, rule="dealias")
    ref = convect(np.moveaxis(u, 0, 2), f, m.xyz, N, dealias=True)
    assert relmax(again.cpu().numpy(), ref) <= 1e-12
    with pytest.raises(ValueError):
        sem.advect(M, ud[:2], fd)
    with pytest.raises(sem.SemError):
        sem.advect(M, ud, fd, out=fd)


@pytest.mark.parametrize("rule", list(RULES))
@pytest.mark.parametrize("N", [2, 6, 7, 9])  # four- and eight-wave workgroups in both precisions
def test_advect_fields_equals_one_field_calls_and_oracle(N, rule):
    # a Boussinesq step's four advected fields: T and the velocity components
    m, u, T = _case(N, shape=(3, 2, 4))
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, N)
    fields = np.concatenate([T[None], u])
    for dt in (torch.float64, torch.float32):
        ud, fd = dev(u, dt), dev(fields, dt)
        many = sem.advect(M, ud, fd, rule=rule)
        for k in range(4):
            one = sem.advect(M, ud, fd[k].contiguous(), rule=rule)
            assert torch.equal(many[k], one)
    ref = np.stack([convect(np.moveaxis(u, 0, 2), fk, m.xyz, N, dealias=RULES[rule])
                    for fk in fields])
    got = sem.advect(M, dev(u), dev(fields), rule=rule).cpu().numpy()
    for k in range(4):
        assert relmax(got[k], ref[k]) <= 1e-12


def test_advect_fields_arguments():
    N = 3
    m, u, f = _case(N)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, N)
    M.setup_advection("dealias")
    lib = L.load()
    ud, fd = dev(u), dev(np.stack([f, 2 * f]))
    out = torch.full_like(fd, 7.0)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.sem_advect_fields(M.handle, 1, ptr(ud), 0, ptr(fd), ptr(out), 0, s) == L.SEM_OK
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())  # nf = 0 writes nothing
    assert lib.sem_advect_fields(M.handle, 1, ptr(ud), -1, ptr(fd), ptr(out), 0, s) == \
        L.SEM_EINVAL
    # out[0] overlapping f[1]
    assert lib.sem_advect_fields(M.handle, 1, ptr(ud), 2, ptr(fd), ptr(fd[1]), 0, s) == \
        L.SEM_EINVAL
    assert lib.sem_advect_fields(M.handle, 1, ptr(ud), 2, ptr(fd), ptr(out), 0, s) == L.SEM_OK
    torch.cuda.synchronize()
    assert torch.allclose(out[1], 2 * out[0], rtol=1e-14, atol=0)


@pytest.mark.parametrize("rule", list(RULES))
@pytest.mark.parametrize("N", [4, 7])
def test_advect_matches_oracle_on_sheared_affine_elements(N, rule):
    """Separate affine elements x = c + M r with full, non-symmetric M
    (rotated and sheared): the metric dr_a/dx_d has no zero entry, so an
    index mistake in the kernel's factors or their use would show."""
    rng = np.random.default_rng(40 + N)
    xi = reference_node_placement(N)
    k, j, i = np.meshgrid(xi, xi, xi, indexing="ij")
    r = np.stack([i.ravel(), j.ravel(), k.ravel()], -1)
    E = 6
    xyz = np.empty((E, r.shape[0], 3))
    for e in range(E):
        Q, R = np.linalg.qr(rng.standard_normal((3, 3)))
        Q = Q * np.sign(np.diag(R))
        if np.linalg.det(Q) < 0:
            Q[:, 0] = -Q[:, 0]
        S = np.diag(rng.uniform(0.3, 0.7, 3))
        S[0, 1], S[0, 2], S[1, 2] = rng.uniform(-0.25, 0.25, 3)
        xyz[e] = rng.uniform(-1, 1, 3) + r @ (Q @ S).T
    gid = np.arange(E * r.shape[0], dtype=np.int64).reshape(E, -1)
    u = rng.standard_normal((3, E, r.shape[0]))
    f = rng.standard_normal((E, r.shape[0]))
    M = sem.Mesh(xyz, gid, None, N)
    M.setup_advection(rule)
    G = M.advection_factors(rule).cpu().numpy()
    assert relmax(G, geometric_factors_q(xyz, N, RULES[rule]).reshape(E, 9, -1)) <= 1e-12
    out = sem.advect(M, dev(u), dev(f), rule=rule).cpu().numpy()
    ref = convect(np.moveaxis(u, 0, 2), f, xyz, N, dealias=RULES[rule])
    assert relmax(out, ref) <= 1e-12
