"""sem_cheb_apply_noalloc (work space in the library's fixed device array)
against sem_cheb_apply, through the C ABI.

Both entry points run the same kernels in the same order on the same data
(Jacobi inverse, free-node averages, Chebyshev recurrence, operator), only
with different work buffers, and none of these kernels sums in an order that
depends on the buffers' addresses: the outputs must be identical bit for bit.
The FP64 result is also held to the oracle's Chebyshev apply (1e-12).
Calls run back to back on one device, each later one on a smaller mesh than
the one before, so stale contents of the shared array from a larger call
would show.
"""

import ctypes

import numpy as np
import pytest
import torch

import oracle
from sem_inputs import config_mesh
from sem_inputs.fields import random_fourier_field

pytestmark = pytest.mark.gpu

sem = pytest.importorskip("paper_2501_13240_amd")


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _case(cfg, N, shape, seed):
    m, _ = config_mesh(cfg, N=N, shape=shape)
    M = sem.Mesh(m.xyz, m.gid, m.dirichlet, m.N)
    return m, M, np.random.default_rng(seed)


def _both(M, r, lmax, k, h2, order, prec):
    z_ref = sem.cheb_apply(M, r, lmax, k=k, h2=h2, order=order, prec=prec)
    z_na = sem.cheb_apply_noalloc(M, r, lmax, k=k, h2=h2, order=order, prec=prec)
    torch.cuda.synchronize()
    return z_ref.cpu().numpy(), z_na.cpu().numpy()


def test_noalloc_chebyshev_matches_allocating_entry_point():
    # (workload, order N, elements, k variable?, h2, Chebyshev order, precision);
    # the meshes shrink from one call to the next
    cases = [
        (1, 7, (4, 4, 4), True, 0.0, 3, "fp64"),
        (1, 5, (3, 3, 3), False, 0.0, 3, "fp64"),
        (1, 7, (3, 3, 2), True, 1.0, 4, "fp32"),
        (1, 4, (2, 2, 2), False, 0.5, 2, "bf16_mfma"),
        (1, 3, (2, 2, 1), False, 0.0, 3, "fp16_mfma"),
    ]
    for i, (cfg, N, shape, var_k, h2, order, prec) in enumerate(cases):
        m, M, rng = _case(cfg, N, shape, 10 + i)
        print(f"case {i}: N={N} shape={shape} k={'var' if var_k else 'none'} h2={h2} "
              f"order={order} prec={prec}", flush=True)
        P = oracle.Problem(m.xyz, m.gid, m.dirichlet, m.N)
        kl = None
        if var_k:
            kl = np.exp(0.3 * random_fourier_field(m.xyz, seed=i))
        rf = rng.standard_normal(P.num.n_free)
        r = dev(P.num.to_local(rf))
        k = dev(kl) if kl is not None else None
        lmax = sem.lmax_estimate(M, k=k, h2=h2)
        z_ref, z_na = _both(M, r, lmax, k, h2, order, prec)
        assert np.array_equal(z_ref, z_na), np.abs(z_ref - z_na).max()
        if prec == "fp64":
            Pk = oracle.Problem(m.xyz, m.gid, m.dirichlet, m.N, k=kl, h2=h2)
            z_or = P.num.to_local(oracle.chebyshev_apply(Pk.apply, 1.0 / Pk.diag(), rf, order,
                                                         lmax))
            e = np.linalg.norm(z_na - z_or) / np.linalg.norm(z_or)
            print(f"  vs oracle: {e:.2e}")
            assert e <= 1e-12
        M.close()


def test_noalloc_chebyshev_allocates_nothing_and_rejects_large_meshes():
    _, M, _ = _case(1, 7, (3, 3, 3), 3)
    _, M2, _ = _case(1, 5, (2, 2, 2), 4)
    info2 = M2.info
    r = torch.randn(M.E, M.P, dtype=torch.float64, device="cuda")
    r = sem.gs(M, r)
    r2 = torch.randn(M2.E, M2.P, dtype=torch.float64, device="cuda")
    r2 = sem.gs(M2, r2)
    z2 = torch.empty_like(r2)
    # first calls on this device (the array's address is looked up, the
    # kernels' code is loaded)
    for prec in ("fp64", "fp32"):
        sem.cheb_apply_noalloc(M, r, 2.0, order=3, prec=prec)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for prec in ("fp64", "fp32"):
        sem.cheb_apply_noalloc(M2, r2, 2.0, order=3, prec=prec, out=z2)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0, (free0, free1)
    ref = sem.cheb_apply(M2, r2, 2.0, order=3, prec="fp32")
    assert torch.equal(ref, z2)
    assert info2["n_free"] > 0
    M.close()
    M2.close()

    # a mesh whose work vectors exceed the 64 MiB array: rejected, nothing written
    mb, _ = config_mesh(1, N=5, shape=(22, 22, 22))
    MB = sem.Mesh(mb.xyz, mb.gid, mb.dirichlet, mb.N)
    nL, nf = MB.info["n_local"], MB.info["n_free"]
    assert 8 * nL + 40 * nf > 64 << 20
    rb = torch.zeros(MB.E, MB.P, dtype=torch.float64, device="cuda")
    zb = torch.full_like(rb, 7.0)
    lib = MB._lib
    st = lib.sem_cheb_apply_noalloc(MB.handle, ctypes.c_void_p(rb.data_ptr()),
                                    ctypes.c_void_p(zb.data_ptr()), None, 0.0, 3, 2.0, 0, None)
    assert st == -1
    msg = lib.sem_last_error().decode()
    assert "bytes of work space" in msg, msg
    torch.cuda.synchronize()
    assert bool((zb == 7.0).all())
    MB.close()
