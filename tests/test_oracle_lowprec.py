"""Pins of the oracle's 16-bit contraction variant of the element operator.

The preconditioner may run the operator's derivative contractions with
bfloat16 or IEEE half operands and exact accumulation (Sec. 2.2 keeps most
preconditioner work in reduced precision for bandwidth; the 16-bit operand
form is this implementation's matrix-core option).  Pins: the two roundings
against torch's own conversions, the power-of-two block scale, and the
a-priori rounding error bound against the FP64 operator, sharp to a small
factor, including residual-sized inputs far below half precision's normal
range.  Where the roundings are placed (D, the u block, each v_a block) is
this design's definition and is not fixed by the paper.
"""

import numpy as np
import pytest
import torch

from oracle.geometry import geometric_factors
from oracle.operator import (block_scale, local_apply, local_apply_lowprec,
                             local_apply_majorant, round_to_format)
from sem_inputs import box_mesh, random_local_normal

UNIT = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11}
TORCH = {"bf16": torch.bfloat16, "fp16": torch.float16}


def _torch_round(x32, fmt):
    return torch.from_numpy(x32).to(TORCH[fmt]).to(torch.float64).numpy()


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_rounding_matches_torch(fmt):
    rng = np.random.default_rng(11)
    hi = 30.0 if fmt == "bf16" else 4.0
    x = rng.standard_normal(20000) * 10.0 ** rng.uniform(-hi, hi, 20000)
    x32 = x.astype(np.float32)
    # exact ties between two neighbours of the target format, both parities
    drop = 16 if fmt == "bf16" else 13
    base = rng.uniform(0.5, 2.0, 4000).astype(np.float32).view(np.uint32)
    base &= np.uint32(~((1 << drop) - 1) & 0xFFFFFFFF)
    ties = (base | np.uint32(1 << (drop - 1))).view(np.float32)
    x32 = np.concatenate([x32, ties, -ties, np.float32([0.0, -0.0, 1.0])])
    np.testing.assert_array_equal(round_to_format(x32, fmt), _torch_round(x32, fmt))


def test_block_scale_puts_block_maximum_in_range():
    rng = np.random.default_rng(12)
    X = rng.standard_normal((50, 64)) * 10.0 ** rng.uniform(-12, 3, (50, 1))
    X[7] = 0.0
    s = block_scale(X, "fp16")
    m = np.max(np.abs(X), axis=1)
    ok = m > 0
    scaled = m[ok] * s[ok]
    assert np.all(scaled >= 2.0 ** 14) and np.all(scaled < 2.0 ** 15)
    assert np.all(np.log2(s) == np.round(np.log2(s)))
    assert s[7] == 1.0
    np.testing.assert_array_equal(block_scale(X, "bf16"), np.ones(50))
    # the exponent stays in FP32's normal range for extreme blocks
    ext = block_scale(np.array([[1e-38], [3e38]]), "fp16")
    np.testing.assert_array_equal(ext, [2.0 ** 126, 2.0 ** -113])


def _problem(N, shape=(2, 2, 4), scale=1.0, seed=13):
    m = box_mesh(N, shape, jitter=0.1, jitter_seed=4, dirichlet="none",
                 deform=dict(a=0.15, seed=2, kind="walls"), z_ratio=4.0)
    G, B, _ = geometric_factors(m.xyz, N)
    u = (scale * random_local_normal((m.E, m.P), seed=seed)).astype(np.float32).astype(np.float64)
    k = np.exp(0.3 * random_local_normal((m.E, m.P), seed=seed + 1))
    return m, G, B, u, k


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
@pytest.mark.parametrize("N", [1, 3, 7, 9])
@pytest.mark.parametrize("scale", [1.0, 1e-9])
def test_lowprec_error_bound_and_sharpness(fmt, N, scale):
    m, G, B, u, k = _problem(N, scale=scale)
    for kk, h2 in ((None, 0.0), (k, 0.7)):
        w = local_apply(u, G, B, N, k=kk, h2=h2)
        w16 = local_apply_lowprec(u, G, B, N, fmt, k=kk, h2=h2)
        M = local_apply_majorant(u, G, N, k=kk)
        ratio = np.abs(w16 - w) / (UNIT[fmt] * M)
        # two roundings of D, one of u and one of v_a: 4u + O(u^2)
        assert ratio.max() <= 4.1, ratio.max()
        # and the roundings do happen
        assert ratio.max() >= 0.2, ratio.max()


def test_unscaled_half_precision_would_lose_residual_sized_inputs():
    """The block scale is what keeps small inputs: rounding them straight to
    half precision flushes them (guards against dropping the scale)."""
    N = 5
    _, G, B, u, _ = _problem(N, scale=1e-9)
    w = local_apply(u, G, B, N)
    raw = round_to_format(u, "fp16")
    assert np.count_nonzero(raw) < 0.1 * raw.size
    w16 = local_apply_lowprec(u, G, B, N, "fp16")
    assert np.linalg.norm(w16 - w) <= 1e-2 * np.linalg.norm(w)
