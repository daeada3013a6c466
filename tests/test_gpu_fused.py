"""The one-sweep product pair (w, y) = (A p, A^T A p) against float64 products.

Both sums run in float64 on float32 data, so the bound is the recursive
summation bound in float64 (Higham, Section 3.1): |w - A p| <= n u |A||p|
componentwise, and y = A^T w adds m u |A|^T |w| plus the propagated error of w.
"""
import numpy as np
import pytest

from paper_2104_10785_amd import gkb

from .gpu_util import banner, device, to_dev, to_host

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53

# (m, n, pad): one row per workgroup, ragged row shares, a single 16-byte group,
# every launch shape (several rows per step for short rows, up to 1024 threads
# with several groups each for long ones), the largest n, padded rows
SHAPES = [(1, 4, 0), (100, 8, 0), (257, 512, 4), (4000, 1000, 0), (3001, 2044, 0), (20000, 2048, 0),
          (3000, 4096, 4), (2500, 8000, 0), (1500, 12000, 0), (1200, 16380, 0), (5000, 20000, 8),
          (777, 24576, 0), (70000, 100, 0), (1, 20000, 0), (257, 19996, 4), (3001, 16388, 0),
          # the pipelined form near its LDS limit (the staged w of 3907 rows per
          # workgroup), and past it (4883 rows: the per-row barrier form)
          (4_000_000, 4, 0), (5_000_000, 4, 0),
          # team sweeps (rows longer than one workgroup holds): just past the
          # limit, uneven slices, a single row, padded rows, one row per team,
          # the longest rows (32 members), many rows per team
          (1000, 24580, 0), (600, 30000, 4), (1, 30000, 0), (300, 80004, 8), (40, 100000, 0),
          (50, 262144, 0), (8000, 40000, 0)]


def _padded(a, pad):
    m, n = a.shape
    out = np.zeros((m, n + pad), dtype=a.dtype)
    out[:, :n] = a
    return out


@pytest.mark.parametrize("shape", SHAPES)
def test_fused_products(shape):
    device()
    m, n, pad = shape
    banner(f"fused sweep {m}x{n} pad={pad}")
    rng = np.random.default_rng(m + 3 * n + pad)
    A = rng.standard_normal((m, n)).astype(np.float32)
    p = rng.standard_normal(n).astype(np.float32)
    Ad = to_dev(_padded(A, pad))[:, :n]
    w, y = gkb.gkb_matvec_fused(Ad, to_dev(p))
    w, y = to_host(w), to_host(y)
    A64, p64 = A.astype(np.float64), p.astype(np.float64)
    wref = A64 @ p64
    wabs = np.abs(A64) @ np.abs(p64)
    assert np.all(np.abs(w - wref) <= n * U64 * wabs + 1e-300)
    yref = A64.T @ wref
    ybound = (m + n + 1) * U64 * (np.abs(A64).T @ wabs) + 1e-300
    assert np.all(np.abs(y - yref) <= ybound)
    w2, y2 = gkb.gkb_matvec_fused(Ad, to_dev(p))
    assert np.array_equal(to_host(w2), w) and np.array_equal(to_host(y2), y)


BF16_SHAPES = [(1, 8, 0), (300, 1000, 8), (2000, 2048, 0), (3001, 4096, 0), (1500, 8000, 8), (1200, 16384, 0),
               (5000, 20000, 8), (777, 24576, 0), (70000, 96, 0), (4_000_000, 8, 0), (5_000_000, 8, 0),
               (500, 30000, 0), (200, 80000, 8), (3, 262144, 0)]


@pytest.mark.parametrize("shape", BF16_SHAPES)
def test_fused_products_bf16(shape):
    """bfloat16 A (8 per 16-byte group, widened exactly): each thread adds its
    at most 24 products of a row in float32 before the float64 reduction (as
    the two-product bfloat16 path does), so w carries a float32 bound
    32 u32 |A||p|; y must be A^T w for the w returned, with float64 sums."""
    import torch
    from oracle import bf16 as obf16
    device()
    m, n, pad = shape
    banner(f"fused sweep bf16 {m}x{n} pad={pad}")
    rng = np.random.default_rng(m + 5 * n + pad)
    bits = obf16.to_bf16_bits(rng.standard_normal((m, n)).astype(np.float32))
    A64 = obf16.from_bf16_bits(bits)
    p = rng.standard_normal(n).astype(np.float32)
    Ad = to_dev(_padded(bits.view(np.int16), pad)).view(torch.bfloat16)[:, :n]
    w, y = gkb.gkb_matvec_fused(Ad, to_dev(p))
    w, y = to_host(w), to_host(y)
    p64 = p.astype(np.float64)
    wref = A64 @ p64
    wabs = np.abs(A64) @ np.abs(p64)
    assert np.all(np.abs(w - wref) <= (32 * 2.0 ** -24 + n * U64) * wabs + 1e-300)
    yref = A64.T @ w
    assert np.all(np.abs(y - yref) <= (m + 1) * U64 * (np.abs(A64).T @ np.abs(w)) + 1e-300)


def test_fused_rejects_shapes():
    device()
    banner("fused sweep shape checks")
    for shape in [(10, 6), (10, 262148)]:
        Ad = to_dev(np.ones(shape, dtype=np.float32))
        with pytest.raises(gkb.GkbError):
            gkb.gkb_matvec_fused(Ad, to_dev(np.ones(shape[1], dtype=np.float32)))
    Ad = to_dev(np.ones((10, 8), dtype=np.float64))
    with pytest.raises(gkb.GkbError):
        gkb.gkb_matvec_fused(Ad, to_dev(np.ones(8)))
    import torch
    Ab = to_dev(np.ones((10, 12), dtype=np.float32)).to(torch.bfloat16)   # n not a multiple of 8
    with pytest.raises(gkb.GkbError):
        gkb.gkb_matvec_fused(Ab, to_dev(np.ones(12, dtype=np.float32)))
