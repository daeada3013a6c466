"""Each HIP building block against a plain definition computed on the host.

Tolerances are the standard worst-case bounds for the arithmetic: a length-n
dot product accumulated in precision u has error at most n u sum |a_i x_i|
(recursive summation; Higham, Accuracy and Stability of Numerical
Algorithms, Section 3.1), and the reference is float64 on the same inputs.
"""
import numpy as np
import pytest

from oracle import bf16 as obf16
from oracle import philox
from paper_2104_10785_amd import gkb

from .gpu_util import banner, device, to_dev, to_host

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U64 = 2.0 ** -53

SHAPES = [(1000, 777), (513, 1), (1, 300), (2000, 1000), (4097, 1030), (64, 64)]


def _padded(a, pad):
    m, n = a.shape
    out = np.zeros((m, n + pad), dtype=a.dtype)
    out[:, :n] = a
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("pad", [0, 3, 8])
def test_matvec(dtype, shape, pad):
    import torch
    device()
    m, n = shape
    banner(f"matvec {dtype} {shape} pad={pad}")
    rng = np.random.default_rng(m * 7 + n + pad)
    A64 = rng.standard_normal((m, n))
    if dtype == "f64":
        Ah = A64
        Ad = to_dev(_padded(Ah, pad))[:, :n]
        xt = np.float64
        u = U64
    elif dtype == "f32":
        Ah = A64.astype(np.float32)
        Ad = to_dev(_padded(Ah, pad))[:, :n]
        xt = np.float32
        u = U32
    else:
        bits = obf16.to_bf16_bits(A64.astype(np.float32))
        Ah = obf16.from_bf16_bits(bits)
        Ad = to_dev(_padded(bits.view(np.int16), pad)).view(torch.bfloat16)[:, :n]
        xt = np.float32
        u = U32
    xn = rng.standard_normal(n).astype(xt)
    xm = rng.standard_normal(m).astype(xt)
    y = to_host(gkb.gkb_matvec(Ad, to_dev(xn), 0))
    ref = Ah.astype(np.float64) @ xn.astype(np.float64)
    bound = n * u * (np.abs(Ah) @ np.abs(xn.astype(np.float64))) + 1e-300
    assert np.all(np.abs(y - ref) <= bound)
    yt = to_host(gkb.gkb_matvec(Ad, to_dev(xm), 1))
    reft = Ah.astype(np.float64).T @ xm.astype(np.float64)
    boundt = m * u * (np.abs(Ah).T @ np.abs(xm.astype(np.float64))) + 1e-300
    assert np.all(np.abs(yt - reft) <= boundt)
    # deterministic: a second run is bitwise identical
    yt2 = to_host(gkb.gkb_matvec(Ad, to_dev(xm), 1))
    assert np.array_equal(yt, yt2)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("MKN,pad", [((1000, 30, 10), 0), ((20000, 121, 50), 0), ((17, 5, 3), 0),
                                     ((333, 64, 64), 0), ((64, 1, 100), 0), ((5000, 86, 85), 0),
                                     ((50000, 121, 50), 48), ((4099, 200, 13), 5), ((130, 33, 129), 3),
                                     ((1001, 0, 4), 0)])
def test_gemm_tall(dtype, MKN, pad):
    """Against a float64 product; several 64 x 64 tiles, ragged M, K and N, K
    across several 32-wide chunks, padded leading dimensions (unaligned ones take
    the element-wise path) and K = 0."""
    import torch
    device()
    M, K, N = MKN
    banner(f"gemm {dtype.__name__} {MKN} pad={pad}")
    rng = np.random.default_rng(M + K + N)
    At = rng.standard_normal((K, M)).astype(dtype)  # column-major M x K
    Bt = rng.standard_normal((N, K)).astype(dtype)  # column-major K x N
    Ad = torch.zeros((K, M + pad), dtype=torch.float64 if dtype == np.float64 else torch.float32,
                     device="cuda:0")
    Ad[:, :M] = to_dev(At)
    Ct = to_host(gkb.gkb_gemm_tall(Ad[:, :M], to_dev(Bt)))  # (N, M)
    ref = (At.T.astype(np.float64) @ Bt.T.astype(np.float64)).T
    u = U64 if dtype == np.float64 else U32
    bound = K * u * (np.abs(Bt.astype(np.float64)) @ np.abs(At.astype(np.float64))) + 1e-300
    assert np.all(np.abs(Ct - ref) <= bound)


def test_cast_bf16_bit_exact():
    import torch
    device()
    banner("cast_bf16")
    rng = np.random.default_rng(0)
    with np.errstate(over="ignore", under="ignore"):
        x = (rng.standard_normal((300, 257)) * 10.0 ** rng.integers(-45, 39, (300, 257))).astype(np.float32)
    special = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8,
                        1.0 + 2 ** -8 + 2 ** -20, 3.4e38, 1e-45, -1e-40], dtype=np.float32)
    x[0, : special.size] = special
    d = to_host(gkb.gkb_cast_bf16(to_dev(x)).view(torch.int16)).view(np.uint16)
    want = obf16.to_bf16_bits(x)
    nan = np.isnan(x)
    assert np.array_equal(d[~nan], want[~nan])
    assert np.all((d[nan] & 0x7F80) == 0x7F80) and np.all((d[nan] & 0x7F) != 0)


def test_device_start_vector_matches_oracle():
    device()
    banner("philox start vector")
    for m, seed in [(1, 0), (1000, 7), (123457, 2 ** 40 + 5)]:
        q = to_host(gkb.gkb_start_vector(m, seed))
        ref = philox.start_vector(m, seed)
        # same integers, same formula; only log/cos rounding may differ
        assert np.max(np.abs(q - ref)) < 1e-13


@pytest.mark.parametrize("MKN", [(1000, 777, 50), (513, 1, 7), (2000, 1030, 100), (130, 33, 64), (64, 64, 65),
                                 (20000, 5000, 32), (3000, 777, 128), (3001, 800, 129), (20000, 5000, 100),
                                 (63, 31, 112), (65, 64, 113), (20000, 5000, 31), (1000, 63, 32)])
@pytest.mark.parametrize("pad", [0, 1])
def test_gemm_rowmajor(MKN, pad):
    device()
    M, K, N = MKN
    banner(f"gemm_rowmajor {MKN} pad={pad}")
    rng = np.random.default_rng(M + K + N + pad)
    A = rng.standard_normal((M, K + pad)).astype(np.float32)
    Bt = rng.standard_normal((N, K + pad)).astype(np.float32)
    Ad = to_dev(A)[:, :K]
    Bd = to_dev(Bt)[:, :K]
    Ct = to_host(gkb.gkb_gemm_rowmajor(Ad, Bd))
    if N <= 32:
        # the narrow form adds two K halves into C: the same bits every time
        assert np.array_equal(to_host(gkb.gkb_gemm_rowmajor(Ad, Bd)), Ct)
    A64 = A[:, :K].astype(np.float64)
    B64 = Bt[:, :K].astype(np.float64).T
    ref = (A64 @ B64).T
    bound = K * U32 * (np.abs(B64).T @ np.abs(A64).T) + 1e-300
    assert np.all(np.abs(Ct - ref) <= bound)


@pytest.mark.parametrize("md", [(5000, 100), (3000, 17), (1, 3), (4097, 64)])
def test_gram(md):
    device()
    m, d = md
    banner(f"gram {md}")
    rng = np.random.default_rng(m + d)
    Wt = rng.standard_normal((d, m)).astype(np.float32)
    G = to_host(gkb.gkb_gram(to_dev(Wt)))
    W64 = Wt.astype(np.float64)
    ref = W64 @ W64.T
    bound = m * U64 * (np.abs(W64) @ np.abs(W64).T) + 1e-300
    assert np.all(np.abs(G - ref) <= bound)
