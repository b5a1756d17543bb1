"""The arithmetic of the split form (FP32 operands as three BF16 parts, six
part products per FP32 product), emulated in numpy on the CPU: the bounds the
kernels' accuracy rests on, and the direction of Eq. (1) computed that way
against the FP64 oracle."""
import math

import numpy as np

from oracle import svgd


def bf16(a):
    """Round FP32 values to BF16 (round to nearest, ties to even), as FP32."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + ((u >> 16) & 1) + 0x7FFF) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def split3(v):
    v = np.asarray(v, dtype=np.float32)
    hi = bf16(v)
    r = (v - hi).astype(np.float32)
    mid = bf16(r)
    lo = bf16((r - mid).astype(np.float32))
    return hi, mid, lo


def test_the_differences_are_exact_and_three_parts_hold_fp32_exactly():
    """An FP32 value has 24 significant bits and each part takes 8 (the
    rounding residuals are multiples of the value's ulp, at most half a BF16
    ulp): hi + mid + lo is the value itself (normal values)."""
    rng = np.random.default_rng(0)
    v = (rng.standard_normal(200_000) * np.exp2(rng.integers(-60, 60, 200_000))).astype(np.float32)
    hi, mid, lo = split3(v)
    v64 = v.astype(np.float64)
    # v - hi and (v - hi) - mid are exact in FP32
    assert np.array_equal((v - hi).astype(np.float64), v64 - hi.astype(np.float64))
    r = (v - hi).astype(np.float32)
    assert np.array_equal((r - mid).astype(np.float64), r.astype(np.float64) - mid.astype(np.float64))
    assert np.array_equal(hi.astype(np.float64) + mid.astype(np.float64) + lo.astype(np.float64), v64)
    assert (np.abs(mid.astype(np.float64)) <= 2.0 ** -8 * np.abs(v64)).all()
    assert (np.abs(lo.astype(np.float64)) <= 2.0 ** -16 * np.abs(v64)).all()


def test_six_part_products_give_a_dot_product_within_fp32_rounding():
    """hh + hm + mh + hl + lh + mm of two 32-vectors, each product exact, the
    sum in FP64: within a few 2^-24 of sum |a_k b_k| of the exact dot."""
    rng = np.random.default_rng(1)
    pairs = ((0, 0), (0, 1), (1, 0), (0, 2), (2, 0), (1, 1))
    worst = 0.0
    for _ in range(2000):
        a = rng.standard_normal(32).astype(np.float32)
        b = rng.standard_normal(32).astype(np.float32)
        pa, pb = split3(a), split3(b)
        got = sum(float(np.dot(pa[i].astype(np.float64), pb[j].astype(np.float64))) for i, j in pairs)
        exact = float(np.dot(a.astype(np.float64), b.astype(np.float64)))
        worst = max(worst, abs(got - exact) / float(np.abs(a.astype(np.float64) * b).sum()))
    assert worst <= 4 * 2.0 ** -24


def _phi_split(th, g, h):
    """Eq. (1) as the split-form kernels compute it: centred rows, the Gram
    from six part products plus -|x_j|^2/2, K = 2^(c D) in FP32, K and V as
    three parts, six part products, FP32 sums (an FP64 sum rounded to FP32
    per 32-wide step stands in for the matrix cores' accumulation)."""
    N, d = th.shape
    pairs = ((0, 0), (0, 1), (1, 0), (0, 2), (2, 0), (1, 1))
    th, g = th.astype(np.float32), g.astype(np.float32)
    x = (th - th.mean(axis=0, dtype=np.float32)).astype(np.float32)
    nrm = (x * x).sum(axis=1, dtype=np.float32)
    xs = split3(x)
    s = np.tile((-0.5 * nrm)[None, :], (N, 1)).astype(np.float32)
    for i, j in pairs:
        s = (s + (xs[i].astype(np.float64) @ xs[j].astype(np.float64).T).astype(np.float32)).astype(np.float32)
    m = np.float32(2.0 * math.log2(math.e) / h)
    k = np.clip(np.exp2((m * s + (-0.5 * m * nrm)[:, None]).astype(np.float32)), 0, 1).astype(np.float32)
    c2 = np.float32(2.0 / h)
    v = np.concatenate([(g - c2 * x).astype(np.float32), np.ones((N, 1), np.float32)], axis=1)
    ks, vs = split3(k), split3(v)
    acc = np.zeros((N, d + 1), np.float32)
    for j0 in range(0, N, 32):
        for i, j in pairs:
            acc = (acc + (ks[i][:, j0:j0 + 32].astype(np.float64) @ vs[j][j0:j0 + 32].astype(np.float64))
                   .astype(np.float32)).astype(np.float32)
    return ((acc[:, :d] + c2 * x * acc[:, d:]) / N).astype(np.float64)


def test_split_direction_matches_the_oracle_at_fp32_level():
    for N, d in ((64, 12), (200, 30)):
        rng = np.random.default_rng(N + d)
        th = rng.standard_normal((N, d)).astype(np.float32).astype(np.float64)
        th[:, ::6] *= 0.1
        g = (rng.standard_normal((N, d)) * 50).astype(np.float32).astype(np.float64)
        h = svgd.bandwidth(th, 0.0)
        ref = svgd.svgd_phi(th, g, h)
        err = (np.abs(_phi_split(th, g, h) - ref) / (np.abs(ref).max(axis=0, keepdims=True) + 1e-30)).max()
        assert err < 5e-6, err
