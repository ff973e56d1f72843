"""CPU checks of the error model behind the l2 exact pass on the BF16 matrix
cores (two-term split of every float32 coordinate; nnmin_split.hip).

The certificate of that pass rests on three facts about the split
v = h + m + r, h = bf16(v), m = bf16(v - h), each round to nearest even:
v - h is exact in float32, |m| <= 2^-8 (1 + 2^-8) |v| and |r| <= 2^-16 |v|;
and on the resulting bound on the dropped terms of the dot product,
|x.b - (xh.bh + xm.bh + xh.bm)| <= 3.03 * 2^-16 |x| |b| (three products) and
|x.b - (xh + xm).(bh + bm)| <= 2.01 * 2^-16 |x| |b| (four products).  BF16
round-to-nearest-even is emulated on the float32 bit pattern here; products
and sums are taken in float64 and Fraction, independently of the kernel.
"""

import math
from fractions import Fraction

import numpy as np
import pytest


def bf16(v):
    """Round float32 values to BF16 (nearest, ties to even), as float32."""
    u = np.ascontiguousarray(v, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u & 0xFFFFFFFF).astype(np.uint32).view(np.float32)


def split(v):
    v = np.asarray(v, np.float32)
    h = bf16(v)
    m = bf16((v - h).astype(np.float32))
    return h, m


def inputs():
    rng = np.random.default_rng(0)
    cases = [rng.standard_normal((64, 128)),
             rng.uniform(-1e6, 1e6, (64, 128)),
             np.exp(rng.uniform(-80, 80, (64, 128))) * rng.choice([-1, 1], (64, 128)),
             # values just off BF16 rounding boundaries
             (1.0 + (rng.integers(0, 256, (64, 128)) + 0.5) / 256.0) *
             2.0 ** rng.integers(-20, 20, (64, 128))]
    return [c.astype(np.float32) for c in cases]


def test_bf16_rounding_matches_definition():
    """Spot-check the emulation against exact nearest-even rounding."""
    rng = np.random.default_rng(1)
    v = (rng.standard_normal(2000) * 10.0 ** rng.integers(-10, 10, 2000)).astype(np.float32)
    h = bf16(v)
    for a, b in zip(v.tolist(), h.tolist()):
        fa = Fraction(a)
        e = math.frexp(a)[1] - 1                 # 2^e <= |a| < 2^(e+1)
        ulp = Fraction(2) ** (e - 7)             # spacing of 8-bit significands there
        lo = (fa / ulp).__floor__() * ulp
        cands = sorted([lo, lo + ulp], key=lambda c: (abs(c - fa), (c / ulp) % 2))
        assert Fraction(b) == cands[0]


@pytest.mark.parametrize("idx", range(4))
def test_split_facts(idx):
    v = inputs()[idx].ravel()
    h, m = split(v)
    d32 = (v - h).astype(np.float32)
    assert np.array_equal(d32.astype(np.float64), v.astype(np.float64) - h.astype(np.float64))
    av = np.abs(v.astype(np.float64))
    assert np.all(np.abs(m.astype(np.float64)) <= 2.0 ** -8 * (1 + 2.0 ** -8) * av)
    r = v.astype(np.float64) - h.astype(np.float64) - m.astype(np.float64)
    assert np.all(np.abs(r) <= 2.0 ** -16 * av)


@pytest.mark.parametrize("idx", range(4))
def test_dropped_terms_bound(idx):
    X = inputs()[idx]
    B = inputs()[(idx + 1) % 4][::-1].copy()
    for x, b in zip(X, B):
        xh, xm = split(x)
        bh, bm = split(b)
        x64, b64 = x.astype(np.float64), b.astype(np.float64)
        exact = sum(Fraction(float(p)) * Fraction(float(q)) for p, q in zip(x64, b64))
        three = sum(Fraction(float(p)) * Fraction(float(q))
                    for p, q in zip(np.concatenate([xh, xm, xh]), np.concatenate([bh, bh, bm])))
        four = three + sum(Fraction(float(p)) * Fraction(float(q)) for p, q in zip(xm, bm))
        norm = float(np.linalg.norm(x64) * np.linalg.norm(b64))
        assert abs(float(exact - three)) <= 3.03 * 2.0 ** -16 * norm
        assert abs(float(exact - four)) <= 2.01 * 2.0 ** -16 * norm


def test_bound_is_nearly_attained():
    """Coordinates whose split leaves the largest residuals: the observed
    error of the three-product form reaches a fair fraction of the bound, so
    the bound is not vacuous (a dropped term in the analysis would show)."""
    k = np.arange(64)
    # v = 1 + 2^-9 + 2^-18 (times 1 or 2): h = 1, m = 2^-9, r = 2^-18, so
    # xm.bm and the residual terms are all of the order the bound allows
    x = np.full(64, 1.0 + 2.0 ** -9 + 2.0 ** -18, np.float32) * (1 + (k % 3 == 0))
    b = x.copy()
    xh, xm = split(x)
    exact = float(np.dot(x.astype(np.float64), b.astype(np.float64)))
    three = float(np.dot(np.concatenate([xh, xm, xh]).astype(np.float64),
                         np.concatenate([xh, xh, xm]).astype(np.float64)))
    norm = float(np.linalg.norm(x.astype(np.float64)) ** 2)
    ratio = abs(exact - three) / (2.0 ** -16 * norm)
    assert 0.05 < ratio <= 3.03
