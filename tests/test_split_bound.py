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


# ------------------------------------------------ the certificate bound E ---
#
# The l2 exact pass starts each accumulator at -|b|^2 / 2, with |b|^2 the
# float32 fma chain over b's coordinates, and adds the BF16 split products;
# the certificate needs |computed score - (|b|^2 - 2 x.b)| <= E for the E the
# library computes (chamfer_split_score_bound, the function the kernels call).
# Below, the accumulation is emulated under the model the bound assumes
# (every product added with one float32 rounding to nearest, in the order
# of the kernel's K steps) on inputs built to make each error source as
# large as it can be, and the error is measured exactly with Fractions.

U = 2.0 ** -24


def f32_round(fr):
    """Round a Fraction to the nearest float32 (ties to even), exactly."""
    if fr == 0:
        return np.float32(0.0)
    sign = -1 if fr < 0 else 1
    mag = abs(fr)
    e = math.frexp(float(mag))[1] - 1
    while Fraction(2) ** e > mag:
        e -= 1
    while Fraction(2) ** (e + 1) <= mag:
        e += 1
    spacing = Fraction(2) ** (max(e, -126) - 23)
    q = mag / spacing
    n = q.numerator // q.denominator
    r = q - n
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and n % 2 == 1):
        n += 1
    return np.float32(sign * float(n * spacing))


def fma_norm(b, d):
    """float32 fma chain of b_k^2 over k ascending (the row norm)."""
    acc = np.float32(0.0)
    for k in range(d):
        acc = f32_round(Fraction(float(b[k])) ** 2 + Fraction(float(acc)))
    return acc


def dpad(d):
    return 32 if d <= 32 else 64 if d <= 64 else 128 if d <= 128 else 256


def emulate_score(x, b, d, terms):
    """Score -2 v of the kernel's accumulation of (x, b) under the model."""
    dp = dpad(d)
    xp = np.zeros(dp, np.float32)
    bp = np.zeros(dp, np.float32)
    xp[:d], bp[:d] = x, b
    xh, xm = split(xp)
    bh, bm = split(bp)
    A = np.float32(-0.5) * fma_norm(b, d)
    kq = dp // 4
    order = [g * kq + 8 * s + t for s in range(kq // 8) for g in range(4) for t in range(8)]
    hi, lo = A, np.float32(0.0)
    small = [(bh, xm), (bm, xh)] + ([(bm, xm)] if terms == 4 else [])
    for s in range(kq // 8):
        ks = order[32 * s:32 * s + 32]
        for k in ks:
            hi = np.float32(hi + np.float32(bh[k] * xh[k]))
        for P, Q in small:
            for k in ks:
                if terms == 4:
                    lo = np.float32(lo + np.float32(P[k] * Q[k]))
                else:
                    hi = np.float32(hi + np.float32(P[k] * Q[k]))
    v = np.float32(hi + lo) if terms == 4 else hi
    return -2.0 * float(v)


def exact_score(x, b):
    xf = [Fraction(float(t)) for t in x]
    bf = [Fraction(float(t)) for t in b]
    return sum(t * t for t in bf) - 2 * sum(p * q for p, q in zip(xf, bf))


def query_norm(x):
    """|x|^2 as the split kernel computes it (4-term fma chains, then a tree);
    it only enters E through |x|, inflated by rho."""
    return np.float32(np.sum(x.astype(np.float64) ** 2))


def rounded_up_row(d, rng):
    """b_k = 1 + j_k 2^-23 chosen one coordinate at a time so that every step
    of the fma chain rounds up by nearly half a float32 spacing: the row norm
    the accumulator starts from is as large as the chain allows."""
    j = np.arange(4096, dtype=np.int64)
    sq = (1 << 46) + (j << 24) + j * j   # b^2 in units of 2^-46
    acc = 0                              # the chain's value in the same units
    b = np.zeros(d, np.float32)
    for k in range(d):
        V = acc + sq
        e = int(V.max()).bit_length() - 1
        sp = 1 << max(e - 23, 0)
        r = V % sp
        up = np.where(r * 2 > sp, sp - r, np.where(r * 2 == sp, 0, -r))
        pick = int(np.argmax(up))
        b[k] = np.float32(1.0 + float(j[pick]) * 2.0 ** -23)
        acc = int(V[pick] + up[pick])
    return b


def lost_products_query(b, d):
    """x_k = the largest BF16 value whose product with bf16(b_k) stays below
    half a float32 spacing of the accumulator's start: every leading product
    is lost to rounding, in the same direction as the rounded-up norm."""
    A = abs(float(np.float32(-0.5) * fma_norm(b, d)))
    half = 2.0 ** (math.frexp(A)[1] - 1 - 24)
    bh, _ = split(b)
    x = np.zeros(d, np.float32)
    for k in range(d):
        # BF16 values are float32 values with 16 zero low bits: truncate, then
        # step down one BF16 spacing while the product reaches half
        bits = int(np.float32(half / float(bh[k])).view(np.uint32)) & 0xFFFF0000
        while float(np.uint32(bits).view(np.float32)) * float(bh[k]) >= half:
            bits -= 0x10000
        x[k] = np.uint32(bits).view(np.float32)
    return x


def old_bound(d, terms, xn2, b2max):
    """E without the row-norm rounding term (for the regression check)."""
    rho = (d + 4) * U * 1.1
    dp = dpad(d)
    crel = ((terms == 4 and 1 or 3) * dp + 8) * U * 1.1
    ctr = (2.01 if terms == 4 else 3.03) / 65536.0 * 1.1
    b2m = b2max * (1 + rho)
    bm, xa = math.sqrt(b2m), math.sqrt(xn2 * (1 + rho))
    return crel * (b2m + 2 * xa * bm) + 2 * ctr * xa * bm


@pytest.mark.parametrize("d", [12, 64, 128, 200, 256])
@pytest.mark.parametrize("terms", [3, 4])
def test_certificate_bound_worst_cases(d, terms):
    import paper_2307_03043_amd as ch
    rng = np.random.default_rng(d * 10 + terms)
    b_up = rounded_up_row(d, rng)
    cases = {
        # query at the origin, the row's norm rounded up at every step
        "origin": (np.zeros(d, np.float32), b_up),
        # every leading product lost to rounding, same sign as the norm error
        "lost": (lost_products_query(b_up, d), b_up),
        # the query far larger than the row, and the reverse
        "big_x": ((rng.standard_normal(d) * 1e3).astype(np.float32),
                  rng.standard_normal(d).astype(np.float32)),
        "big_b": (rng.standard_normal(d).astype(np.float32) * np.float32(1e-3),
                  (rng.standard_normal(d) * 1e2).astype(np.float32)),
        # a common offset: |b|^2 and 2 x.b cancel almost entirely
        "offset": ((1e4 + rng.standard_normal(d)).astype(np.float32),
                   (1e4 + rng.standard_normal(d)).astype(np.float32)),
    }
    for name, (x, b) in cases.items():
        err = abs(Fraction(emulate_score(x, b, d, terms)) - exact_score(x, b))
        b2max = float(fma_norm(b, d))
        xn2 = float(query_norm(x))
        E = ch.chamfer_split_score_bound(d, terms, xn2, b2max)
        assert float(err) <= E, (name, float(err), E)
        if name == "lost" and terms == 4 and d in (64, 128, 256):
            # the norm's rounding is a real part of the error: without its
            # term the bound fails on this row (|b|^2 / 2 just above a power
            # of two, where a lost product is a full half spacing)
            assert float(err) > old_bound(d, terms, xn2, b2max), (float(err), E)
        if name == "lost":
            # the construction reaches the accumulation model's regime
            assert float(err) > 0.5 * (dpad(d) if terms == 4 else d) * U * b2max * 0.5


def test_certificate_bound_rejects_bad_arguments():
    import paper_2307_03043_amd as ch
    assert ch.chamfer_split_score_bound(0, 3, 1.0, 1.0) == -1.0
    assert ch.chamfer_split_score_bound(257, 3, 1.0, 1.0) == -1.0
    assert ch.chamfer_split_score_bound(128, 2, 1.0, 1.0) == -1.0
    assert math.isinf(ch.chamfer_split_score_bound(128, 3, 1.0, float("inf")))
