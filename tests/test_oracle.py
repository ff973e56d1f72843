"""Pins for the CPU oracle: each test ties a piece of the oracle to something
other than the oracle itself -- an independent library implementation, a
closed form, a value derived by hand, or a statement the paper proves.

Where the oracle computes a plain definition (CH, nearest neighbours) it is
checked against scipy and hand-derived values; where it follows the paper's
randomized algorithms it is checked against the lemmas the paper proves
about them (collision probability of the grid hash, the l2->l1 embedding's
normalisation, D_a >= min_b d(a,b), unbiasedness and the variance bound of
the estimator, the outlier scenario of the experiments section).
"""

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.distance import cdist
from scipy import stats

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U32 = 2.0 ** -24  # unit roundoff of float32


# ---------------------------------------------------------------- Philox ---

def test_philox_matches_numpy(orc):
    """Philox4x64-10 vs numpy's own implementation (numpy increments the
    counter before producing each block)."""
    rng = np.random.default_rng(1)
    for _ in range(50):
        key = rng.integers(0, 2**63, size=2, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
        ctr = rng.integers(1, 2**63, size=4, dtype=np.uint64)
        bg = np.random.Philox(key=key, counter=ctr - np.array([1, 0, 0, 0], np.uint64))
        ref = bg.random_raw(4)
        np.testing.assert_array_equal(orc.philox4x64(ctr, key), ref)


# ---------------------------------------------------------- exact CH -------

def test_exact_hand_cases(orc):
    with open(os.path.join(GOLDEN, "hand_cases.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        A = np.array(c["A"], np.float32)
        B = np.array(c["B"], np.float32)
        for metric, key in ((1, "l1"), (2, "l2")):
            ch, _, _ = orc.chamfer_exact(A, B, metric)
            assert ch == pytest.approx(c[key], rel=1e-15, abs=1e-15)


@pytest.mark.parametrize("metric", [1, 2])
@pytest.mark.parametrize("d", [1, 3, 17])
def test_exact_vs_scipy(orc, metric, d):
    rng = np.random.default_rng(d * 10 + metric)
    A = rng.standard_normal((57, d)).astype(np.float32)
    B = rng.standard_normal((41, d)).astype(np.float32)
    ch, mind, arg = orc.chamfer_exact(A, B, metric)
    M = cdist(A.astype(np.float64), B.astype(np.float64),
              "cityblock" if metric == 1 else "euclidean")
    np.testing.assert_allclose(mind, M.min(axis=1), rtol=1e-13)
    np.testing.assert_array_equal(arg, M.argmin(axis=1))
    dist, _ = cKDTree(B.astype(np.float64)).query(A.astype(np.float64), k=1, p=metric)
    assert ch == pytest.approx(float(np.sum(dist)), rel=1e-12)


@pytest.mark.parametrize("metric", [1, 2])
def test_exact_invariants(orc, metric):
    rng = np.random.default_rng(5)
    A = rng.integers(-50, 50, size=(40, 4)).astype(np.float32)
    B = rng.integers(-50, 50, size=(33, 4)).astype(np.float32)
    ch, _, _ = orc.chamfer_exact(A, B, metric)
    assert orc.chamfer_exact(A, A, metric)[0] == 0.0
    # permutation of either set
    assert orc.chamfer_exact(A[::-1].copy(), B[rng.permutation(33)], metric)[0] == pytest.approx(ch, rel=1e-15)
    # integer translation (exact in float32) and scaling by 2 (exact)
    assert orc.chamfer_exact(A + 7, B + 7, metric)[0] == pytest.approx(ch, rel=1e-15)
    assert orc.chamfer_exact(2 * A, 2 * B, metric)[0] == pytest.approx(2 * ch, rel=1e-15)
    # |B| = 1: CH is the plain sum of distances to the single point
    b = B[:1]
    ref = np.sum(np.abs(A - b).sum(1)) if metric == 1 else np.sum(np.sqrt(((A.astype(np.float64) - b) ** 2).sum(1)))
    assert orc.chamfer_exact(A, b, metric)[0] == pytest.approx(float(ref), rel=1e-14)


def test_dist32_exact_on_small_integers(orc):
    """With small integer coordinates every float32 step is exact, so
    dist32 equals the closed-form integer distance."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        d = int(rng.integers(1, 40))
        a = rng.integers(-100, 100, size=d).astype(np.float32)
        b = rng.integers(-100, 100, size=d).astype(np.float32)
        l1 = int(np.abs(a.astype(np.int64) - b.astype(np.int64)).sum())
        l2sq = int(((a.astype(np.int64) - b.astype(np.int64)) ** 2).sum())
        assert orc.dist32(a, b, 1) == np.float32(l1)
        assert orc.dist32(a, b, 2) == np.float32(math.sqrt(l2sq))


@pytest.mark.parametrize("metric", [1, 2])
def test_dist32_error_bound(orc, metric):
    """dist32 is within the float32 rounding bound of the exact distance."""
    rng = np.random.default_rng(12)
    for _ in range(200):
        d = int(rng.integers(1, 300))
        a = (rng.standard_normal(d) * 10).astype(np.float32)
        b = (rng.standard_normal(d) * 10).astype(np.float32)
        ex = cdist(a[None].astype(np.float64), b[None].astype(np.float64),
                   "cityblock" if metric == 1 else "euclidean")[0, 0]
        bound = (d + 3) * U32 * ex
        assert abs(float(orc.dist32(a, b, metric)) - ex) <= bound


def test_nn_f32_is_canonical_argmin(orc):
    """nn_f32 picks, among equal float32 distances, the lower index."""
    A = np.array([[0.0, 0.0]], np.float32)
    B = np.array([[3.0, 4.0], [1.0, 0.0], [0.0, 1.0], [-1.0, 0.0]], np.float32)
    for metric in (1, 2):
        m, arg = orc.nn_f32(A, B, metric)
        assert arg[0] == 1 and m[0] == 1.0
        m64, arg64 = orc.nn_f64(A, B, metric)
        assert arg64[0] == 1 and m64[0] == 1.0


# ---------------------------------------------------------- parameters -----

def test_default_parameters(orc):
    with open(os.path.join(GOLDEN, "parameters.json")) as f:
        g = json.load(f)
    for c in g["scales"]:
        assert orc.default_scales(c["n_a"], c["n_b"], c["eps"]) == c["L"]
    for c in g["samples"]:
        assert orc.default_samples(c["n_a"], c["eps"]) == c["T"]


def test_calibration_hand_cases(orc):
    A = np.array([[0, 0], [1, 3]], np.float32)
    B = np.array([[-1, 2]], np.float32)
    lo, hi, S, e = orc.calibrate(A, B)
    np.testing.assert_array_equal(lo, [-1, 0])
    np.testing.assert_array_equal(hi, [1, 3])
    assert S == 5.0 and e == 3          # 2^2 < 5 <= 2^3
    lo, hi, S, e = orc.calibrate(np.array([[0, 0]], np.float32), np.array([[4, 0]], np.float32))
    assert S == 4.0 and e == 2          # exact power of two
    lo, hi, S, e = orc.calibrate(np.ones((3, 2), np.float32), np.ones((2, 2), np.float32))
    assert S == 0.0 and e == 0          # all points coincide
    lo, hi, S, e = orc.calibrate(np.array([[0.0]], np.float32), np.array([[0.75]], np.float32))
    assert e == 0                       # 2^-1 < 0.75 <= 2^0


# ------------------------------------------------------------- hashing -----

def _keys_at(orc, X, seed, e, lo=None, metric=1, Zs=None, kh=None):
    """Keys of X at one scale of side 2^e (L = 1, e_top = e)."""
    d = X.shape[1]
    kh = kh or d
    zf, mt = orc.grid_tables(seed, 1, kh)
    lo = np.zeros(d, np.float32) if lo is None else lo
    return orc.hash_keys(X, metric, lo, Zs, 1, e, zf, mt)[0]


def test_grid_collision_probability(orc):
    """Appendix lemma on the grid hash: Pr[h(x) = h(y)] =
    prod_k max(0, 1 - |x_k - y_k| / r).  Monte Carlo over seeds."""
    x = np.array([0.3, 0.1, 0.7, 2.0], np.float32)
    cases = [
        (np.array([0.2, -0.1, 0.05, 0.0], np.float32), 0),    # r = 1
        (np.array([0.6, 0.3, 0.0, -0.5], np.float32), 1),     # r = 2
        (np.array([1.5, 0.0, 0.0, 0.0], np.float32), 0),      # separated: prob 0
        (np.array([0.05, 0.02, 0.01, 0.0], np.float32), -2),  # r = 1/4
    ]
    n_seeds = 3000
    for delta, e in cases:
        y = x + delta
        r = 2.0 ** e
        p = float(np.prod(np.maximum(0.0, 1.0 - np.abs((y.astype(np.float64) - x)) / r)))
        X = np.stack([x, y])
        hits = 0
        for s in range(n_seeds):
            k = _keys_at(orc, X, 1000 + s, e)
            hits += int(k[0] == k[1])
        sd = math.sqrt(max(p * (1 - p), 1e-12) / n_seeds)
        assert abs(hits / n_seeds - p) <= 4.5 * sd + 1e-9, (delta, e, hits / n_seeds, p)


def test_same_cell_same_key_distinct_cells_distinct_keys(orc):
    rng = np.random.default_rng(3)
    X = rng.uniform(0, 64, size=(4000, 6)).astype(np.float32)
    zf, mt = orc.grid_tables(77, 1, 6)
    keys = orc.hash_keys(X, 1, np.zeros(6, np.float32), None, 1, 3, zf, mt)[0]
    # X 2^-3 is exact in float32; one rounding of the shifted sum, then floor
    cells = np.floor(np.ldexp(X, -3).astype(np.float32) + zf[0]).astype(np.int64)
    for p in range(0, 4000, 97):
        assert int(keys[p]) == _key_from_cells(cells[p], mt[0])
    # equal cells <=> equal keys on this sample (no 63-bit collisions expected)
    _, inv_c = np.unique(cells, axis=0, return_inverse=True)
    _, inv_k = np.unique(keys, return_inverse=True)
    assert len(np.unique(inv_c)) == len(np.unique(inv_k))
    pairs = set(zip(inv_c.ravel().tolist(), inv_k.ravel().tolist()))
    assert len(pairs) == len(np.unique(inv_c))
    assert int(keys.max()) < 2 ** 63


def test_shift_table_range(orc):
    zf, mt = orc.grid_tables(5, 24, 64)
    assert zf.min() >= 0.0 and zf.max() < 1.0
    assert np.all(np.ldexp(zf.astype(np.float64), 24) == np.round(np.ldexp(zf.astype(np.float64), 24)))
    # two odd 24-bit multipliers per (scale, coordinate), from the second
    # Philox word (numpy's independent Philox4x64-10 for the reference)
    m1, m2 = mt & np.uint64(0xFFFFFFFF), mt >> np.uint64(32)
    assert np.all(m1 & np.uint64(1) == 1) and np.all(m2 & np.uint64(1) == 1)
    assert int(m1.max()) < 2 ** 24 and int(m2.max()) < 2 ** 24
    for i, k in [(0, 1), (3, 17), (23, 63)]:
        bg = np.random.Philox(key=np.array([5, 0], np.uint64),
                              counter=np.array([k, i, 1, 0], np.uint64) - np.array([1, 0, 0, 0], np.uint64))
        w = bg.random_raw(4)
        assert int(m1[i, k]) == (int(w[1]) & 0xFFFFFF) | 1
        assert int(m2[i, k]) == ((int(w[1]) >> 32) & 0xFFFFFF) | 1
        assert float(zf[i, k]) == (int(w[0]) >> 40) * 2.0 ** -24
    # roughly uniform on [0, 1)
    assert stats.kstest(zf.ravel(), "uniform").pvalue > 1e-4
    # independent per scale
    assert not np.array_equal(zf[0], zf[1])


BETA = math.sqrt(2 / math.pi)


def _quantised_gaussian_law(scale=32.0, cap=127):
    """P(clamp(rint(scale g), -cap, cap) = m) for g ~ N(0, 1), m = -cap..cap."""
    m = np.arange(-cap, cap + 1)
    p = stats.norm.cdf((m + 0.5) / scale) - stats.norm.cdf((m - 0.5) / scale)
    p[0] = stats.norm.cdf((-cap + 0.5) / scale)
    p[-1] = stats.norm.sf((cap - 0.5) / scale)
    return m, p


def test_embedding_entries_quantised_gaussian(orc):
    """The embedding's entries are clamp(rint(32 g), -127, 127) of standard
    Gaussians g (the finite-precision form of the Gaussian matrix of the
    appendix theorem embedding l2 into l1): chi-square against that
    discrete law, and the second moment against its exact value."""
    Z = np.concatenate([orc.embedding(s, 64, 64).ravel() for s in range(40)]).astype(np.int64)
    m, p = _quantised_gaussian_law()
    counts = np.bincount(Z + 127, minlength=255)
    # pool the sparse tails into two bins
    lo_t, hi_t = np.searchsorted(m, -90), np.searchsorted(m, 90)
    obs = np.concatenate([[counts[:lo_t].sum()], counts[lo_t:hi_t + 1], [counts[hi_t + 1:].sum()]])
    exp = np.concatenate([[p[:lo_t].sum()], p[lo_t:hi_t + 1], [p[hi_t + 1:].sum()]]) * len(Z)
    assert stats.chisquare(obs, exp).pvalue > 1e-4
    ez2 = float((m.astype(np.float64) ** 2 * p).sum())
    assert abs(float(np.mean(Z.astype(np.float64) ** 2)) - ez2) < 4.5 * math.sqrt(
        float((m.astype(np.float64) ** 4 * p).sum()) - ez2 ** 2) / math.sqrt(len(Z))


def test_embedding_normalisation(orc):
    """Appendix theorem embedding l2 into l1: T(x) = Z x / (beta ke), beta =
    sqrt(2/pi), has E ||T(x)||_1 = ||x||_2 for Gaussian Z.  With Z = the
    quantised matrix / 32: the second moment of each coordinate is exactly
    E[Zq^2] |x|^2 / (32 beta ke)^2 (independent zero-mean entries), and the
    l1 norm matches |x|_2 up to the quantisation's effect on E|g|
    (well below 0.5% here).  Averaged over seeds."""
    rng = np.random.default_rng(9)
    d, ke = 24, 32
    x = rng.standard_normal(d)
    m, p = _quantised_gaussian_law()
    ez2 = float((m.astype(np.float64) ** 2 * p).sum())
    l1, sq = [], []
    for s in range(600):
        T = orc.embedding(s, d, ke).astype(np.float64) / (32.0 * BETA * ke)
        y = T @ x
        l1.append(np.abs(y).sum())
        sq.append(float(y @ y))
    l1, sq = np.array(l1), np.array(sq)
    want_sq = ke * ez2 * float(x @ x) / (32.0 * BETA * ke) ** 2
    assert abs(sq.mean() - want_sq) < 4.5 * sq.std() / math.sqrt(len(sq))
    ratio = l1.mean() / np.linalg.norm(x)
    assert abs(ratio - 1.0) < 4.5 * l1.std() / np.linalg.norm(x) / math.sqrt(len(l1)) + 0.005


def _embed_reference(orc, X, lo, Zq, e_top):
    """float64 T(x - lo) = Zq (x - lo) / (32 beta ke) from the unquantised
    coordinates, and the bound on its distance to the hashed coordinates:
    quantising each coordinate to 24 bits of 2^e_top moves it by less than
    one step q = 2^(e_top - 24) (plus the float32 rounding of x - lo), so
    |y_j - T_j| <= sum_k |Zq_jk| (q + u |x_k - lo_k|) / (32 beta ke) plus the
    two final roundings (double product, float32)."""
    ke = Zq.shape[0]
    inv = 1.0 / (BETA * ke * 32.0)
    Xc = X.astype(np.float64) - lo.astype(np.float64)
    ref = (Xc @ Zq.astype(np.float64).T) * inv
    q = 2.0 ** (e_top - 24)
    bound = ((q + U32 * np.abs(Xc)) @ np.abs(Zq.astype(np.float64)).T) * inv
    bound += 2 * U32 * np.abs(ref) + 1e-300
    return ref, bound


@pytest.mark.parametrize("d", [5, 32, 128])
def test_l2_hashed_coords_vs_float64(orc, d):
    """The l2 hashed coordinates are the embedding T(x - lo) of the appendix
    theorem embedding l2 into l1 in its quantised form: compared with a
    float64 matrix product of the unquantised coordinates within the
    quantisation bound.  d = 32 = ke makes a transposed matrix index produce
    a valid but different product, and the offset of the cloud makes a
    dropped - lo visible; both planted mistakes are shown to fail the
    bound, as does a wrong normalisation."""
    rng = np.random.default_rng(100 + d)
    X = (rng.standard_normal((300, d)) * 3.0 + 40.0).astype(np.float32)
    lo = X.min(axis=0) - np.float32(0.5)
    S = float(np.sum(X.max(axis=0).astype(np.float64) - lo.astype(np.float64)))
    e_top = math.ceil(math.log2(S))
    Zq = orc.embedding(11, d, 32)
    Y = orc.hashed_coords(X, 2, lo, Zq, e_top).astype(np.float64)
    ref, bound = _embed_reference(orc, X, lo, Zq, e_top)
    assert Y.shape == (300, 32)
    assert np.all(np.abs(Y - ref) <= bound), np.max(np.abs(Y - ref) / bound)
    # l1 hashes x - lo, one float32 subtraction per coordinate
    Y1 = orc.hashed_coords(X, 1, lo, None, e_top)
    assert np.array_equal(Y1, (X - lo).astype(np.float32))
    # the pin rejects the plausible mistakes
    inv = 1.0 / (BETA * 32 * 32.0)
    no_lo = (X.astype(np.float64) @ Zq.astype(np.float64).T) * inv
    assert np.any(np.abs(no_lo - ref) > bound)
    assert np.any(np.abs(ref * 1.01 - ref) > bound)
    if d == 32:
        transposed = ((X.astype(np.float64) - lo.astype(np.float64)) @ Zq.astype(np.float64)) * inv
        assert np.any(np.abs(transposed - ref) > bound)


def _key_from_cells(cells, mult):
    """The bucket key of integer cells in Python integers:
    K1 = sum_k (c_k mod 2^24) M1_k mod 2^32, K2 likewise with M2,
    key = (K1 2^32 + K2) >> 1, M = M1 | M2 << 32."""
    k1 = k2 = 0
    for c, m in zip((int(v) for v in cells), (int(v) for v in mult)):
        c24 = c % (1 << 24)
        k1 = (k1 + c24 * (m & 0xFFFFFFFF)) % (1 << 32)
        k2 = (k2 + c24 * (m >> 32)) % (1 << 32)
    return ((k1 << 32) | k2) >> 1


def test_l2_keys_from_float64_cells(orc):
    """l2 keys end to end: cells floor(y / r + z') computed from the float64
    embedding, keyed in Python integers, equal the oracle's keys at every
    scale for every coordinate whose cell boundary is farther away than the
    embedding's quantisation bound and the float32 rounding of the shifted
    coordinate (the others are skipped: there either cell is right)."""
    rng = np.random.default_rng(7)
    n, d, ke, L = 200, 24, 32, 6
    X = (rng.standard_normal((n, d)) * 2.0 - 5.0).astype(np.float32)
    lo = X.min(axis=0)
    Zq = orc.embedding(5, d, ke)
    zf, mt = orc.grid_tables(5, L, ke)
    e_top = 7
    keys = orc.hash_keys(X, 2, lo, Zq, L, e_top, zf, mt)
    y64, yerr = _embed_reference(orc, X, lo, Zq, e_top)
    checked = 0
    for i in range(L):
        e = e_top - (L - 1 - i)
        q = np.ldexp(y64, -e) + zf[i].astype(np.float64)
        # float32 of y, then one rounding of the shifted sum
        margin = np.ldexp(yerr, -e) + 2 * U32 * (np.abs(q) + 1.0)
        frac_dist = q - np.floor(q)
        near = (frac_dist <= margin) | (1.0 - frac_dist <= margin)
        cells = np.floor(q).astype(np.int64)
        for p in range(n):
            if near[p].any():
                continue
            assert int(keys[i, p]) == _key_from_cells(cells[p], mt[i]), (i, p)
            checked += 1
    assert checked > 0.8 * n * L


@pytest.mark.parametrize("ratio", [0.3, 1.0, 2.5])
def test_l2_collision_probability(orc, ratio):
    """l2 grid hash through the embedding: given the embedding Zs drawn by a
    seed, the keys of x and x' at side r collide with probability
    prod_j max(0, 1 - |(Zs (x - x'))_j| / r) (appendix lemma on the grid
    hash, applied to the embedded coordinates; shifts and embedding come
    from independent streams).  Monte Carlo over seeds: the mean of the
    collision indicator matches the mean predicted probability."""
    d, ke, e = 6, 32, 0
    rng = np.random.default_rng(int(ratio * 10))
    x = rng.uniform(0.0, 4.0, d).astype(np.float32)
    v = rng.standard_normal(d)
    xp = (x + ratio * v / np.linalg.norm(v)).astype(np.float32)
    X = np.stack([x, xp])
    lo = np.full(d, -4.0, np.float32)
    n_seeds = 2500
    hits, probs = 0, []
    # coordinates within 2^e_top of lo (the calibration's guarantee); the
    # finest of L scales has side 2^e
    e_top, L = 4, 5
    for s in range(n_seeds):
        Zq = orc.embedding(3000 + s, d, ke)
        zf, mt = orc.grid_tables(3000 + s, L, ke)
        k = orc.hash_keys(X, 2, lo, Zq, L, e_top, zf, mt)[0]
        hits += int(k[0] == k[1])
        y = orc.hashed_coords(X, 2, lo, Zq, e_top).astype(np.float64)
        dy = y[1] - y[0]
        probs.append(float(np.prod(np.maximum(0.0, 1.0 - np.abs(dy) / 2.0 ** e))))
    probs = np.array(probs)
    p = probs.mean()
    sd = math.sqrt(max(float(np.mean(probs * (1 - probs))), 1e-12) / n_seeds)
    assert abs(hits / n_seeds - p) <= 4.5 * sd + 1e-3, (ratio, hits / n_seeds, p)
    assert 0.02 < p < 0.95


# -------------------------------------------------------------- CrudeNN ----

@pytest.mark.parametrize("metric", [1, 2])
def test_crude_nn_join_brute_force(orc, metric):
    """CrudeNN figure, step 3, checked by brute force over all (a, b, i):
    the reported scale is the first with any b sharing a's key, and the
    candidate is the lowest such b."""
    rng = np.random.default_rng(21 + metric)
    A = rng.uniform(-3, 3, size=(150, 5)).astype(np.float32)
    B = rng.uniform(-3, 3, size=(90, 5)).astype(np.float32)
    r = orc.crude_nn(A, B, metric, 0.3, seed=99, n_scales=12)
    kA, kB, L = r["keys_a"], r["keys_b"], r["L"]
    for a in range(A.shape[0]):
        first, cand = L, 0
        for i in range(L):
            hit = np.nonzero(kB[i] == kA[i, a])[0]
            if hit.size:
                first, cand = i, int(hit[0])
                break
        assert r["scale"][a] == first and r["nn"][a] == cand
        assert r["D"][a] == orc.dist32(A[a], B[cand], metric)


@pytest.mark.parametrize("metric", [1, 2])
def test_crude_nn_upper_bound(orc, metric):
    """Oversampling lemma: D_a >= min_b d(a, b) with probability one."""
    A, B = workloads.clusters_l2(seed=4, n=600, d=12, k=20)
    r = orc.crude_nn(A, B, metric, 0.2, seed=5)
    m32, _ = orc.nn_f32(A, B, metric)
    m64, _ = orc.nn_f64(A, B, metric)
    assert np.all(r["D"] >= m32)
    assert np.all(r["D"].astype(np.float64) >= m64 * (1 - 1e-6))
    lam = r["D"].astype(np.float64).sum() / m64.sum()
    assert 1.0 <= lam < 8.0          # E[D_a] <= O(log n) min_b d(a,b)


def test_crude_nn_single_b_and_self(orc):
    rng = np.random.default_rng(6)
    A = rng.standard_normal((50, 7)).astype(np.float32)
    b = rng.standard_normal((1, 7)).astype(np.float32)
    for metric in (1, 2):
        r = orc.crude_nn(A, b, metric, 0.1, seed=1)
        assert np.all(r["nn"] == 0)
        assert np.all(r["D"] == np.array([orc.dist32(a, b[0], metric) for a in A]))
    # A = B with well separated points: every a finds itself at the finest scale
    P = rng.uniform(0, 1, size=(100, 3)).astype(np.float32)
    for metric in (1, 2):
        r = orc.crude_nn(P, P, metric, 0.1, seed=2)
        assert np.all(r["D"] == 0.0)


def test_grid_stream_repetitions(orc):
    """The shifts and multipliers of LSH structure r come from the counter
    (k, i, GRID, r): checked against numpy's Philox; r = 0 is the single
    structure of the base algorithm, other r are independent."""
    seed, L, kh = 77, 6, 5
    base = orc.grid_tables(seed, L, kh)
    for r in (0, 1, 5):
        z, m = orc.grid_tables(seed, L, kh, r)
        for i in range(L):
            for k in range(kh):
                # numpy adds one to the 256-bit counter before each block
                ctr = [k, i, 1, r]
                for j in range(4):
                    if ctr[j]:
                        ctr[j] -= 1
                        break
                    ctr[j] = 2**64 - 1
                bg = np.random.Philox(key=np.array([seed, 0], np.uint64),
                                      counter=np.array(ctr, np.uint64))
                w = bg.random_raw(4)
                assert z[i, k] == np.float32(math.ldexp(int(w[0]) >> 40, -24))
                w1 = int(w[1])
                assert int(m[i, k]) == ((w1 & 0xFFFFFF) | 1) | ((((w1 >> 32) & 0xFFFFFF) | 1) << 32)
        if r == 0:
            assert np.array_equal(z, base[0]) and np.array_equal(m, base[1])
        else:
            assert not np.array_equal(z, base[0])


def _window_brute_force(orc, A, B, metric, seed, L, W, reps):
    """The k x W retrieval written out with Python dicts over each
    structure's keys: first W distinct b finest scale first, ascending b
    within a bucket; the closest retrieved b (ties to the lower b)."""
    lo, hi, S, e_top = orc.calibrate(A, B)
    Zs = orc.embedding(seed, A.shape[1]) if metric == 2 else None
    kh = A.shape[1] if metric == 1 else Zs.shape[0]
    best = [None] * A.shape[0]
    first = [L] * A.shape[0]
    for r in range(reps):
        z, m = orc.grid_tables(seed, L, kh, r)
        kA = orc.hash_keys(A, metric, lo, Zs, L, e_top, z, m)
        kB = orc.hash_keys(B, metric, lo, Zs, L, e_top, z, m)
        buckets = []
        for i in range(L):
            d = {}
            for b in range(B.shape[0]):
                d.setdefault(int(kB[i, b]), []).append(b)
            buckets.append(d)
        for a in range(A.shape[0]):
            got = []
            for i in range(L):
                for b in buckets[i].get(int(kA[i, a]), []):
                    if len(got) < W and b not in got:
                        if not got:
                            first[a] = min(first[a], i)
                        got.append(b)
            if not got:
                got = list(range(min(W, B.shape[0])))
            for b in got:
                cand = (float(orc.dist32(A[a], B[b], metric)), b)
                if best[a] is None or cand < best[a]:
                    best[a] = cand
    return best, first


@pytest.mark.parametrize("metric", [1, 2])
@pytest.mark.parametrize("W,reps", [(1, 1), (3, 1), (1, 3), (5, 2)])
def test_crude_window_brute_force(orc, metric, W, reps):
    """Large-scale variant of the experiments (k LSH structures, window W)
    against the dictionary form above, on inputs small enough to have many
    multi-point buckets and some points with no collision."""
    rng = np.random.default_rng(40 + metric + 3 * W + reps)
    A = rng.uniform(-4, 4, size=(60, 4)).astype(np.float32)
    B = rng.uniform(-4, 4, size=(45, 4)).astype(np.float32)
    L = 9
    r = orc.crude_nn(A, B, metric, 0.3, seed=31, n_scales=L, window=W, reps=reps)
    best, first = _window_brute_force(orc, A, B, metric, 31, L, W, reps)
    for a in range(A.shape[0]):
        assert (float(r["D"][a]), int(r["nn"][a])) == best[a], a
        assert r["scale"][a] == first[a]


@pytest.mark.parametrize("metric", [1, 2])
def test_crude_window_monotone(orc, metric):
    """Retrieval sets grow with W (same order) and with k (more structures),
    so D_a can only decrease, and stays >= the exact nearest-neighbour
    distance (oversampling lemma)."""
    A, B = workloads.clusters_l2(seed=14, n=500, d=8, k=12)
    m32, _ = orc.nn_f32(A, B, metric)
    prev = None
    for W in (1, 2, 4, 8):
        r = orc.crude_nn(A, B, metric, 0.2, seed=3, window=W)
        assert np.all(r["D"] >= m32)
        if prev is not None:
            assert np.all(r["D"] <= prev)
        prev = r["D"]
    prev = None
    for k in (1, 2, 4):
        r = orc.crude_nn(A, B, metric, 0.2, seed=3, window=2, reps=k)
        assert np.all(r["D"] >= m32)
        if prev is not None:
            assert np.all(r["D"] <= prev)
        prev = r["D"]


def test_grid_levels_vs_quality(orc):
    """More grid levels cannot make D_a worse on average here (experiments
    section: a few levels already give D_a within ~2x)."""
    A, B = workloads.small_l2(seed=3, n=1500, d=3)
    m64, _ = orc.nn_f64(A, B, 1)
    lam = {}
    for L in (3, 8, 16):
        r = orc.crude_nn(A, B, 1, 0.2, seed=8, n_scales=L)
        lam[L] = r["D"].astype(np.float64).sum() / m64.sum()
    assert lam[16] <= lam[3] + 1e-9
    assert lam[16] < 4.0


# -------------------------------------------------------------- weights ----

def test_weights_closed_form(orc):
    rng = np.random.default_rng(7)
    for n in (1, 2, 3, 1000, 4097):
        D = np.abs(rng.standard_normal(n) * rng.choice([1e-6, 1.0, 1e6])).astype(np.float32)
        D[rng.integers(0, n, size=max(1, n // 10))] = 0.0
        D[0] = max(D[0], np.float32(1e-3))
        s, w, P, W, zero = orc.weights(D)
        assert not zero
        q = max(0, math.ceil(math.log2(n))) if n > 1 else 0
        assert 2 ** q >= n and (q == 0 or 2 ** (q - 1) < n)
        mx = Fraction(float(D.max())) * (Fraction(2) ** s)
        assert Fraction(2) ** (46 - q) <= mx < Fraction(2) ** (47 - q)
        for a in range(0, n, max(1, n // 200)):
            assert int(w[a]) == math.ceil(Fraction(float(D[a])) * (Fraction(2) ** s))
        assert np.array_equal(P, np.cumsum(w, dtype=np.uint64))
        assert W == int(P[-1]) and W <= 2 ** 47
        assert np.all((w == 0) == (D == 0))
    s, w, P, W, zero = orc.weights(np.zeros(5, np.float32))
    assert zero and W == 0


def test_sampling_frequencies(orc):
    """Draws follow Pr[x = a] = w_a / W (chi-square)."""
    D = np.array([1, 100, 1, 0, 50, 3, 100, 7], np.float32)
    s, w, P, W, _ = orc.weights(D)
    T = 200_000
    idx = orc.sample(12345, P, W, T)
    cnt = np.bincount(idx, minlength=len(D))
    assert cnt[3] == 0                    # zero weight is never drawn
    nz = w > 0
    expected = T * w[nz].astype(np.float64) / W
    chi = ((cnt[nz] - expected) ** 2 / expected).sum()
    assert stats.chi2.sf(chi, nz.sum() - 1) > 1e-4


def test_sampling_small_totals(orc):
    """With W = 1 every draw is the one point of weight 1; with tiny W all
    draws land on positive-weight points and cover them."""
    P = np.array([0, 0, 1, 1], np.uint64)
    assert np.all(orc.sample(3, P, 1, 100) == 2)
    P = np.array([1, 1, 3], np.uint64)
    idx = orc.sample(4, P, 3, 3000)
    assert set(idx.tolist()) == {0, 2}
    assert abs(np.mean(idx == 2) - 2 / 3) < 0.05


# ------------------------------------------------------------ estimator ----

def test_estimator_single_a(orc):
    """|A| = 1: every sample is that point with weight W/w = 1."""
    rng = np.random.default_rng(13)
    A = rng.standard_normal((1, 5)).astype(np.float32)
    B = rng.standard_normal((300, 5)).astype(np.float32)
    for metric in (1, 2):
        ch, _, _ = orc.chamfer_exact(A, B, metric)
        for seed in range(5):
            r = orc.chamfer_estimate(A, B, metric, 0.1, 50, seed)
            assert r["eta"] == pytest.approx(ch, rel=1e-15)


def test_estimator_single_b(orc):
    """|B| = 1: D_a is the true distance (in float32), so every seed gives
    CH up to float32 rounding and the 2^-(47-q) weight quantisation."""
    rng = np.random.default_rng(14)
    A = rng.standard_normal((700, 6)).astype(np.float32)
    b = rng.standard_normal((1, 6)).astype(np.float32)
    for metric in (1, 2):
        ch, _, _ = orc.chamfer_exact(A, b, metric)
        for seed in range(5):
            r = orc.chamfer_estimate(A, b, metric, 0.1, 64, seed)
            assert r["eta"] == pytest.approx(ch, rel=2e-6)


def test_estimator_degenerate(orc):
    rng = np.random.default_rng(15)
    P = rng.standard_normal((200, 4)).astype(np.float32)
    for metric in (1, 2):
        assert orc.chamfer_estimate(P, P, metric, 0.1, 100, 3)["eta"] == 0.0
        same = np.ones((20, 4), np.float32)
        assert orc.chamfer_estimate(same, same[:3], metric, 0.1, 100, 3)["eta"] == 0.0
        assert orc.chamfer_estimate(P[:0], P, metric, 0.1, 100, 3)["eta"] == 0.0


def test_estimator_unbiased_and_variance(orc):
    """Variance lemma: E[eta] = CH and Var[eta] <= CH^2 (D/CH - 1) / T,
    for a fixed CrudeNN output, over the sampling randomness."""
    A, B = workloads.small_l2(seed=17, n=300, d=4)
    metric, T = 1, 20
    ch, m64, _ = orc.chamfer_exact(A, B, metric)
    crude = orc.crude_nn(A, B, metric, 0.2, seed=1)
    s, w, P, W, _ = orc.weights(crude["D"])
    # variance of one term under the quantised distribution, in closed form
    wf = w.astype(np.float64)
    pos = wf > 0
    second = np.sum((W / wf[pos]) * m64[pos] ** 2)
    var_exact = (second - ch ** 2) / T
    Dn = math.ldexp(W, -s)
    assert var_exact <= ch ** 2 * (Dn / ch - 1) / T * (1 + 1e-9)
    etas = np.array([orc.chamfer_estimate(A, B, metric, 0.2, T, seed, crude=crude)["eta"]
                     for seed in range(1500)])
    # the crude output above must not depend on the sampling seed
    assert abs(etas.mean() - ch) <= 4.5 * math.sqrt(var_exact / len(etas))
    ratio = etas.var(ddof=1) / var_exact
    lo, hi = stats.chi2.ppf([1e-5, 1 - 1e-5], len(etas) - 1) / (len(etas) - 1)
    assert lo <= ratio <= hi * 1.2     # heavy tails: allow some slack above


def test_estimator_unbiased_over_hash_seeds(orc):
    """Unbiasedness also holds averaging over the hash randomness."""
    A, B = workloads.small_l2(seed=18, n=200, d=3)
    ch, _, _ = orc.chamfer_exact(A, B, 2)
    etas = np.array([orc.chamfer_estimate(A, B, 2, 0.2, 16, s)["eta"] for s in range(800)])
    assert abs(etas.mean() - ch) <= 4.5 * etas.std(ddof=1) / math.sqrt(len(etas))


def test_estimator_coverage_small_config(orc):
    """Main theorem: within (1 +- eps) CH with probability >= 99/100.
    Small configuration (l2, d = 16, eps = 0.2, T = 512), 300 seeds here
    (the GPU suite runs 1000)."""
    A, B = workloads.small_l2()
    ch, _, _ = orc.chamfer_exact(A, B, 2)
    crude_fail = 0
    for seed in range(300):
        eta = orc.chamfer_estimate(A, B, 2, 0.2, 512, seed)["eta"]
        crude_fail += int(abs(eta - ch) > 0.2 * ch)
    assert crude_fail <= 3


@pytest.mark.parametrize("d", [2, 100])
def test_outlier_scenario(orc, d):
    """Experiments section, outliers: a Gaussian cloud plus one point at
    0.5 n (1,...,1).  Importance sampling finds the outlier and stays within
    eps; uniform sampling of the same budget misses it."""
    A, B = workloads.outlier_cloud(seed=d, n=2000, d=d)
    ch, m64, _ = orc.chamfer_exact(A, B, 1)
    share = m64[-1] / ch
    assert share > 0.25                     # the outlier carries much of CH
    rng = np.random.default_rng(0)
    for seed in range(10):
        r = orc.chamfer_estimate(A, B, 1, 0.1, 100, seed)
        assert abs(r["eta"] - ch) <= 0.1 * ch
        uni = rng.integers(0, A.shape[0], size=100)
        u_est = A.shape[0] * m64[uni].mean()
        if A.shape[0] - 1 not in uni:
            assert abs(u_est - ch) > 0.5 * share * ch


# ------------------------------------------- uniform sampling, symmetric ---

def test_uniform_sampling_draws_and_weights(orc):
    """Uniform-sampling baseline: every point gets the same weight, so the
    draws are uniform over A (chi-square) and W / w = n_A exactly."""
    A, B = workloads.small_l2(seed=5, n=200, d=3)
    r = orc.chamfer_estimate(A, B, 1, 0.2, 40000, 9, sampling=orc.SAMPLING_UNIFORM)
    assert np.all(r["w"] == r["w"][0]) and r["W"] == 200 * int(r["w"][0])
    assert float(r["W"]) / float(r["w"][0]) == 200.0
    counts = np.bincount(r["idx"], minlength=200)
    assert stats.chisquare(counts).pvalue > 1e-4


def test_uniform_sampling_closed_form(orc):
    """Every point at the same distance from B: the uniform estimate equals
    CH for any draws (l1: the cube's vertices around the origin)."""
    A = np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)], np.float32)
    B = np.zeros((1, 3), np.float32)
    for seed in range(5):
        r = orc.chamfer_estimate(A, B, 1, 0.5, 7, seed, sampling=orc.SAMPLING_UNIFORM)
        assert r["eta"] == 24.0


def test_uniform_sampling_unbiased(orc):
    """E[eta] = CH over the draws, with the variance of the plain uniform
    estimator, n_A^2 Var(m) / T."""
    A, B = workloads.small_l2(seed=23, n=300, d=4)
    T = 25
    ch, m64, _ = orc.chamfer_exact(A, B, 1)
    etas = np.array([orc.chamfer_estimate(A, B, 1, 0.2, T, s, sampling=orc.SAMPLING_UNIFORM)["eta"]
                     for s in range(1500)])
    var = 300.0 ** 2 * m64.var() / T
    assert abs(etas.mean() - ch) <= 4.5 * math.sqrt(var / len(etas))
    ratio = etas.var(ddof=1) / var
    lo, hi = stats.chi2.ppf([1e-5, 1 - 1e-5], len(etas) - 1) / (len(etas) - 1)
    assert lo <= ratio <= hi


def test_uniform_misses_outlier(orc):
    """Outlier scenario: with 100 samples uniform sampling rarely draws the
    outlier and is then far off, where importance sampling is within eps."""
    A, B = workloads.outlier_cloud(seed=100, n=2000, d=100)
    ch, m64, _ = orc.chamfer_exact(A, B, 1)
    far = 0
    for seed in range(20):
        u = orc.chamfer_estimate(A, B, 1, 0.1, 100, seed, sampling=orc.SAMPLING_UNIFORM)
        i = orc.chamfer_estimate(A, B, 1, 0.1, 100, seed)
        assert abs(i["eta"] - ch) <= 0.1 * ch
        far += abs(u["eta"] - ch) > 0.2 * ch
    assert far >= 15


@pytest.mark.parametrize("metric", [1, 2])
def test_symmetric_exact(orc, metric):
    """CH(A, B) + CH(B, A) against scipy's tree both ways; symmetric in its
    arguments, zero for A = B."""
    rng = np.random.default_rng(30 + metric)
    A = rng.standard_normal((400, 5)).astype(np.float32)
    B = rng.standard_normal((250, 5)).astype(np.float32)
    p = 1 if metric == 1 else 2
    ref = (cKDTree(B.astype(np.float64)).query(A.astype(np.float64), p=p)[0].sum()
           + cKDTree(A.astype(np.float64)).query(B.astype(np.float64), p=p)[0].sum())
    tot, ab, ba = orc.chamfer_symmetric_exact(A, B, metric)
    assert tot == pytest.approx(ref, rel=1e-12)
    assert orc.chamfer_symmetric_exact(B, A, metric)[0] == pytest.approx(tot, rel=1e-15)
    assert orc.chamfer_symmetric_exact(A, A, metric)[0] == 0.0
    e_tot, e_ab, e_ba = orc.chamfer_symmetric_estimate(A, B, metric, 0.2, 2000, 4)
    assert e_tot == e_ab + e_ba
    assert e_tot == pytest.approx(tot, rel=0.05)


def test_retrieval_composition(orc):
    """Retrieval with k = m re-ranks every cloud exactly, so it returns the
    brute-force ranking; a resample of a member is retrieved first."""
    clouds, queries, src = workloads.retrieval_collection(seed=3, m=12, n_min=60, n_max=120,
                                                          queries=2)
    for q, s in zip(queries, src):
        est, top, vals = orc.retrieve(q, clouds, 1, 0.2, 50, 7, len(clouds), n_scales=3)
        brute = sorted((orc.chamfer_symmetric_exact(q, B, 1)[0], i) for i, B in enumerate(clouds))
        assert top == [i for _, i in brute] and vals == [v for v, _ in brute]
        assert top[0] == s
        est3, top3, _ = orc.retrieve(q, clouds, 1, 0.2, 50, 7, 3, n_scales=3)
        assert np.array_equal(est3, est) and len(top3) == 3
        assert top3 == sorted(top3, key=lambda i: orc.chamfer_symmetric_exact(q, clouds[i], 1)[0])


# ------------------------------------------ reduction to bounded aspect ratio

def test_sketch_direction_is_p_stable(orc):
    """<v, g> / |v|_p has the p-stable law: |Cauchy| has median 1 (l1), a
    standard normal has second moment 1 (l2).  A Gaussian g in l1 (median
    0.674 |v|_2 = 0.30 |v|_1 here) or a wrong scale fails."""
    v = np.array([1.0, -2.0, 0.5, 3.0, 1.5])
    r1 = [abs(float(orc.sketch_direction(s, 5, 1) @ v)) / np.abs(v).sum() for s in range(4000)]
    assert abs(np.median(r1) - 1.0) < 0.1
    r2 = [float(orc.sketch_direction(s, 5, 2) @ v) ** 2 / float(v @ v) for s in range(4000)]
    assert abs(np.mean(r2) - 1.0) < 0.1
    g = orc.sketch_direction(3, 1000, 1)
    assert abs(np.mean(np.abs(g) < 1.0) - 0.5) < 0.05          # P(|C| < 1) = 1/2


def test_projection_and_nearest_1d(orc):
    """Projections agree with a float64 matrix product; the sorted-search
    t_a equals the brute-force min_b |pa - pb| bit for bit, also with ties
    and duplicates."""
    rng = np.random.default_rng(0)
    X = rng.standard_normal((300, 17)).astype(np.float32)
    g = orc.sketch_direction(5, 17, 1)
    p = orc.project(X, g)
    ref = X.astype(np.float64) @ g
    assert np.all(np.abs(p - ref) <= 1e-12 * (np.abs(X).astype(np.float64) @ np.abs(g)))
    pa = rng.integers(-20, 20, 200).astype(np.float64) * 0.25
    pb = rng.integers(-20, 20, 50).astype(np.float64) * 0.25
    pa = np.concatenate([pa, [-100.0, 100.0, pb[0]]])
    brute = np.abs(pa[:, None] - pb[None, :]).min(axis=1)
    assert np.array_equal(orc.nearest_1d(pa, pb), brute)
    pa, pb = rng.standard_normal(500), rng.standard_normal(77)
    assert np.array_equal(orc.nearest_1d(pa, pb), np.abs(pa[:, None] - pb[None, :]).min(axis=1))


@pytest.mark.parametrize("metric", [1, 2])
def test_reduce_bounds_bracket_ch(orc, metric):
    """eta_lo <= CH(A, B) <= eta_hi on varied instances and seeds, the
    partition side is at least c n eta_hi, and the sum of t_a (the 1-D
    Chamfer distance) lies within the poly(n) band as well."""
    rng = np.random.default_rng(metric)
    for case in range(12):
        n_a, n_b = (int(x) for x in rng.integers(2, 400, size=2))
        d = int(rng.integers(1, 20))
        A, B = workloads.uniform_cube(case, n_a, n_b, d, lo=-float(10 ** case % 7 + 1), hi=3.0)
        ch = orc.chamfer_exact(A, B, metric)[0]
        r = orc.aspect_reduce(A, B, metric, 0.2, 100 + case)
        assert not r["degenerate"]
        assert r["eta_lo"] <= ch <= r["eta_hi"], (case, r["eta_lo"], ch, r["eta_hi"])
        assert r["eta_lo"] <= r["ch1"] * 2.0 ** r["k_lo"] and ch <= r["ch1"] * 2.0 ** r["k_lo"]
        n = max(n_a, n_b)
        assert 2.0 ** r["e_part"] >= (r["eta_hi"] / r["eta_lo"]) * n * r["eta_hi"]
        assert r["m"] >= 3 * orc.ceil_log2(n)
        assert (d + r["m"]) in (16, 32, 64, 128) or (d + r["m"] > 128 and (d + r["m"]) % 16 == 0)


def test_part_keys_match_exact_arithmetic(orc):
    """Partition keys (l1) equal the cell formula evaluated in exact
    rational arithmetic, at a side small enough for many cells."""
    from fractions import Fraction
    rng = np.random.default_rng(4)
    X = (rng.standard_normal((200, 4)) * 50).astype(np.float32)
    lo = X.min(axis=0)
    zf, mt = orc.part_tables(9, 4)
    for e in (-3, 0, 4, 9):
        keys = orc.part_keys(X, 1, lo, 0, None, e, zf, mt)
        for p in range(0, 200, 7):
            acc = 0
            for k in range(4):
                y = np.float32(X[p, k]) - np.float32(lo[k])      # float32 subtraction
                c = math.ceil(Fraction(float(y)) / Fraction(2) ** e + Fraction(float(zf[k])))
                acc = (acc + (c % 2 ** 64) * int(mt[k])) % 2 ** 64
            assert int(keys[p]) == acc >> 1, (e, p)


def test_partition_splits_far_groups(orc):
    """Two groups 1e30 apart with neighbours 0.5 and 1e20 inside them (1e20
    is 2^-33 of the group's magnitude: the double-precision projection still
    resolves it): the partition separates them, every part of A has points
    of B, and the sum of the parts' exact Chamfer distances is CH(A, B); the
    reduced estimate is the sum of the parts' estimates (here exact: every
    part's D_a is its true nearest distance)."""
    A = np.array([[0, 0], [1, 0], [1e30, 0]], np.float32)
    B = np.array([[0.5, 0], [1.5, 0], [1e30, 1e20]], np.float32)
    ch = orc.chamfer_exact(A, B, 1)[0]
    split = 0
    for seed in range(8):
        r = orc.aspect_reduce(A, B, 1, 0.2, seed)
        pl = orc.parts(r["keys_A"], r["keys_B"])
        assert pl is not None
        if len(pl) == 2:
            split += 1
            assert sum(orc.chamfer_exact(A[ra], B[rb], 1)[0] for ra, rb in pl) == ch
            est = orc.chamfer_estimate_reduced(A, B, 1, 0.2, 50, seed)
            assert est["parts"] == 2
            assert est["eta"] == pytest.approx(ch, rel=1e-12)
    assert split >= 6


@pytest.mark.parametrize("metric", [1, 2])
def test_padding_properties(orc, metric):
    """Padding: every appended vector has l1 norm m q, signs are fair, rows
    with different sign vectors are at least 2q apart, and CH(A', B') lies
    in [CH, CH + 2 m q n_A] (l1; sqrt(m) for l2), within (1 + eps) CH at
    the reduction's q."""
    A, B = workloads.clusters_l2(seed=5, n=500, d=8, k=5, n_b=400)
    r = orc.aspect_reduce(A, B, metric, 0.2, 11)
    m, q = r["m"], float(r["q"])
    Ap, Bp = orc.pad(A, m, 0, 11, r["q"]), orc.pad(B, m, 1, 11, r["q"])
    assert np.array_equal(Ap[:, :8], A) and np.array_equal(Bp[:, :8], B)
    V = Ap[:, 8:].astype(np.float64)
    assert np.all(np.abs(V) == q) and np.allclose(np.abs(V).sum(axis=1), m * q)
    assert abs(np.mean(V < 0) - 0.5) < 0.02
    signs = {tuple(row) for row in (V < 0)}
    assert len(signs) == len(V)
    ch = orc.chamfer_exact(A, B, metric)[0]
    chp = orc.chamfer_exact(Ap, Bp, metric)[0]
    slack = 2 * q * (m if metric == 1 else math.sqrt(m)) * A.shape[0]
    assert ch <= chp <= ch + slack
    assert chp <= (1 + 0.2) * ch
    # a large q makes the bound tight enough to see
    Ap, Bp = orc.pad(A, m, 0, 11, 1.0), orc.pad(B, m, 1, 11, 1.0)
    assert orc.chamfer_exact(Ap, Bp, 1)[0] > ch + A.shape[0]


def test_reduced_estimate_trivial_and_degenerate(orc):
    """An ordinary instance has one part: the partition-only reduction is
    the plain estimate; A inside B gives M = 0 (no partition, q = 0) and
    eta = 0."""
    A, B = workloads.clusters_l2(seed=6, n=700, d=16, k=7, n_b=900)
    for metric in (1, 2):
        red = orc.chamfer_estimate_reduced(A, B, metric, 0.2, 0, 3, orc.REDUCE_PARTITION)
        assert red["parts"] == 1
        assert red["eta"] == orc.chamfer_estimate(A, B, metric, 0.2, 0, 3)["eta"]
    r = orc.aspect_reduce(B[:100], B, 1, 0.2, 3)
    assert r["degenerate"] and r["max_t"] == 0.0 and r["q"] == 0.0
    assert orc.chamfer_estimate_reduced(B[:100], B, 1, 0.2, 0, 3, orc.REDUCE_PAD)["eta"] == 0.0
