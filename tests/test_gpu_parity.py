"""GPU parity: every stage of the hot path against the CPU oracle on the same
seeded inputs, through the C ABI.

Integer and index outputs (bucket keys, e_top, first colliding scale,
candidate b, D_a bit patterns, sampled indices, W, s, arg-mins) must be
bit-identical.  Float outputs follow the tolerance of the path: the
canonical float32 distances equal the oracle's float32 values bit for bit,
and agree with its double-precision distances within 1e-5 relative; eta and
CH agree with the oracle within 1e-5 relative.
"""

import math

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL = 1e-5


@pytest.fixture(scope="module")
def ch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_03043_amd as lib
    lib.lib()
    return lib


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def banner(msg):
    print(f"[case] {msg}", flush=True)


SHAPES = [  # (n_a, n_b, d) spanning several tiles with ragged tails
    (1000, 777, 3),
    (2049, 3001, 16),
    (513, 4100, 64),
    (300, 2500, 128),
    (130, 211, 37),
    (1, 1, 5),
    (65, 1, 32),
]


def clouds(n_a, n_b, d, seed):
    A, _ = workloads.clusters_l2(seed=seed, n=n_a, d=d, k=max(2, n_a // 50), n_b=1)
    _, B = workloads.clusters_l2(seed=seed, n=1, d=d, k=max(2, n_a // 50), n_b=n_b)
    return A, B


# ----------------------------------------------------------------- keys --

@pytest.mark.parametrize("metric", [1, 2])
@pytest.mark.parametrize("shape", [(1000, 777, 3), (2049, 3001, 16), (300, 500, 64),
                                   (129, 70, 128), (100, 90, 300)])
def test_hash_keys_bit_exact(ch, orc, metric, shape):
    n_a, n_b, d = shape
    banner(f"hash_keys metric={metric} shape={shape}")
    A, B = clouds(n_a, n_b, d, seed=d)
    for seed in (1, 2**35 + 11):
        ka, kb, et = ch.chamfer_hash_keys(dev(A), dev(B), metric, 0.1, seed)
        ref = orc.crude_nn(A, B, metric, 0.1, seed)
        assert int(host(et)[0]) == ref["e_top"]
        assert np.array_equal(host(ka).view(np.uint64), ref["keys_a"])
        assert np.array_equal(host(kb).view(np.uint64), ref["keys_b"])


def test_hash_keys_embed_dims(ch, orc):
    A, B = clouds(300, 200, 24, seed=3)
    for ke in (8, 16, 64):
        ka, kb, _ = ch.chamfer_hash_keys(dev(A), dev(B), 2, 0.2, 9, embed_dim=ke, n_scales=11)
        ref = orc.crude_nn(A, B, 2, 0.2, 9, n_scales=11, embed_dim=ke)
        assert np.array_equal(host(ka).view(np.uint64), ref["keys_a"])
        assert np.array_equal(host(kb).view(np.uint64), ref["keys_b"])


# -------------------------------------------------------------- CrudeNN --

@pytest.mark.parametrize("metric", [1, 2])
@pytest.mark.parametrize("shape", SHAPES)
def test_crude_nn_bit_exact(ch, orc, metric, shape):
    n_a, n_b, d = shape
    banner(f"crude_nn metric={metric} shape={shape}")
    A, B = clouds(n_a, n_b, d, seed=n_a + d)
    for seed in (5, 123456789):
        D, nn, sc = ch.crude_nn(dev(A), dev(B), metric, 0.1, seed)
        ref = orc.crude_nn(A, B, metric, 0.1, seed)
        assert np.array_equal(host(sc), ref["scale"])
        assert np.array_equal(host(nn), ref["nn"])
        assert np.array_equal(host(D).view(np.uint32), ref["D"].view(np.uint32))


def test_crude_nn_self_and_single(ch, orc):
    rng = np.random.default_rng(1)
    P = rng.uniform(0, 1, size=(500, 3)).astype(np.float32)
    for metric in (1, 2):
        D, nn, sc = ch.crude_nn(dev(P), dev(P), metric, 0.1, 4)
        ref = orc.crude_nn(P, P, metric, 0.1, 4)
        assert np.array_equal(host(D).view(np.uint32), ref["D"].view(np.uint32))
        assert np.array_equal(host(nn), ref["nn"])
    b = P[:1]
    D, nn, _ = ch.crude_nn(dev(P), dev(b), 2, 0.1, 4)
    assert np.all(host(nn) == 0)


# --------------------------------------------------- multi-probe CrudeNN ---

MULTI = [(4, 1), (1, 3), (8, 4), (32, 2)]  # (window W, structures k)


@pytest.mark.parametrize("metric", [1, 2])
@pytest.mark.parametrize("shape", [(1000, 777, 3), (2049, 3001, 16), (300, 2500, 128),
                                   (130, 211, 37), (65, 1, 32), (5, 3, 4)])
@pytest.mark.parametrize("W,reps", MULTI)
def test_crude_multiprobe_bit_exact(ch, orc, metric, shape, W, reps):
    """k x W CrudeNN (window tables, repeated structures) against the oracle:
    first colliding scale, candidate and D_a bits."""
    n_a, n_b, d = shape
    banner(f"crude_nn multiprobe metric={metric} shape={shape} W={W} k={reps}")
    A, B = clouds(n_a, n_b, d, seed=n_a + d + 5)
    D, nn, sc = ch.crude_nn(dev(A), dev(B), metric, 0.1, 17, window=W, reps=reps)
    ref = orc.crude_nn(A, B, metric, 0.1, 17, window=W, reps=reps)
    assert np.array_equal(host(sc), ref["scale"])
    assert np.array_equal(host(nn), ref["nn"])
    assert np.array_equal(host(D).view(np.uint32), ref["D"].view(np.uint32))


@pytest.mark.parametrize("d,W", [(230, 16), (250, 4), (224, 16)])
def test_crude_multiprobe_wide_l1(ch, orc, d, W):
    """l1 rows too wide to stage in LDS next to the window (coordinates read
    from HBM instead), and the widest that still fits."""
    banner(f"crude_nn multiprobe l1 d={d} W={W}")
    A, B = clouds(400, 600, d, seed=d)
    D, nn, sc = ch.crude_nn(dev(A), dev(B), 1, 0.2, 3, window=W, reps=2)
    ref = orc.crude_nn(A, B, 1, 0.2, 3, window=W, reps=2)
    assert np.array_equal(host(sc), ref["scale"])
    assert np.array_equal(host(nn), ref["nn"])
    assert np.array_equal(host(D).view(np.uint32), ref["D"].view(np.uint32))


@pytest.mark.parametrize("metric", [1, 2])
@pytest.mark.parametrize("shape", [(2049, 3001, 16), (300, 2500, 128)])
def test_estimate_multiprobe(ch, orc, metric, shape):
    """The estimator on top of the k x W crude distances: weights, draws,
    sample minima and eta as the oracle."""
    n_a, n_b, d = shape
    banner(f"estimate multiprobe metric={metric} shape={shape}")
    A, B = clouds(n_a, n_b, d, seed=11 * d)
    out = ch.chamfer_estimate(dev(A), dev(B), metric, 0.2, 300, 8, window=8, reps=4)
    ref = orc.chamfer_estimate(A, B, metric, 0.2, 300, 8, window=8, reps=4)
    c = ref["crude"]
    assert np.array_equal(host(out["crude_D"]).view(np.uint32), c["D"].view(np.uint32))
    assert np.array_equal(host(out["crude_nn"]), c["nn"])
    assert np.array_equal(host(out["crude_scale"]), c["scale"])
    assert int(host(out["W"])[0]) == ref["W"] and int(host(out["s"])[0]) == ref["s"]
    assert np.array_equal(host(out["sample_idx"]), ref["idx"])
    m32, a32 = orc.nn_f32(A, B, metric, rows=ref["idx"])
    assert np.array_equal(host(out["sample_nn"]), a32)
    assert np.array_equal(host(out["sample_min"]).view(np.uint32), m32.view(np.uint32))
    assert float(host(out["eta"])[0]) == pytest.approx(ref["eta"], rel=REL)


def test_multiprobe_lowers_crude_distances(ch):
    """More structures and a wider window retrieve supersets: D_a can only
    go down (the window W = 1, k = 1 run is the base algorithm)."""
    A, B = clouds(3000, 3000, 16, seed=99)
    base, _, _ = ch.crude_nn(dev(A), dev(B), 2, 0.1, 5)
    one, _, _ = ch.crude_nn(dev(A), dev(B), 2, 0.1, 5, window=1, reps=1)
    wide, _, _ = ch.crude_nn(dev(A), dev(B), 2, 0.1, 5, window=8, reps=1)
    many, _, _ = ch.crude_nn(dev(A), dev(B), 2, 0.1, 5, window=8, reps=8)
    b, o, w, m = host(base), host(one), host(wide), host(many)
    assert np.array_equal(b.view(np.uint32), o.view(np.uint32))
    assert np.all(w <= b) and np.all(m <= w)
    assert m.sum() < b.sum()


# ------------------------------------------ uniform sampling, symmetric ---

@pytest.mark.parametrize("metric", [1, 2])
@pytest.mark.parametrize("shape,T", [((1000, 777, 3), 100), ((2049, 3001, 16), 512),
                                     ((300, 2500, 128), 257), ((130, 211, 37), 64),
                                     ((1, 1, 5), 10)])
def test_uniform_estimate_parity(ch, orc, metric, shape, T):
    """Uniform-sampling baseline: unit weights, draws, sampled minima and
    eta as the oracle; no CrudeNN output."""
    n_a, n_b, d = shape
    banner(f"uniform estimate metric={metric} shape={shape} T={T}")
    A, B = clouds(n_a, n_b, d, seed=5 * d + 2)
    for seed in (0, 77):
        out = ch.chamfer_estimate(dev(A), dev(B), metric, 0.2, T, seed, sampling=ch.UNIFORM)
        ref = orc.chamfer_estimate(A, B, metric, 0.2, T, seed, sampling=orc.SAMPLING_UNIFORM)
        assert int(host(out["status"])[0]) == 0
        assert np.all(host(out["crude_D"]) == 1.0) and np.all(host(out["crude_nn"]) == -1)
        assert int(host(out["W"])[0]) == ref["W"] and int(host(out["s"])[0]) == ref["s"]
        assert np.array_equal(host(out["sample_idx"]), ref["idx"])
        m32, a32 = orc.nn_f32(A, B, metric, rows=ref["idx"])
        assert np.array_equal(host(out["sample_nn"]), a32)
        assert np.array_equal(host(out["sample_min"]).view(np.uint32), m32.view(np.uint32))
        assert float(host(out["eta"])[0]) == pytest.approx(ref["eta"], rel=REL)


def test_uniform_estimate_lowp(ch, orc):
    """Uniform draws with the BF16 exact pass (its own norms, no CrudeNN)."""
    A, B = clouds(700, 2000, 128, seed=4)
    out = ch.chamfer_estimate(dev(A), dev(B), 2, 0.2, 300, 3, sampling=ch.UNIFORM, precision=1)
    ref = orc.chamfer_estimate(A, B, 2, 0.2, 300, 3, sampling=orc.SAMPLING_UNIFORM)
    assert np.array_equal(host(out["sample_idx"]), ref["idx"])
    m32, _ = orc.nn_f32(A, B, 2, rows=ref["idx"])
    got = host(out["sample_min"])
    assert np.mean(got.view(np.uint32) == m32.view(np.uint32)) >= 0.99
    assert float(host(out["eta"])[0]) == pytest.approx(ref["eta"], rel=1e-4)


@pytest.mark.parametrize("metric", [1, 2])
@pytest.mark.parametrize("shape", [(1000, 777, 3), (513, 4100, 64), (300, 250, 128)])
def test_symmetric_parity(ch, orc, metric, shape):
    """CH(A, B) + CH(B, A), exact and estimated (both samplings), as the
    oracle; each direction and the sum."""
    n_a, n_b, d = shape
    banner(f"symmetric metric={metric} shape={shape}")
    A, B = clouds(n_a, n_b, d, seed=9 * d + 1)
    ex = host(ch.chamfer_exact_symmetric(dev(A), dev(B), metric))
    ref = orc.chamfer_symmetric_exact(A, B, metric)
    np.testing.assert_allclose(ex, np.array(ref), rtol=REL, atol=0)
    assert ex[0] == ex[1] + ex[2]
    for sampling in (0, 1):
        est = host(ch.chamfer_estimate_symmetric(dev(A), dev(B), metric, 0.2, 0, 12,
                                                 sampling=sampling))
        r = orc.chamfer_symmetric_estimate(A, B, metric, 0.2, 0, 12, sampling=sampling)
        np.testing.assert_allclose(est, np.array(r), rtol=REL, atol=0)
        assert est[0] == est[1] + est[2]


# -------------------------------------------------------- nearest rows ---

@pytest.mark.parametrize("metric", [1, 2])
@pytest.mark.parametrize("shape", SHAPES)
def test_exact_parity(ch, orc, metric, shape):
    n_a, n_b, d = shape
    banner(f"exact metric={metric} shape={shape}")
    A, B = clouds(n_a, n_b, d, seed=7 * d + n_b)
    chv, rmin, rnn = ch.chamfer_exact(dev(A), dev(B), metric)
    m32, a32 = orc.nn_f32(A, B, metric)
    m64, _ = orc.nn_f64(A, B, metric)
    assert np.array_equal(host(rnn), a32)
    assert np.array_equal(host(rmin).view(np.uint32), m32.view(np.uint32))
    np.testing.assert_allclose(host(rmin), m64, rtol=REL, atol=0)
    ref = math.fsum(m64.tolist())
    assert float(host(chv)[0]) == pytest.approx(ref, rel=REL)


def test_exact_ties_lowest_index(ch):
    A = np.array([[0.0, 0.0], [5.0, 5.0]], np.float32)
    B = np.array([[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0], [5.0, 6.0], [6.0, 5.0]], np.float32)
    for metric in (1, 2):
        _, rmin, rnn = ch.chamfer_exact(dev(A), dev(B), metric)
        assert host(rnn).tolist() == [0, 3]
        assert host(rmin).tolist() == [1.0, 1.0]


@pytest.mark.parametrize("metric", [1, 2])
def test_nn_min_rows(ch, orc, metric):
    A, B = clouds(3000, 2000, 64, seed=11)
    rows = np.random.default_rng(0).integers(0, 3000, size=777).astype(np.int32)
    mn, arg = ch.chamfer_nn_min(dev(A), dev(B), metric, rows=dev(rows))
    m32, a32 = orc.nn_f32(A, B, metric, rows=rows)
    assert np.array_equal(host(arg), a32)
    assert np.array_equal(host(mn).view(np.uint32), m32.view(np.uint32))


# ------------------------------------------------------------ estimator --

@pytest.mark.parametrize("metric", [1, 2])
@pytest.mark.parametrize("shape,T", [((1000, 777, 3), 100), ((2049, 3001, 16), 512),
                                     ((513, 4100, 64), 300), ((300, 2500, 128), 257),
                                     ((130, 211, 37), 64), ((1, 1, 5), 10)])
def test_estimate_parity(ch, orc, metric, shape, T):
    n_a, n_b, d = shape
    banner(f"estimate metric={metric} shape={shape} T={T}")
    A, B = clouds(n_a, n_b, d, seed=3 * d + 1)
    for seed in (0, 99):
        out = ch.chamfer_estimate(dev(A), dev(B), metric, 0.2, T, seed)
        ref = orc.chamfer_estimate(A, B, metric, 0.2, T, seed)
        c = ref["crude"]
        assert int(host(out["status"])[0]) == 0
        assert np.array_equal(host(out["crude_D"]).view(np.uint32), c["D"].view(np.uint32))
        assert np.array_equal(host(out["crude_nn"]), c["nn"])
        assert int(host(out["W"])[0]) == ref["W"]
        assert int(host(out["s"])[0]) == ref["s"]
        assert np.array_equal(host(out["sample_idx"]), ref["idx"])
        np.testing.assert_allclose(host(out["sample_min"]), ref["m"], rtol=REL, atol=0)
        m32, a32 = orc.nn_f32(A, B, metric, rows=ref["idx"])
        assert np.array_equal(host(out["sample_nn"]), a32)
        assert np.array_equal(host(out["sample_min"]).view(np.uint32), m32.view(np.uint32))
        assert float(host(out["D"])[0]) == ref["D_norm"]
        assert float(host(out["eta"])[0]) == pytest.approx(ref["eta"], rel=REL)


def test_estimate_default_T_and_L(ch, orc):
    A, B = workloads.small_l2(seed=42, n=2000, d=16)
    out = ch.chamfer_estimate(dev(A), dev(B), 2, 0.3, 0, 5)
    ref = orc.chamfer_estimate(A, B, 2, 0.3, 0, 5)
    assert out["T"] == ref["T"] == orc.default_samples(2000, 0.3)
    assert np.array_equal(host(out["sample_idx"]), ref["idx"])
    assert float(host(out["eta"])[0]) == pytest.approx(ref["eta"], rel=REL)


def test_estimate_degenerate(ch, orc):
    rng = np.random.default_rng(2)
    P = rng.standard_normal((300, 8)).astype(np.float32)
    for metric in (1, 2):
        out = ch.chamfer_estimate(dev(P), dev(P), metric, 0.1, 50, 3)
        assert float(host(out["eta"])[0]) == 0.0
        same = np.ones((40, 8), np.float32)
        out = ch.chamfer_estimate(dev(same), dev(same[:2]), metric, 0.1, 50, 3)
        assert float(host(out["eta"])[0]) == 0.0
        assert int(host(out["W"])[0]) == 0
        out = ch.chamfer_estimate(dev(P[:0]), dev(P), metric, 0.1, 50, 3, with_aux=False)
        assert float(host(out["eta"])[0]) == 0.0
        chv, _, _ = ch.chamfer_exact(dev(P[:0]), dev(P), metric)
        assert float(host(chv)[0]) == 0.0


def test_nonfinite_input_reports_status(ch):
    """A NaN coordinate is detected on the device: status -4, eta NaN."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((200, 4)).astype(np.float32)
    B = rng.standard_normal((100, 4)).astype(np.float32)
    A[17, 2] = np.nan
    out = ch.chamfer_estimate(dev(A), dev(B), 2, 0.1, 20, 1)
    assert int(host(out["status"])[0]) == -4
    assert math.isnan(float(host(out["eta"])[0]))
    B[3, 0] = np.inf
    chv, _, _ = ch.chamfer_exact(dev(A * 0), dev(B), 1)
    assert math.isnan(float(host(chv)[0]))


def test_determinism(ch):
    A, B = workloads.small_l2(seed=8, n=4096, d=16)
    a, b = dev(A), dev(B)
    outs = [ch.chamfer_estimate(a, b, 2, 0.2, 512, 77) for _ in range(3)]
    for o in outs[1:]:
        for k in ("eta", "sample_idx", "sample_min", "crude_D", "crude_nn"):
            assert torch.equal(o[k], outs[0][k]), k
    e = [ch.chamfer_exact(a, b, 2)[0] for _ in range(3)]
    assert torch.equal(e[0], e[1]) and torch.equal(e[0], e[2])


# -------------------------------------------------------------- coverage --

def test_coverage_small_config(ch, orc):
    """Main theorem, small configuration (l2, |A|=|B|=4096, d=16, eps=0.2,
    T=512): within (1 +- eps) CH in >= 99% of 1000 seeds."""
    A, B = workloads.small_l2()
    exact, _, _ = orc.chamfer_exact(A, B, 2)
    a, b = dev(A), dev(B)
    etas = []
    for seed in range(1000):
        etas.append(ch.chamfer_estimate(a, b, 2, 0.2, 512, seed, with_aux=False)["eta"])
    etas = host(torch.cat(etas))
    frac = np.mean(np.abs(etas - exact) <= 0.2 * exact)
    print(f"coverage {frac:.4f} mean rel err {np.mean(np.abs(etas - exact)) / exact:.4e}")
    assert frac >= 0.99


# ------------------------------------------------- precision (BF16 / FP8) --

PRECISIONS = [(1, "bf16", 0.99, 1e-3), (2, "fp8", 0.90, 1e-2)]


@pytest.mark.parametrize("prec,name,min_exact,ch_tol", PRECISIONS)
@pytest.mark.parametrize("shape", [(1000, 1500, 16), (700, 2000, 64), (513, 3001, 128),
                                   (300, 2500, 200), (257, 2049, 256)])
def test_lowp_exact_rerank(ch, orc, prec, name, min_exact, ch_tol, shape):
    """Low-precision tiles + float32 re-rank: every reported minimum is the
    canonical float32 distance to the reported row (so never below the true
    minimum), most arg-mins are exact, and CH is within the stated error."""
    n_a, n_b, d = shape
    banner(f"lowp {name} shape={shape}")
    A, B = clouds(n_a, n_b, d, seed=d + prec)
    chv, rmin, rnn = ch.chamfer_exact(dev(A), dev(B), 2, precision=prec)
    rmin, rnn = host(rmin), host(rnn)
    m32, a32 = orc.nn_f32(A, B, 2)
    m64, _ = orc.nn_f64(A, B, 2)
    chosen = np.array([orc.dist32(A[i], B[rnn[i]], 2) for i in range(n_a)], np.float32)
    assert np.array_equal(chosen.view(np.uint32), rmin.view(np.uint32))
    assert np.all(rmin >= m32)
    frac = np.mean(rnn == a32)
    err = abs(float(host(chv)[0]) - math.fsum(m64.tolist())) / math.fsum(m64.tolist())
    print(f"{name} d={d}: exact arg-min {frac:.4f}, CH rel err {err:.2e}")
    assert frac >= min_exact
    assert err <= ch_tol


@pytest.mark.parametrize("prec,name,min_exact,ch_tol", PRECISIONS)
def test_lowp_estimate(ch, orc, prec, name, min_exact, ch_tol):
    """The estimator with a low-precision exact pass: CrudeNN and the draws
    are the float32 path's (bit-exact); each sample minimum is a true float32
    distance, never below the oracle's minimum."""
    A, B = workloads.precision_l2(seed=3, n=3000, d=256, k=60)
    T = 400
    out = ch.chamfer_estimate(dev(A), dev(B), 2, 0.1, T, 11, precision=prec)
    ref = ch.chamfer_estimate(dev(A), dev(B), 2, 0.1, T, 11)
    assert torch.equal(out["sample_idx"], ref["sample_idx"])
    assert torch.equal(out["crude_D"], ref["crude_D"])
    m = host(out["sample_min"])
    m32 = host(ref["sample_min"])
    assert np.all(m >= m32)
    assert np.mean(m == m32) >= min_exact
    e_lp, e_32 = float(host(out["eta"])[0]), float(host(ref["eta"])[0])
    assert abs(e_lp - e_32) / e_32 <= ch_tol


def test_lowp_deterministic(ch):
    A, B = workloads.precision_l2(seed=4, n=2000, d=128, k=40)
    a, b = dev(A), dev(B)
    for prec in (1, 2):
        r = [ch.chamfer_exact(a, b, 2, precision=prec) for _ in range(2)]
        assert torch.equal(r[0][1], r[1][1]) and torch.equal(r[0][2], r[1][2])


def test_lowp_l1_ignores_precision(ch, orc):
    A, B = clouds(300, 400, 64, seed=9)
    _, rmin, rnn = ch.chamfer_exact(dev(A), dev(B), 1, precision=1)
    m32, a32 = orc.nn_f32(A, B, 1)
    assert np.array_equal(host(rnn), a32)


# ------------------------------------------------------------ retrieval ---

@pytest.mark.parametrize("metric", [1, 2])
def test_retrieval_parity(ch, orc, metric):
    """One-vs-many retrieval over 70 clouds (140 jobs: three batches, the
    last ragged): every symmetric estimate as the oracle's and bit-identical
    to the direct symmetric call; the top-k as the oracle's, ranked by exact
    CH; k = m gives the brute-force ranking and puts the source cloud first."""
    banner(f"retrieval metric={metric}")
    cl, qs, src = workloads.retrieval_collection(seed=21 + metric, m=70, n_min=50, n_max=300,
                                                 queries=2)
    for q, s in zip(qs, src):
        est, top, vals = ch.chamfer_retrieve(dev(q), [dev(B) for B in cl], metric, 0.2, 50, 7, 5,
                                             n_scales=3)
        r_est, r_top, r_vals = orc.retrieve(q, cl, metric, 0.2, 50, 7, 5, n_scales=3)
        e = host(est)
        np.testing.assert_allclose(e, r_est, rtol=REL, atol=0)
        assert top == r_top
        np.testing.assert_allclose(vals, r_vals, rtol=REL, atol=0)
        for i in (0, 33, 69):
            direct = host(ch.chamfer_estimate_symmetric(dev(q), dev(cl[i]), metric, 0.2, 50, 7,
                                                        n_scales=3))
            assert e[i] == direct[0]
        _, top_all, vals_all = ch.chamfer_retrieve(dev(q), [dev(B) for B in cl], metric, 0.2, 50,
                                                   7, len(cl), n_scales=3)
        brute = sorted((orc.chamfer_symmetric_exact(q, B, metric)[0], i) for i, B in enumerate(cl))
        assert top_all[0] == s
        np.testing.assert_allclose(vals_all, [v for v, _ in brute], rtol=REL, atol=0)
        assert sorted(top_all) == list(range(len(cl)))


def test_retrieval_wide_and_lowp(ch, orc):
    """d = 64 clouds (MFMA exact passes) of mixed sizes, one much larger
    than A: estimates as the oracle's; with BF16 the estimates equal the
    direct BF16 symmetric calls and the re-rank stays exact (float32)."""
    banner("retrieval d=64")
    rng = np.random.default_rng(5)
    A = clouds(400, 1, 64, seed=77)[0]
    cl = [clouds(1, int(n), 64, seed=78 + j)[1] for j, n in enumerate(rng.integers(20, 3000, 9))]
    est, top, vals = ch.chamfer_retrieve(dev(A), [dev(B) for B in cl], 2, 0.2, 0, 3, 3)
    r_est, r_top, r_vals = orc.retrieve(A, cl, 2, 0.2, 0, 3, 3)
    np.testing.assert_allclose(host(est), r_est, rtol=REL, atol=0)
    assert top == r_top
    np.testing.assert_allclose(vals, r_vals, rtol=REL, atol=0)
    est_b, top_b, vals_b = ch.chamfer_retrieve(dev(A), [dev(B) for B in cl], 2, 0.2, 0, 3, 3,
                                               precision=1)
    e = host(est_b)
    for i in range(len(cl)):
        direct = host(ch.chamfer_estimate_symmetric(dev(A), dev(cl[i]), 2, 0.2, 0, 3,
                                                    precision=1))
        assert e[i] == direct[0], i
    for i, v in zip(top_b, vals_b):
        np.testing.assert_allclose(v, orc.chamfer_symmetric_exact(A, cl[i], 2)[0], rtol=REL)


def test_retrieval_nonfinite_cloud_and_edges(ch, orc):
    """A cloud with a NaN coordinate gets a NaN estimate and ranks last, the
    others keep their estimates; k = m and a single cloud work."""
    banner("retrieval edges")
    cl, qs, _ = workloads.retrieval_collection(seed=31, m=9, n_min=40, n_max=90, queries=1)
    q = qs[0]
    bad = [c.copy() for c in cl]
    bad[4][7, 1] = np.nan
    est, top, vals = ch.chamfer_retrieve(dev(q), [dev(B) for B in bad], 1, 0.2, 30, 5, 9)
    e = host(est)
    assert math.isnan(e[4]) and top[-1] == 4 and sorted(top) == list(range(9))
    ref, _, _ = ch.chamfer_retrieve(dev(q), [dev(B) for B in cl], 1, 0.2, 30, 5, 9)
    r = host(ref)
    keep = [i for i in range(9) if i != 4]
    assert np.array_equal(e[keep], r[keep])
    est1, top1, vals1 = ch.chamfer_retrieve(dev(q), [dev(cl[2])], 1, 0.2, 30, 5, 1)
    assert top1 == [0]
    assert host(est1)[0] == pytest.approx(
        orc.chamfer_symmetric_estimate(q, cl[2], 1, 0.2, 30, 5)[0], rel=REL)
    assert vals1[0] == pytest.approx(orc.chamfer_symmetric_exact(q, cl[2], 1)[0], rel=REL)


def test_misaligned_inputs(ch):
    """Point sets starting 4 bytes past a 16-byte boundary (d a multiple of
    4) take the scalar load paths and give the same results."""
    banner("misaligned inputs")
    A, B = clouds(700, 900, 16, seed=41)
    def shifted(X):
        buf = torch.empty(X.size + 1, dtype=torch.float32, device="cuda:0")
        buf[1:] = dev(X.reshape(-1))
        v = buf[1:].view(X.shape)
        assert v.data_ptr() % 16 == 4
        return v
    for metric in (1, 2):
        a0 = host(ch.chamfer_estimate(dev(A), dev(B), metric, 0.2, 0, 3)["eta"])
        a1 = host(ch.chamfer_estimate(shifted(A), shifted(B), metric, 0.2, 0, 3)["eta"])
        assert a0[0] == a1[0]
        e0 = host(ch.chamfer_exact(dev(A), dev(B), metric)[0])
        e1 = host(ch.chamfer_exact(shifted(A), shifted(B), metric)[0])
        assert e0[0] == e1[0]
        r0 = ch.chamfer_aspect_reduce(dev(A), dev(B), metric, 0.2, 3)
        r1 = ch.chamfer_aspect_reduce(shifted(A), shifted(B), metric, 0.2, 3)
        assert np.array_equal(host(r0["t"]), host(r1["t"]))
        assert np.array_equal(host(r0["keys_A"]), host(r1["keys_A"]))


@pytest.mark.parametrize("metric", [1, 2])
@pytest.mark.parametrize("d", [241, 1000, 2048])
def test_wide_points(ch, orc, metric, d):
    """Wide points (the l1 hash reads rows from global memory above 240
    coordinates; l2 above 256 leaves the matrix cores): keys, CrudeNN, the
    estimate and exact CH as the oracle's."""
    n_a, n_b = 300, 410
    banner(f"wide metric={metric} d={d}")
    A, B = clouds(n_a, n_b, d, seed=d + metric)
    D, nn, sc = ch.crude_nn(dev(A), dev(B), metric, 0.2, 4)
    ref = orc.crude_nn(A, B, metric, 0.2, 4)
    assert np.array_equal(host(sc), ref["scale"])
    assert np.array_equal(host(nn), ref["nn"])
    assert np.array_equal(host(D).view(np.uint32), np.asarray(ref["D"], np.float32).view(np.uint32))
    out = ch.chamfer_estimate(dev(A), dev(B), metric, 0.2, 0, 4)
    r = orc.chamfer_estimate(A, B, metric, 0.2, 0, 4)
    assert np.array_equal(host(out["sample_idx"]), r["idx"])
    assert float(host(out["eta"])[0]) == pytest.approx(r["eta"], rel=REL)
    ex = float(host(ch.chamfer_exact(dev(A), dev(B), metric)[0])[0])
    assert ex == pytest.approx(orc.chamfer_exact(A, B, metric)[0], rel=REL)
