"""GPU parity of the l2 exact pass on the BF16 matrix cores (two-term split
of each coordinate, certified against the canonical float32 distance).

The pass must return exactly what the oracle's float32 nearest-neighbour
search returns (minimum and arg-min, ties to the lower index) on inputs
chosen to stress the certificate: near-ties far below the split's rounding,
large common offsets (large error bound E relative to the gaps), norms that
overflow (E infinite: every chunk rescanned), subnormal coordinates,
duplicated rows, every padded-dimension class with ragged tails, and both
forms of the pass (three products, and four for launches over many
queries).
"""

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

L2 = 2


@pytest.fixture(scope="module")
def ch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_03043_amd as lib
    lib.lib()
    return lib


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def banner(msg):
    print(f"[case] {msg}", flush=True)


def check_exact(ch, orc, A, B):
    _, rmin, rnn = ch.chamfer_exact(dev(A), dev(B), L2)
    m32, a32 = orc.nn_f32(A, B, L2)
    got_nn, got_min = host(rnn), host(rmin)
    bad = np.flatnonzero(got_nn != a32)
    assert bad.size == 0, f"{bad.size} arg-min mismatches, first row {bad[:5]}"
    assert np.array_equal(got_min.view(np.uint32), m32.view(np.uint32))


@pytest.mark.parametrize("d", [12, 31, 32, 33, 64, 65, 127, 128, 129, 200, 256])
def test_dimension_classes(ch, orc, d):
    banner(f"split d={d}")
    A, B = workloads.clusters_l2(seed=100 + d, n=777, d=d, k=20, n_b=1533)
    check_exact(ch, orc, A, B)


@pytest.mark.parametrize("d", [64, 128])
def test_four_product_form(ch, orc, d):
    """20000 queries: the launch takes the four-product form."""
    banner(f"split four products d={d}")
    A, B = workloads.clusters_l2(seed=5 + d, n=20000, d=d, k=200, n_b=2100)
    check_exact(ch, orc, A, B)


@pytest.mark.parametrize("n_a", [1000, 20000])
def test_near_ties(ch, orc, n_a):
    """Each query has two rows of B at distances that differ by a few float32
    ulps, far below the BF16 split's rounding: only the exact rescan can
    separate them."""
    banner(f"split near ties n_a={n_a}")
    rng = np.random.default_rng(3)
    d = 96
    A = rng.normal(size=(n_a, d)).astype(np.float32)
    base = A[rng.integers(0, n_a, size=1500)]
    B = np.empty((3000, d), np.float32)
    B[0::2] = base + np.float32(0.25)
    B[1::2] = base + np.float32(0.25)
    B[1::2, 0] = np.nextafter(B[1::2, 0], np.float32(np.inf))
    check_exact(ch, orc, A, B)


def test_large_offset(ch, orc):
    """A common offset of 1e4 in every coordinate: |x| |b| is 1e8 times the
    spread, so the error bound covers many rows and most chunks rescan."""
    banner("split large offset")
    A, B = workloads.clusters_l2(seed=9, n=1200, d=64, k=30, n_b=2500)
    A = (A + np.float32(1e4)).astype(np.float32)
    B = (B + np.float32(1e4)).astype(np.float32)
    check_exact(ch, orc, A, B)


def test_overflowing_norm(ch, orc):
    """One row of B with a coordinate near FLT_MAX (|b|^2 and its BF16 split
    overflow): the bound is infinite and every chunk is rescanned."""
    banner("split overflowing norm")
    A, B = workloads.clusters_l2(seed=21, n=500, d=48, k=10, n_b=900)
    B[17, 3] = np.float32(3.39e38)
    check_exact(ch, orc, A, B)


def test_subnormal_coordinates(ch, orc):
    """Coordinates around 1e-19 (squared distances near the float32
    subnormal range) with some at 1e-39 (float32 and BF16 subnormals)."""
    banner("split subnormals")
    rng = np.random.default_rng(4)
    A = (rng.normal(size=(400, 40)) * 1e-19).astype(np.float32)
    B = (rng.normal(size=(700, 40)) * 1e-19).astype(np.float32)
    A[:, ::5] = (rng.normal(size=(400, 8)) * 1e-39).astype(np.float32)
    B[::3, 1::5] = (rng.normal(size=(234, 8)) * 1e-39).astype(np.float32)
    B[::7] = 0.0
    check_exact(ch, orc, A, B)


def test_duplicate_rows_lowest_index(ch, orc):
    banner("split duplicates")
    A, B0 = workloads.clusters_l2(seed=13, n=600, d=128, k=12, n_b=400)
    B = np.concatenate([B0, B0, B0[::-1]]).astype(np.float32)
    check_exact(ch, orc, A, B)
    _, _, rnn = ch.chamfer_exact(dev(A), dev(B), L2)
    assert host(rnn).max() < 400   # the first copy always wins


def test_estimate_matches_oracle_on_offset_data(ch, orc):
    """The estimator's exact pass over the draws on offset data (many
    rescans) still gives the oracle's eta."""
    banner("split estimate offset")
    A, B = workloads.clusters_l2(seed=31, n=3000, d=64, k=40, n_b=2800)
    A = (A + np.float32(300.0)).astype(np.float32)
    B = (B + np.float32(300.0)).astype(np.float32)
    out = ch.chamfer_estimate(dev(A), dev(B), L2, 0.2, 400, 5)
    ref = orc.chamfer_estimate(A, B, L2, 0.2, 400, 5)
    assert np.array_equal(host(out["sample_idx"]), ref["idx"])
    m32, a32 = orc.nn_f32(A, B, L2, rows=ref["idx"])
    assert np.array_equal(host(out["sample_nn"]), a32)
    assert np.array_equal(host(out["sample_min"]).view(np.uint32), m32.view(np.uint32))
    assert float(host(out["eta"])[0]) == pytest.approx(ref["eta"], rel=1e-5)


def check_estimate_draws(ch, orc, A, B, eps, T, seed):
    out = ch.chamfer_estimate(dev(A), dev(B), L2, eps, T, seed)
    ref = orc.chamfer_estimate(A, B, L2, eps, T, seed)
    assert np.array_equal(host(out["sample_idx"]), ref["idx"])
    m32, a32 = orc.nn_f32(A, B, L2, rows=ref["idx"])
    assert np.array_equal(host(out["sample_nn"]), a32)
    assert np.array_equal(host(out["sample_min"]).view(np.uint32), m32.view(np.uint32))


def test_estimate_draws_near_ties(ch, orc):
    """The estimator's pass over its draws (chunk candidates recorded, then
    certified per draw) on near-ties one float32 ulp apart: each draw's two
    nearest rows of B are in different chunks or the same one."""
    banner("split estimate near ties")
    rng = np.random.default_rng(8)
    d = 96
    A = rng.normal(size=(3000, d)).astype(np.float32)
    base = A[rng.integers(0, 3000, size=1500)]
    B = np.empty((3000, d), np.float32)
    B[0::2] = base + np.float32(0.25)
    B[1::2] = base + np.float32(0.25)
    B[1::2, 0] = np.nextafter(B[1::2, 0], np.float32(np.inf))
    # and a second copy far away in B's order (another chunk)
    B = np.concatenate([B, B[::-1]]).astype(np.float32)
    check_estimate_draws(ch, orc, A, B, 0.2, 600, 3)


def test_estimate_draws_duplicates(ch, orc):
    """Exact duplicate rows of B next to each other (equal candidates in one
    chunk: the chunk is rescanned) and the lowest index must win."""
    banner("split estimate duplicates")
    A, B0 = workloads.clusters_l2(seed=17, n=2500, d=128, k=25, n_b=900)
    B = np.repeat(B0, 3, axis=0).astype(np.float32)
    check_estimate_draws(ch, orc, A, B, 0.2, 500, 11)


@pytest.mark.parametrize("d", [16, 64, 200])
def test_estimate_draws_dimension_classes(ch, orc, d):
    banner(f"split estimate d={d}")
    A, B = workloads.clusters_l2(seed=60 + d, n=4000, d=d, k=40, n_b=5000)
    check_estimate_draws(ch, orc, A, B, 0.2, 700, 2)


@pytest.mark.parametrize("offset", [0.0, 300.0])
def test_estimate_draws_long_chunks(ch, orc, offset):
    """2000 draws against 80000 rows at d = 16: chunks of more than 512
    rows, whose rescans are cut into pieces over the whole device; with an
    offset of 300 most (draw, chunk) pairs are rescanned."""
    banner(f"split estimate long chunks offset={offset}")
    A, B = workloads.clusters_l2(seed=77, n=5000, d=16, k=50, n_b=80000)
    A = (A + np.float32(offset)).astype(np.float32)
    B = (B + np.float32(offset)).astype(np.float32)
    check_estimate_draws(ch, orc, A, B, 0.1, 2000, 4)


def test_estimate_draws_many_chunks(ch, orc):
    """100 draws against 200000 rows: one block of draws, so B is cut into
    more than 512 chunks and the per-draw certificate reads its records from
    memory in each pass instead of holding them in registers."""
    banner("split estimate many chunks")
    A, B = workloads.clusters_l2(seed=91, n=3000, d=16, k=60, n_b=200000)
    check_estimate_draws(ch, orc, A, B, 0.2, 100, 6)
