"""The reduction to bounded aspect ratio on the GPU against the oracle: the
sketch's t_a and maximum bit for bit, the derived exponents and padding
value exactly, the partition keys and padded copies bit for bit, and the
estimate after the reduction within the estimator's tolerance (one part:
bit-identical to the plain estimate; several parts: the sum of the parts'
estimates)."""


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


def clouds(n_a, n_b, d, seed):
    A, _ = workloads.clusters_l2(seed=seed, n=n_a, d=d, k=max(2, n_a // 50), n_b=1)
    _, B = workloads.clusters_l2(seed=seed, n=1, d=d, k=max(2, n_a // 50), n_b=n_b)
    return A, B


def far_groups(groups, per, seed):
    """`groups` clusters 1e35 apart along the first axis, `per` points of A
    and of B in each, neighbours ~1e24 apart inside a group (resolved by the
    double-precision projection)."""
    rng = np.random.default_rng(seed)
    A, B = [], []
    for g in range(groups):
        base = np.array([g * 1e35, 0.0])
        A.append(base + rng.uniform(0, 1e25, size=(per, 2)))
        B.append(base + rng.uniform(0, 1e25, size=(per, 2)))
    return np.concatenate(A).astype(np.float32), np.concatenate(B).astype(np.float32)


def check_reduce(ch, orc, A, B, metric, seed, eps=0.2):
    got = ch.chamfer_aspect_reduce(dev(A), dev(B), metric, eps, seed, pad=True)
    ref = orc.aspect_reduce(A, B, metric, eps, seed)
    info = got["info"]
    assert np.array_equal(host(got["t"]), ref["t"])
    assert info["max_t"] == ref["max_t"]
    assert info["ch1"] == pytest.approx(ref["ch1"], rel=1e-12)
    assert bool(info["degenerate"]) == ref["degenerate"]
    if not ref["degenerate"]:
        assert info["e_M"] == ref["e_M"] and info["e_part"] == ref["e_part"]
        assert info["eta_lo"] == ref["eta_lo"] and info["eta_hi"] == ref["eta_hi"]
    assert info["pad_dims"] == ref["m"]
    assert np.float32(info["pad_value"]) == ref["q"]
    kA = host(got["keys_A"]).view(np.uint64)
    kB = host(got["keys_B"]).view(np.uint64)
    assert np.array_equal(kA, ref["keys_A"]) and np.array_equal(kB, ref["keys_B"])
    one = bool(np.all(ref["keys_A"] == ref["keys_A"][0]) and np.all(ref["keys_B"] == ref["keys_A"][0]))
    assert bool(info["one_part"]) == one
    assert np.array_equal(host(got["A_pad"]), orc.pad(A, ref["m"], 0, seed, ref["q"]))
    assert np.array_equal(host(got["B_pad"]), orc.pad(B, ref["m"], 1, seed, ref["q"]))
    return info, ref


@pytest.mark.parametrize("metric", [1, 2])
@pytest.mark.parametrize("shape", [(1000, 777, 3), (2049, 3001, 16), (300, 2500, 128),
                                   (130, 211, 37), (1, 1, 5)])
def test_reduce_parity(ch, orc, metric, shape):
    n_a, n_b, d = shape
    banner(f"reduce metric={metric} shape={shape}")
    A, B = clouds(n_a, n_b, d, seed=3 * d + n_a)
    info, _ = check_reduce(ch, orc, A, B, metric, seed=17 + d)
    assert info["one_part"] == 1 or n_a == 1


def test_reduce_far_groups(ch, orc):
    """Groups far apart: the partition splits them on both sides alike, and
    the estimate after the reduction is the oracle's sum over the parts."""
    banner("reduce far groups")
    split = 0
    for seed in range(6):
        A, B = far_groups(4, 2, seed)
        info, ref = check_reduce(ch, orc, A, B, 1, seed)
        pl = orc.parts(ref["keys_A"], ref["keys_B"])
        r = orc.chamfer_estimate_reduced(A, B, 1, 0.2, 20, seed, orc.REDUCE_PARTITION)
        got = float(host(ch.chamfer_estimate(dev(A), dev(B), 1, 0.2, 20, seed,
                                             reduction=ch.REDUCE_PARTITION)["eta"])[0])
        assert got == pytest.approx(r["eta"], rel=REL)
        split += pl is not None and len(pl) > 1
    assert split >= 3


@pytest.mark.parametrize("metric", [1, 2])
@pytest.mark.parametrize("shape", [(2049, 3001, 16), (700, 2000, 64), (1000, 777, 3)])
def test_reduced_estimate_parity(ch, orc, metric, shape):
    """One part: the partition-only reduction is bit-identical to the plain
    estimate; with padding (d + m coordinates) the estimate matches the
    oracle's on the padded sets."""
    n_a, n_b, d = shape
    banner(f"reduced estimate metric={metric} shape={shape}")
    A, B = clouds(n_a, n_b, d, seed=5 * d + 1)
    plain = host(ch.chamfer_estimate(dev(A), dev(B), metric, 0.2, 0, 9)["eta"])[0]
    part = host(ch.chamfer_estimate(dev(A), dev(B), metric, 0.2, 0, 9,
                                    reduction=ch.REDUCE_PARTITION)["eta"])[0]
    assert part == plain
    padded = host(ch.chamfer_estimate(dev(A), dev(B), metric, 0.2, 0, 9,
                                      reduction=ch.REDUCE_PAD)["eta"])[0]
    ref = orc.chamfer_estimate_reduced(A, B, metric, 0.2, 0, 9, orc.REDUCE_PAD)
    assert ref["parts"] == 1
    assert padded == pytest.approx(ref["eta"], rel=REL)
    exact = orc.chamfer_exact(A, B, metric)[0]
    assert abs(padded - exact) <= 0.5 * exact


def test_reduction_degenerate(ch, orc):
    """A inside B: every t_a = 0, no partition, eta = 0."""
    banner("reduce degenerate")
    _, B = clouds(1, 500, 8, seed=4)
    A = B[:100].copy()
    info, _ = check_reduce(ch, orc, A, B, 2, 3)
    assert info["degenerate"] == 1
    for red in (1, 2):
        eta = host(ch.chamfer_estimate(dev(A), dev(B), 2, 0.2, 0, 3, reduction=red)["eta"])[0]
        assert eta == 0.0
