"""The partitioned LDS table build keeps aside the keys whose linear probe
runs past the end of their region (it never wraps); a global insert then
places them, continuing into the next region or, past the last slot, at
the start of the table.  These cases are chosen so that the build does keep
keys aside (counted here on the CPU from the oracle's keys, with the build's
home slots and region sizes), and the CrudeNN bits are compared with the
oracle's.
"""

import numpy as np
import pytest

import workloads

GOLDEN = 0x9E3779B97F4A7C15  # the home-slot multiplier
REGION_BITS = 11


def table_log2cap(n_b):
    """2^log2cap >= 2 n_B slots per scale, at least 64."""
    return max(6, (2 * n_b - 1).bit_length())


def home_slots(keys, log2cap):
    k = np.asarray(keys, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return (k * np.uint64(GOLDEN)) >> np.uint64(64 - log2cap)


def parking_spills(homes, log2cap):
    """Keys a region-by-region build without wrap-around keeps aside: in
    each region of 2^min(log2cap, 11) slots a key takes the first free slot
    at or after its home; one that finds none before the region's end is
    kept aside.  The count does not depend on the order of insertion."""
    rb = min(log2cap, REGION_BITS)
    size = 1 << rb
    homes = np.sort(np.asarray(homes, dtype=np.int64))
    spilled = 0
    for region in np.unique(homes >> rb):
        nxt = 0
        for h in homes[(homes >> rb) == region] & (size - 1):
            pos = max(int(h), nxt)
            if pos >= size:
                spilled += 1
            else:
                nxt = pos + 1
    return spilled


def build_spills(keys_b, n_b):
    lc = table_log2cap(n_b)
    return [parking_spills(home_slots(np.unique(k), lc), lc) for k in keys_b]


def test_parking_spills_by_hand():
    # one region of 8 slots (log2cap 3)
    assert parking_spills([0, 0, 0], 3) == 0
    assert parking_spills([7, 7], 3) == 1
    assert parking_spills([6, 7, 7], 3) == 1
    assert parking_spills([5, 6, 6, 6], 3) == 1
    assert parking_spills([1, 3, 5, 7], 3) == 0
    # regions of 2048 slots (log2cap 12): the end of region 0 does not
    # continue into region 1 in the build
    assert parking_spills([2047, 2047, 2048], 12) == 1
    assert parking_spills([2046, 2047, 2048, 2048], 12) == 0


def test_table_log2cap():
    assert table_log2cap(1) == 6
    assert table_log2cap(32) == 6
    assert table_log2cap(33) == 7
    assert table_log2cap(100_000) == 18
    assert table_log2cap(1_000_000) == 21


def spill_case(orc, metric, n_a, n_b, d, L):
    """The first seed (of 40) whose B keys make the build keep keys aside."""
    for seed in range(40):
        rng = np.random.default_rng(1000 + seed)
        A = rng.uniform(-10, 10, (n_a, d)).astype(np.float32)
        B = rng.uniform(-10, 10, (n_b, d)).astype(np.float32)
        c = orc.crude_nn(A, B, metric, 0.2, seed, n_scales=L)
        if sum(build_spills(c["keys_b"], n_b)) > 0:
            return seed, A, B, c
    return None


@pytest.mark.gpu
@pytest.mark.parametrize("metric,n_a,n_b,d,L", [(2, 500, 60, 16, 12), (1, 500, 60, 8, 12),
                                                 (2, 3000, 3000, 32, 14)])
def test_spilled_keys_bit_exact(orc, metric, n_a, n_b, d, L):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_03043_amd as ch
    case = spill_case(orc, metric, n_a, n_b, d, L)
    assert case is not None, "no seed with keys kept aside"
    seed, A, B, c = case
    print(f"[case] spilled keys metric={metric} n_b={n_b} seed={seed}", flush=True)
    out = ch.chamfer_estimate(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), metric,
                              0.2, 100, seed, n_scales=L)
    torch.cuda.synchronize()
    assert np.array_equal(out["crude_scale"].cpu().numpy(), c["scale"])
    assert np.array_equal(out["crude_nn"].cpu().numpy(), c["nn"])
    assert np.array_equal(out["crude_D"].cpu().numpy().view(np.uint32), c["D"].view(np.uint32))
