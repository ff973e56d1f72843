"""Serving: requests through the continuous-batching server give the same
result as the same call made alone, whatever else is in flight; admission
respects the arena."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_03043_amd as lib
    lib.lib()
    return lib


def make_requests(n, seed=0, n_max=40000):
    """Mixed requests; host arrays are pinned so copy-in is asynchronous."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        d = [3, 16, 128, 64][i % 4]
        metric = 1 + (i % 2)
        n_a, n_b = (int(x) for x in rng.integers(50, n_max, size=2))
        A = torch.from_numpy((rng.standard_normal((n_a, d)) * rng.uniform(0.5, 5))
                             .astype(np.float32)).pin_memory()
        B = torch.from_numpy((rng.standard_normal((n_b, d)) * rng.uniform(0.5, 5))
                             .astype(np.float32)).pin_memory()
        eps = [0.1, 0.2][i % 2]
        prec = 1 if (metric == 2 and d >= 12 and i % 3 == 0) else 0
        reqs.append(dict(A=A, B=B, metric=metric, eps=eps, seed=1000 + i, precision=prec))
    return reqs


def footprint(ch, r):
    n_a, d = r["A"].shape
    return (ch.chamfer_workspace_bytes(n_a, r["B"].shape[0], d, r["metric"], r["eps"], 0,
                                       precision=r["precision"])
            + 4 * d * (n_a + r["B"].shape[0]) + 4096)


def test_server_same_alone_and_in_mix(ch):
    reqs = make_requests(48)
    biggest = max(footprint(ch, r) for r in reqs)
    arena = 3 * biggest  # only a few requests fit at once: admission binds
    results = {}
    max_in_flight = 0
    with ch.ChamferServer(arena, slots=8) as srv:
        ids = [srv.submit(r["A"], r["B"], r["metric"], r["eps"], 0, r["seed"],
                          precision=r["precision"]) for r in reqs]
        while len(results) < len(ids):
            srv.progress()
            st = srv.stats()
            max_in_flight = max(max_in_flight, st["in_flight"])
            assert st["arena_used"] <= arena
            for res in srv.results():
                results[res["id"]] = res
        assert srv.stats()["arena_peak"] <= arena
    assert max_in_flight >= 2          # requests really overlapped
    for rid, r in zip(ids, reqs):
        res = results[rid]
        assert res["status"] == 0
        alone = ch.chamfer_estimate(r["A"].cuda(), r["B"].cuda(),
                                    r["metric"], r["eps"], 0, r["seed"], precision=r["precision"])
        torch.cuda.synchronize()
        assert res["eta"] == float(alone["eta"].item()), (rid, r["A"].shape, r["B"].shape)
        assert res["W"] == int(alone["W"].item())


def test_server_rejects_oversized(ch):
    r = make_requests(1)[0]
    with ch.ChamferServer(footprint(ch, r) // 4, slots=2) as srv:
        with pytest.raises(ch.ChamferError):
            srv.submit(r["A"], r["B"], r["metric"], r["eps"], 0, r["seed"])


def test_server_drains_burst_with_one_slot(ch):
    reqs = make_requests(10, seed=5, n_max=5000)
    with ch.ChamferServer(1 << 30, slots=1) as srv:
        ids = [srv.submit(r["A"], r["B"], r["metric"], r["eps"], 0, r["seed"]) for r in reqs]
        got = {}
        while len(got) < len(ids):
            srv.progress()
            assert srv.stats()["in_flight"] <= 1
            for res in srv.results():
                got[res["id"]] = res
    assert sorted(got) == sorted(ids)
    # admitted in order (one slot, everything fits)
    admits = [got[i]["admit_s"] for i in ids]
    assert admits == sorted(admits)
