"""Serving: requests through the continuous-batching server (same-stage work
of a whole batch in persistent launches replayed from captured graphs) give
the same result as the same call made alone, whatever else is in the batch
or in flight; admission respects the arena and keeps the oldest request
first."""

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
    with ch.ChamferServer(arena, lanes=4) as srv:
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
    with ch.ChamferServer(footprint(ch, r) // 4, lanes=2) as srv:
        with pytest.raises(ch.ChamferError):
            srv.submit(r["A"], r["B"], r["metric"], r["eps"], 0, r["seed"])


def test_server_drains_burst_with_one_lane(ch):
    """One lane: batches run one at a time, and every batch holds the oldest
    request still queued when it was formed (everything fits the arena)."""
    reqs = make_requests(24, seed=5, n_max=5000)
    with ch.ChamferServer(1 << 30, lanes=1) as srv:
        ids = [srv.submit(r["A"], r["B"], r["metric"], r["eps"], 0, r["seed"]) for r in reqs]
        got = {}
        while len(got) < len(ids):
            srv.progress()
            assert srv.stats()["lanes_busy"] <= 1
            for res in srv.results():
                got[res["id"]] = res
        st = srv.stats()
    assert sorted(got) == sorted(ids)
    assert st["batches"] < len(ids)          # requests of one class shared a batch
    pending = set(ids)
    for t in sorted({got[i]["admit_s"] for i in ids}):
        batch = {i for i in ids if got[i]["admit_s"] == t}
        assert min(batch) == min(pending)
        pending -= batch
    assert not pending


def _estimate_alone(ch, r):
    out = ch.chamfer_estimate(r["A"].cuda(), r["B"].cuda(), r["metric"], r["eps"], r.get("T", 0),
                              r["seed"], precision=r.get("precision", 0))
    torch.cuda.synchronize()
    return out


def test_server_one_class_one_graph(ch):
    """Forty small requests of one class: a handful of batches, one graph per
    lane used, each result identical to the call made alone."""
    rng = np.random.default_rng(11)
    reqs = []
    for i in range(40):
        n_a, n_b = (int(x) for x in rng.integers(100, 3000, size=2))
        A = torch.from_numpy(rng.standard_normal((n_a, 3)).astype(np.float32)).pin_memory()
        B = torch.from_numpy(rng.standard_normal((n_b, 3)).astype(np.float32)).pin_memory()
        reqs.append(dict(A=A, B=B, metric=2, eps=0.2, seed=500 + i))
    with ch.ChamferServer(1 << 30, lanes=2) as srv:
        ids = [srv.submit(r["A"], r["B"], r["metric"], r["eps"], 0, r["seed"]) for r in reqs]
        got = {}
        while len(got) < len(ids):
            srv.progress()
            for res in srv.results():
                got[res["id"]] = res
        st = srv.stats()
    assert st["batched"] == len(reqs)
    assert st["batches"] <= 4
    assert st["graphs"] <= 2
    for rid, r in zip(ids, reqs):
        alone = _estimate_alone(ch, r)
        assert got[rid]["status"] == 0
        assert got[rid]["eta"] == float(alone["eta"].item())
        assert got[rid]["W"] == int(alone["W"].item())
        assert got[rid]["s"] == int(alone["s"].item())
        assert got[rid]["D"] == float(alone["D"].item())


def test_server_edge_requests(ch):
    """Degenerate and ragged requests batched together with ordinary ones:
    empty A (finished at submit, eta 0), single points, a partial last tile,
    explicit T, FP8, and a non-finite coordinate (status ENONFINITE, the
    other members unaffected)."""
    rng = np.random.default_rng(12)

    def pts(n, d, scale=1.0):
        return torch.from_numpy((rng.standard_normal((n, d)) * scale).astype(np.float32)).pin_memory()

    bad = pts(300, 16)
    bad[17, 5] = float("nan")
    reqs = [dict(A=pts(0, 16), B=pts(50, 16), metric=2, eps=0.3, seed=1),
            dict(A=pts(1, 16), B=pts(1, 16), metric=2, eps=0.3, seed=2),
            dict(A=pts(65, 16), B=pts(129, 16), metric=2, eps=0.3, seed=3),
            dict(A=pts(1, 3), B=pts(2, 3), metric=1, eps=0.5, seed=4),
            dict(A=pts(777, 3), B=pts(1, 3), metric=1, eps=0.5, seed=5, T=33),
            dict(A=bad, B=pts(400, 16), metric=2, eps=0.3, seed=6),
            dict(A=pts(2000, 16), B=pts(3000, 16), metric=2, eps=0.3, seed=7),
            dict(A=pts(1500, 128, 3.0), B=pts(2500, 128, 3.0), metric=2, eps=0.2, seed=8,
                 precision=2),
            dict(A=pts(1500, 128, 3.0), B=pts(2500, 128, 3.0), metric=2, eps=0.2, seed=9,
                 precision=2)]
    with ch.ChamferServer(1 << 30, lanes=2) as srv:
        ids = [srv.submit(r["A"], r["B"], r["metric"], r["eps"], r.get("T", 0), r["seed"],
                          precision=r.get("precision", 0)) for r in reqs]
        got = {}
        while len(got) < len(ids):
            srv.progress()
            for res in srv.results():
                got[res["id"]] = res
    for rid, r in zip(ids, reqs):
        res = got[rid]
        if r["A"].shape[0] == 0:
            assert res["status"] == 0 and res["eta"] == 0.0
            continue
        alone = _estimate_alone(ch, r)
        if r is reqs[5]:
            assert res["status"] == -4 and int(alone["status"].item()) == -4
            continue
        assert res["status"] == 0, rid
        assert res["eta"] == float(alone["eta"].item()), rid
        assert res["W"] == int(alone["W"].item())


def test_server_warm(ch):
    """warm() instantiates a class graph on every lane once; a request of
    that class then adds no graph; bad classes are rejected."""
    with ch.ChamferServer(1 << 28, lanes=3) as srv:
        srv.warm(3, 2)
        srv.warm(3, 2)
        assert srv.stats()["graphs"] == 3
        srv.warm(128, 2, precision=1)
        assert srv.stats()["graphs"] == 6
        for bad in ((0, 2), (4096, 2), (3, 5)):
            with pytest.raises(ch.ChamferError):
                srv.warm(*bad)
        rng = np.random.default_rng(13)
        A = torch.from_numpy(rng.standard_normal((500, 3)).astype(np.float32)).pin_memory()
        B = torch.from_numpy(rng.standard_normal((700, 3)).astype(np.float32)).pin_memory()
        rid = srv.submit(A, B, 2, 0.2, 0, 77)
        got = []
        while not got:
            srv.progress()
            got = srv.results()
        assert srv.stats()["graphs"] == 6
    alone = _estimate_alone(ch, dict(A=A, B=B, metric=2, eps=0.2, seed=77))
    assert got[0]["id"] == rid and got[0]["eta"] == float(alone["eta"].item())


def test_server_matches_oracle(orc, ch):
    """Every served result against the CPU oracle (the Chamfer-Estimate
    figure run on the same request): eta within 1e-5 relative, the
    fixed-point total W, exponent s and normaliser D exactly.  The requests
    are the serving mix (d = 3 surface clouds and d = 128 clusters, l1/l2,
    eps 0.1/0.2) at reduced sizes, plus d = 16 and d = 64 Gaussian pairs and
    BF16 exact passes, all submitted at once to an arena that holds only a
    few of them, so they batch and overlap."""
    import workloads
    stream = workloads.serving_stream(seed=77, count=28, rate_hz=500.0, n_min=300, n_max=6000)
    reqs = []
    for q in stream:
        A, B = workloads.request_clouds(q)
        reqs.append(dict(A=A, B=B, metric=q.metric, eps=q.eps, seed=q.seed, precision=0))
    rng = np.random.default_rng(78)
    for i in range(12):
        d = [16, 64][i % 2]
        n_a, n_b = (int(x) for x in rng.integers(200, 5000, size=2))
        A = (rng.standard_normal((n_a, d)) * 2).astype(np.float32)
        B = (rng.standard_normal((n_b, d)) * 2).astype(np.float32)
        metric = 1 + (i % 3 != 0)
        prec = 1 if metric == 2 and i % 4 == 1 else 0
        reqs.append(dict(A=A, B=B, metric=metric, eps=[0.1, 0.2][i % 2], seed=900 + i,
                         precision=prec))
    for r in reqs:
        r["At"] = torch.from_numpy(r["A"]).pin_memory()
        r["Bt"] = torch.from_numpy(r["B"]).pin_memory()
    biggest = max(ch.chamfer_workspace_bytes(r["A"].shape[0], r["B"].shape[0], r["A"].shape[1],
                                             r["metric"], r["eps"], 0, precision=r["precision"])
                  + 4 * r["A"].shape[1] * (r["A"].shape[0] + r["B"].shape[0]) + 4096
                  for r in reqs)
    print(f"[case] serving vs oracle: {len(reqs)} requests", flush=True)
    got = {}
    with ch.ChamferServer(4 * biggest, lanes=4) as srv:
        ids = [srv.submit(r["At"], r["Bt"], r["metric"], r["eps"], 0, r["seed"],
                          precision=r["precision"]) for r in reqs]
        while len(got) < len(ids):
            srv.progress()
            for res in srv.results():
                got[res["id"]] = res
        st = srv.stats()
    assert st["batches"] < len(reqs)
    for rid, r in zip(ids, reqs):
        res = got[rid]
        assert res["status"] == 0, rid
        ref = orc.chamfer_estimate(r["A"], r["B"], r["metric"], r["eps"], 0, r["seed"])
        assert res["W"] == ref["W"] and res["s"] == ref["s"], rid
        assert res["D"] == ref["D_norm"], rid
        assert res["eta"] == pytest.approx(ref["eta"], rel=1e-5), (rid, r["A"].shape, r["metric"])
