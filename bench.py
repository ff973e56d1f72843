#!/usr/bin/env python3
"""Benchmark of the Chamfer estimator on one MI355X.

One step = one chamfer_estimate call (calibration, grid tables, bucketing of
B, CrudeNN probe of A, fixed-point weights and draws, exact nearest
neighbours of the T draws, reweighted mean) on inputs already resident in
HBM.  The default workload is l2, |A| = |B| = 100,000, d = 128, 1000-cluster
Gaussian mixture, eps = 0.1, T = 2000, L = 20 scales.  Also timed on the
same inputs: brute-force exact CH on the GPU (chamfer_exact), per-stage
times from HIP events recorded by the library, per-step latency
percentiles, and the CPU oracle on the host.

Prints one JSON line.  --gpus N with N > 1 exits with a message: this build
runs on one GPU.
"""

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC_NAME = "Chamfer points/s at ε=0.1 vs GPU brute force; %HBM/MFMA peak; p50/p99 ms"

# MI355X published peaks.
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_TFLOPS = 157.3   # 256 CUs x 256 FP32 flops/clk x 2.4 GHz
BF16_MFMA_TFLOPS = 2500.0
FP8_MFMA_TFLOPS = 5000.0

WORKLOADS = {
    # name: (generator, kwargs, metric, eps, T, L, description)
    "l2_100k_d128": ("clusters_l2", dict(n=100_000, d=128, k=1000), 2, 0.1, 2000, 20,
                     "l2, |A|=|B|=100000, d=128, 1000-cluster Gaussian mixture "
                     "(centres N(0,16 I), sigma~U[0.2,1]); eps=0.1, T=2000, L=20"),
    "l2_1m_d128": ("clusters_l2", dict(n=1_000_000, d=128, k=1000), 2, 0.1, 2000, 24,
                   "l2, |A|=|B|=1000000, d=128, 1000-cluster Gaussian mixture; eps=0.1, "
                   "T=2000, L=24"),
    "l1_1m_d64": ("mixed_l1", dict(n=1_000_000, d=64, k=5000), 1, 0.1, 2000, 24,
                  "l1, |A|=|B|=1000000, d=64, 70% 5000-cluster Laplace(0,0.5) mixture + "
                  "30% uniform [-50,50]^64; eps=0.1, T=2000, L=24"),
    "l2_1m_d256": ("precision_l2", dict(n=1_000_000, d=256, k=10_000), 2, 0.1, 2000, 24,
                   "l2, |A|=|B|=1000000, d=256, 10000-cluster Gaussian mixture (centres "
                   "N(0,I), sigma=0.3); eps=0.1, T=2000, L=24"),
    "l2_4k_d16": ("small_l2", dict(n=4096, d=16), 2, 0.2, 512, 15,
                  "l2, |A|=|B|=4096, d=16, 16-centre mixture; eps=0.2, T=512, L=15"),
}


def loaded_hip_runtime():
    """Path of the HIP runtime already mapped into this process (the one torch
    and libchamfer use), so events and streams come from one runtime."""
    with open("/proc/self/maps") as f:
        for line in f:
            path = line.split()[-1]
            if "libamdhip64.so" in path:
                return path
    return "libamdhip64.so.7"


class HipEvents:
    """hipEvent_t handles through the HIP runtime (ctypes)."""

    def __init__(self, n):
        self.hip = ctypes.CDLL(loaded_hip_runtime())
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float),
                                                 ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.arr = (ctypes.c_void_p * n)()
        for i in range(n):
            h = ctypes.c_void_p()
            rc = self.hip.hipEventCreate(ctypes.byref(h))
            if rc != 0:
                raise RuntimeError(f"hipEventCreate failed: {rc}")
            self.arr[i] = h

    def ms(self, i, j):
        self.hip.hipEventSynchronize(self.arr[j])
        out = ctypes.c_float()
        rc = self.hip.hipEventElapsedTime(ctypes.byref(out), self.arr[i], self.arr[j])
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed: {rc}")
        return float(out.value)

    def close(self):
        for h in self.arr:
            self.hip.hipEventDestroy(h)


def algorithmic_sample_pass(metric, T, n_b, d):
    """Work of the exact pass over the draws: T * n_B * d coordinate terms.
    l2 (12 <= d <= 256) runs on the BF16 matrix cores: 2 flops (one
    multiply-add of x.b) per term, each computed as three BF16 products of
    the two-term split of the coordinates (four when T >= 16384), so the
    peak is the BF16 MFMA peak and the form's own ceiling is that peak over
    the product count.  l1 runs on the vector ALU: 2 flops (subtract, add
    |t|) per term, against the FP32 vector peak."""
    elems = float(T) * n_b * d
    if metric == 2 and 12 <= d <= 256:
        products = 4 if T >= 16384 else 3
        return dict(bound="mfma", unit="TFLOP/s", ops=2.0 * elems, peak=BF16_MFMA_TFLOPS,
                    products=products,
                    note=f"2 flops (x.b multiply-add) per coordinate term, computed as {products} "
                         "BF16 MFMA products of the two-term split coordinates")
    if metric == 2:
        return dict(bound="alu", unit="TFLOP/s", ops=3.0 * elems, peak=FP32_VECTOR_TFLOPS,
                    note="3 FP32 flops (subtract, fma) per coordinate term on the vector ALU")
    return dict(bound="alu", unit="TFLOP/s", ops=2.0 * elems, peak=FP32_VECTOR_TFLOPS,
                note="2 FP32 flops (subtract, add |t|) per coordinate term on the vector ALU")


def measured_traffic(workload, kernel_ms):
    """HBM bytes per launch of the exact pass over the draws (the sum over its
    kernels) from the committed counter record (FETCH_SIZE/WRITE_SIZE,
    copy-calibrated), or None when there is no record for this workload or
    the kernels' sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if not rec.get("sources"):
        return None
    for src, sha in rec["sources"].items():
        path = os.path.join(ROOT, src)
        if not os.path.exists(path):
            return None
        with open(path, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != sha:
                return None
    return rec["traffic_bytes"]


# Calls timed with stage events for the per-stage split and p50/p99 latency.
LATENCY_CALLS = 100

# Rows of A in the CPU oracle's timed brute-force sample.
CPU_BRUTE_ROWS = 500

# Points per set for the CPU oracle's timed sample (full workload when smaller).
CPU_SAMPLE_POINTS = 250_000


def cpu_baseline(args, A, B, metric, eps, T, L, seed):
    import oracle
    n_a = min(A.shape[0], CPU_SAMPLE_POINTS)
    n_b = min(B.shape[0], CPU_SAMPLE_POINTS)
    full = n_a == A.shape[0] and n_b == B.shape[0]
    As, Bs = A[:n_a], B[:n_b]
    t0 = time.perf_counter()
    ref = oracle.chamfer_estimate(As, Bs, metric, eps, T, seed, n_scales=L)
    dt = time.perf_counter() - t0
    cores = oracle.threads()
    # the same estimate on one thread, on a tenth of the sample's rows of A
    # and of B (the exact pass is linear in T n_B, the rest in n_A + n_B)
    oracle.set_threads(1)
    n1, m1 = max(1, n_a // 10), max(1, n_b // 10)
    t0 = time.perf_counter()
    oracle.chamfer_estimate(As[:n1], Bs[:m1], metric, eps, T, seed, n_scales=L)
    dt1 = time.perf_counter() - t0
    oracle.set_threads(cores)
    # the oracle's float64 brute force on a sample of rows of A, all of B
    rows = np.arange(0, n_a, max(1, n_a // CPU_BRUTE_ROWS), dtype=np.int32)[:CPU_BRUTE_ROWS]
    t0 = time.perf_counter()
    oracle.nn_f64(As, Bs, metric, rows=rows)
    dtb = time.perf_counter() - t0
    what = (f"full workload (|A|={n_a}, |B|={n_b})" if full else
            f"the first {n_a} points of A and {n_b} of B (same generator)")
    return dict(value=(n_a + n_b) / dt, unit="points/s", cores=cores,
                brute_force={"rows": int(len(rows)), "seconds": dtb,
                             "full_seconds_extrapolated": dtb * n_a / max(1, len(rows)),
                             "kind": "float64, all OpenMP threads"},
                kind="oracle", seconds=dt, host_cpu=host_cpu(), nproc=os.cpu_count(),
                single_thread={"points_per_s": (n1 + m1) / dt1, "seconds": dt1,
                               "sample": f"|A|={n1}, |B|={m1}, same eps, T and L"},
                sample=f"{what}, one estimate with the same eps, T and L; double-precision "
                       f"exact pass on {cores} OpenMP threads, hashing "
                       f"single-threaded"), (ref if full else None)


def host_cpu():
    """The host CPU model (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def precision_report(args, ch, torch, A, B, At, Bt, metric, eps, T, L, desc):
    """Exact CH and the estimator with float32, BF16 and FP8-E4M3 distance
    tiles (float32 re-rank of each row's top candidates, float64 sums).
    Errors: full CH against the canonical float32 CH (each row of which is
    within (d+4) 2^-24 relative of float64), and a seeded sample of rows
    against the float64 oracle."""
    import oracle
    n_a, d = A.shape
    seed = 1
    rows = np.random.default_rng(7).choice(n_a, size=min(n_a, 1000), replace=False)
    rows = np.sort(rows).astype(np.int32)
    t0 = time.perf_counter()
    m64, a64 = oracle.nn_f64(A, B, metric, rows=rows)
    oracle_s = time.perf_counter() - t0
    res = {"workload": desc, "sample_rows": int(len(rows)), "oracle_rows_seconds": oracle_s}
    ref = {}
    for prec, name in ((0, "fp32"), (1, "bf16"), (2, "fp8")):
        ch.chamfer_exact(At, Bt, metric, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.brute_steps):
            chv, rmin, rnn = ch.chamfer_exact(At, Bt, metric, precision=prec)
        torch.cuda.synchronize()
        bt = (time.perf_counter() - t0) / args.brute_steps
        for _ in range(args.warmup):
            ch.chamfer_estimate(At, Bt, metric, eps, T, seed, n_scales=L, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = ch.chamfer_estimate(At, Bt, metric, eps, T, seed, n_scales=L, precision=prec)
        torch.cuda.synchronize()
        et = (time.perf_counter() - t0) / args.steps
        chf = float(chv.item())
        eta = float(out["eta"].item())
        rm = rmin.cpu().numpy()
        rn = rnn.cpu().numpy()
        if prec == 0:
            ref = dict(ch=chf, eta=eta, rnn=rn, smin=out["sample_min"].cpu().numpy())
        rel = np.abs(rm[rows].astype(np.float64) - m64) / np.maximum(m64, 1e-30)
        res[name] = {
            "exact_ms": bt * 1e3, "estimate_ms": et * 1e3, "CH": chf, "eta": eta,
            "exact_points_per_s": 2 * n_a / bt, "estimate_points_per_s": 2 * n_a / et,
            "CH_rel_err_vs_fp32_canonical": abs(chf - ref["ch"]) / ref["ch"],
            "rows_exact_argmin_frac": float(np.mean(rn == ref["rnn"])),
            "sampled_rows_vs_fp64": {"max_rel_err": float(rel.max()),
                                      "mean_rel_err": float(rel.mean()),
                                      "argmin_match_frac": float(np.mean(rn[rows] == a64))},
            "eta_rel_err_vs_fp32_eta": abs(eta - ref["eta"]) / ref["eta"],
            "eta_rel_err_vs_CH": abs(eta - ref["ch"]) / ref["ch"],
            "sample_min_exact_frac": float(np.mean(out["sample_min"].cpu().numpy() == ref["smin"])),
        }
        print(f"[bench] {name}: exact {bt * 1e3:.1f} ms, estimate {et * 1e3:.2f} ms",
              file=sys.stderr, flush=True)
    for name in ("bf16", "fp8"):
        res[name]["exact_speedup_vs_fp32"] = res["fp32"]["exact_ms"] / res[name]["exact_ms"]
        res[name]["estimate_speedup_vs_fp32"] = res["fp32"]["estimate_ms"] / res[name]["estimate_ms"]
    return {"precision_report": res}


SERVE_POOL_SURFACES = 64
SERVE_POOL_CLUSTERS = 8
SERVE_N_MAX = 200_000


def serve_pool(torch, workloads):
    """Pinned host pool of cloud pairs at the largest request size; a request
    uses prefixes of one pair (its points are i.i.d., so a prefix is a sample
    of the same cloud)."""
    pool = {"surface": [], "clusters": []}
    for e in range(SERVE_POOL_SURFACES):
        rng = np.random.default_rng(1000 + e)
        a, b = workloads.surface_pair(rng, SERVE_N_MAX, SERVE_N_MAX)
        pool["surface"].append((torch.from_numpy(a).pin_memory(), torch.from_numpy(b).pin_memory()))
    for e in range(SERVE_POOL_CLUSTERS):
        rng = np.random.default_rng(2000 + e)
        centres = 4.0 * rng.standard_normal((64, 128))
        sig = rng.uniform(0.2, 1.0, size=64)
        a = workloads.mixture(rng, SERVE_N_MAX, centres, sig).astype(np.float32)
        b = workloads.mixture(rng, SERVE_N_MAX, centres, sig).astype(np.float32)
        pool["clusters"].append((torch.from_numpy(a).pin_memory(), torch.from_numpy(b).pin_memory()))
    return pool


def serve_run(srv, reqs, pool, precision, saturate=False):
    """Drive a server in real time: submit each request at its arrival
    time (or all at t = 0 when saturating), progress, drain results."""
    n = len(reqs)
    etas = np.zeros(n)
    lat = np.zeros(n)
    wait = np.zeros(n)
    id2i = {}
    done = 0
    st0 = srv.stats()
    t0 = time.monotonic()
    i = 0
    in_flight_sum = 0
    polls = 0
    arena_max = 0
    while done < n:
        now = time.monotonic() - t0
        while i < n and (saturate or reqs[i].arrival_s <= now):
            r = reqs[i]
            src = pool[r.kind][r.rid % len(pool[r.kind])]
            prec = precision if (r.metric == 2 and r.d >= 12) else 0
            rid = srv.submit(src[0][:r.n_a], src[1][:r.n_b], r.metric, r.eps, 0, r.seed,
                             precision=prec)
            id2i[rid] = i
            i += 1
        srv.progress()
        for res in srv.results():
            k = id2i.pop(res["id"])
            arrival = t0 + (0.0 if saturate else reqs[k].arrival_s)
            lat[k] = res["done_s"] - arrival
            wait[k] = res["admit_s"] - arrival
            etas[k] = res["eta"] if res["status"] == 0 else np.nan
            done += 1
        st = srv.stats()
        in_flight_sum += st["in_flight"]
        arena_max = max(arena_max, st["arena_used"])
        polls += 1
    wall = time.monotonic() - t0
    st = srv.stats()
    batches = st["batches"] - st0["batches"]
    return dict(completed=done, wall_s=wall, req_per_s=done / wall,
                p50_ms=float(np.percentile(lat, 50) * 1e3),
                p99_ms=float(np.percentile(lat, 99) * 1e3),
                max_ms=float(lat.max() * 1e3),
                admit_wait_p99_ms=float(np.percentile(wait, 99) * 1e3),
                mean_in_flight=in_flight_sum / max(polls, 1),
                batches=batches, mean_batch=(st["batched"] - st0["batched"]) / max(batches, 1),
                admission_stalls=st["stalls"] - st0["stalls"],
                arena_max_gib=arena_max / 2**30, failed=int(np.isnan(etas).sum())), etas


SERVE_CLASSES = ((3, 1), (3, 2), (128, 1), (128, 2))


def serve_bench(args, ch, torch, workloads):
    reqs = workloads.serving_stream(seed=args.seed, count=args.requests, rate_hz=args.rate)
    pool = serve_pool(torch, workloads)
    arena = int(args.arena_gib * 2**30)
    out = {"workload": (f"{args.requests} requests, Poisson {args.rate} req/s; 80% d=3 surface "
                        f"clouds, 20% d=128 clusters; sizes log-uniform [1k, 200k]; l2 70% / "
                        f"l1 30%; eps in {{0.1, 0.2}}; arena {args.arena_gib} GiB, "
                        f"{args.lanes} batch lanes"),
           "mix": {"d128": sum(r.d == 128 for r in reqs), "l2": sum(r.metric == 2 for r in reqs)}}
    etas = {}
    for name, prec in (("fp32", 0), ("bf16", 1)):
        with ch.ChamferServer(arena, args.lanes) as srv:
            # graphs of every request class on every lane, then a short burst
            # to warm the kernels and the host paths
            for d, metric in SERVE_CLASSES:
                srv.warm(d, metric, precision=prec if (metric == 2 and d >= 12) else 0)
            serve_run(srv, reqs[:256], pool, prec, saturate=True)
            res, etas[name] = serve_run(srv, reqs, pool, prec)
            sat, _ = serve_run(srv, reqs, pool, prec, saturate=True)
            res["graphs"] = srv.stats()["graphs"]
        res["saturated"] = {k: sat[k] for k in ("req_per_s", "p50_ms", "p99_ms", "wall_s",
                                                "batches", "mean_batch", "admission_stalls",
                                                "arena_max_gib")}
        out[name] = res
        print(f"[bench] serve {name}: p50 {res['p50_ms']:.2f} ms, p99 {res['p99_ms']:.2f} ms, "
              f"{res['req_per_s']:.0f} req/s, mean batch {res['mean_batch']:.2f}; saturated "
              f"{sat['req_per_s']:.0f} req/s, mean batch {sat['mean_batch']:.1f}",
              file=sys.stderr, flush=True)
    e32, e16 = etas["fp32"], etas["bf16"]
    rel = np.abs(e16 - e32) / np.maximum(np.abs(e32), 1e-300)
    d128 = np.array([r.d == 128 and r.metric == 2 for r in reqs])
    out["bf16_vs_fp32"] = {"p99_speedup": out["fp32"]["p99_ms"] / out["bf16"]["p99_ms"],
                           "saturated_throughput_ratio": out["bf16"]["saturated"]["req_per_s"]
                           / out["fp32"]["saturated"]["req_per_s"],
                           "eta_max_rel_diff": float(rel.max()),
                           "eta_max_rel_diff_d128_l2": float(rel[d128].max()) if d128.any() else 0.0,
                           "identical_eta_frac": float(np.mean(e16 == e32))}
    return {"serving": out}


# (k structures, window W) of the multi-probe CrudeNN report; (1, 1) is the
# base algorithm.
KW_CONFIGS = ((1, 1), (1, 4), (1, 16), (4, 1), (4, 4), (8, 8), (16, 4))
KW_SEEDS = 20
KW_T = (50, 200, 2000)


def kw_report(args, ch, torch, At, Bt, metric, eps, T, L, desc):
    """Multi-probe CrudeNN: for each (k, W), the estimate's time (CrudeNN
    stages and total), lambda_hat = D / CH, and the relative error of eta
    over KW_SEEDS hash/sampling seeds at several T (the sample-complexity
    comparison of the large-scale experiments).  CH is the GPU brute force
    (canonical float32 minima, float64 sum)."""
    ex, _, _ = ch.chamfer_exact(At, Bt, metric, rows_out=False)
    CH = float(ex.item())
    out = {"workload": desc, "CH": CH, "seeds": KW_SEEDS, "configs": []}
    ev = HipEvents(ch.STAGE_EVENTS)
    for k, W in KW_CONFIGS:
        def run(seed, t):
            return ch.chamfer_estimate(At, Bt, metric, eps, t, seed, n_scales=L, window=W, reps=k,
                                       stage_events=ev.arr)
        run(1, T)
        torch.cuda.synchronize()
        crude, total = [], []
        for _ in range(5):
            o = run(1, T)
            torch.cuda.synchronize()
            crude.append(ev.ms(0, 3))
            total.append(ev.ms(0, ch.STAGE_EVENTS - 1))
        lam = float(o["D"].item()) / CH
        errs = {}
        for t in KW_T:
            e = []
            for s in range(KW_SEEDS):
                o = run(100 + s, t)
                e.append(abs(float(o["eta"].item()) - CH) / CH)
            errs[str(t)] = {"mean_rel_err": float(np.mean(e)), "rms_rel_err":
                            float(np.sqrt(np.mean(np.square(e)))), "max_rel_err": float(np.max(e))}
        row = {"k": k, "W": W, "crude_ms": float(np.median(crude)),
               "estimate_ms": float(np.median(total)), "lambda_hat": lam, "rel_err": errs}
        out["configs"].append(row)
        print(f"[bench] k={k} W={W}: crude {row['crude_ms']:.3f} ms, estimate "
              f"{row['estimate_ms']:.3f} ms, lambda_hat {lam:.3f}, rms err T={T}: "
              f"{errs[str(KW_T[-1])]['rms_rel_err']:.4f}", file=sys.stderr, flush=True)
    ev.close()
    return {"kw_report": out}


SAMPLING_T = (10, 20, 50, 100, 200, 500, 1000, 2000)
SAMPLING_SEEDS = 20


def sampling_report(args, ch, torch, workloads):
    """Importance vs uniform sampling (the comparison of the experiments):
    RMS relative error of the estimate over SAMPLING_SEEDS seeds at each T,
    the smallest T reaching 2% and 1% RMS error, and the time of one
    estimate there.  Three synthetic stand-ins: the default l2 clusters
    (A -> B), a d = 3 surface pair in l1 with the symmetric CH(A,B) +
    CH(B,A) (the small-scale protocol), and the outlier scenario (Gaussian
    clouds in d = 100 plus one point at 0.5 n (1, ..., 1), l1)."""
    cases = []
    A, B = workloads.clusters_l2(seed=args.seed, n=100_000, d=128, k=1000)
    cases.append(("clusters l2 |A|=|B|=100000 d=128", A, B, 2, False))
    A, B = workloads.surface_pair(np.random.default_rng(args.seed), 20_000, 20_000)
    cases.append(("surface pair l1 |A|=|B|=20000 d=3, symmetric", A, B, 1, True))
    A, B = workloads.outlier_cloud(seed=args.seed, n=20_000, d=100)
    cases.append(("outlier l1 |A|=20001 |B|=20000 d=100", A, B, 1, False))
    out = {"seeds": SAMPLING_SEEDS, "T": list(SAMPLING_T), "cases": []}
    for name, A, B, metric, sym in cases:
        At = torch.from_numpy(np.ascontiguousarray(A, np.float32)).cuda()
        Bt = torch.from_numpy(np.ascontiguousarray(B, np.float32)).cuda()
        if sym:
            CH = float(ch.chamfer_exact_symmetric(At, Bt, metric)[0].item())
        else:
            CH = float(ch.chamfer_exact(At, Bt, metric, rows_out=False)[0].item())

        def est(sampling, T, seed, reps):
            if sym:
                return ch.chamfer_estimate_symmetric(At, Bt, metric, 0.1, T, seed,
                                                     sampling=sampling, reps=reps)[0]
            return ch.chamfer_estimate(At, Bt, metric, 0.1, T, seed, sampling=sampling,
                                       reps=reps, with_aux=False)["eta"]

        row = {"case": name, "CH": CH}
        for sname, sampling, reps in (("importance", 0, 1), ("importance_4x1", 0, 4),
                                      ("uniform", 1, 1)):
            curve, times = [], []
            for T in SAMPLING_T:
                errs = [abs(float(est(sampling, T, 100 + s, reps).item()) - CH) / CH
                        for s in range(SAMPLING_SEEDS)]
                curve.append(float(np.sqrt(np.mean(np.square(errs)))))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for s in range(5):
                    est(sampling, T, s, reps)
                torch.cuda.synchronize()
                times.append((time.perf_counter() - t0) / 5 * 1e3)
            need = {}
            for tgt in (0.02, 0.01):
                ok = [i for i, e in enumerate(curve) if e <= tgt]
                need[f"{tgt:g}"] = ({"T": SAMPLING_T[ok[0]], "ms": times[ok[0]]} if ok
                                    else None)
            row[sname] = {"rms_rel_err": curve, "ms": times, "to_reach": need}
        out["cases"].append(row)
        print(f"[bench] {name}: to reach 2% / 1% rms: "
              + "; ".join(f"{k} {row[k]['to_reach']}" for k in ("importance", "importance_4x1",
                                                               "uniform")),
              file=sys.stderr, flush=True)
        del At, Bt
    return {"sampling_report": out}


def reduction_report(args, ch, torch, workloads):
    """The reduction to bounded aspect ratio: its bounds against the exact
    CH, the number of parts, the time of the reduction itself (sketch,
    sort, 1-D search, partition keys; padded copies) and of the estimate
    plain / after the partition / on the padded sets, with the error of each
    estimate over REDUCTION_SEEDS seeds."""
    cases = [("clusters l2 |A|=|B|=100000 d=128", "clusters_l2", dict(n=100_000, d=128, k=1000),
              2, 0.2),
             ("mixed l1 |A|=|B|=1000000 d=64", "mixed_l1", dict(), 1, 0.2),
             ("surface pair l1 |A|=|B|=200000 d=3", None, None, 1, 0.2)]
    out = []
    for name, gen, kw, metric, eps in cases:
        if gen is None:
            A, B = workloads.surface_pair(np.random.default_rng(args.seed), 200_000, 200_000)
        else:
            A, B = getattr(workloads, gen)(seed=args.seed, **kw)
        At, Bt = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        exact = float(ch.chamfer_exact(At, Bt, metric, rows_out=False)[0].item())

        def timed(fn, reps=5):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / reps * 1e3

        red = ch.chamfer_aspect_reduce(At, Bt, metric, eps, 1)
        info = red["info"]
        ka = red["keys_A"].cpu().numpy()
        kb = red["keys_B"].cpu().numpy()
        parts = len(np.unique(np.concatenate([ka, kb])))
        row = {"case": name, "CH": exact, "eta_lo": info["eta_lo"], "eta_hi": info["eta_hi"],
               "ch1": info["ch1"], "e_part": info["e_part"], "pad_dims": info["pad_dims"],
               "pad_value": info["pad_value"], "parts": parts,
               "ms_reduce": timed(lambda: ch.chamfer_aspect_reduce(At, Bt, metric, eps, 1)),
               "ms_reduce_pad": timed(lambda: ch.chamfer_aspect_reduce(At, Bt, metric, eps, 1,
                                                                      pad=True))}
        for label, red_mode in (("plain", 0), ("partition", 1), ("pad", 2)):
            row[f"ms_{label}"] = timed(lambda: ch.chamfer_estimate(
                At, Bt, metric, eps, 0, 1, reduction=red_mode, with_aux=False))
            errs = [abs(float(ch.chamfer_estimate(At, Bt, metric, eps, 0, 100 + s,
                                                  reduction=red_mode, with_aux=False)
                              ["eta"].item()) - exact) / exact
                    for s in range(REDUCTION_SEEDS)]
            row[f"rms_err_{label}"] = float(np.sqrt(np.mean(np.square(errs))))
        out.append(row)
        print(f"[bench] {name}: parts {parts}, reduce {row['ms_reduce']:.3f} ms, estimate "
              f"plain/partition/pad {row['ms_plain']:.3f}/{row['ms_partition']:.3f}/"
              f"{row['ms_pad']:.3f} ms, rms err {row['rms_err_plain']:.4f}/"
              f"{row['rms_err_partition']:.4f}/{row['rms_err_pad']:.4f}",
              file=sys.stderr, flush=True)
        del At, Bt
    return {"reduction_report": {"seeds": REDUCTION_SEEDS, "cases": out}}


REDUCTION_SEEDS = 10
RETRIEVAL_K = (1, 5, 10, 30)
RETRIEVAL_SETS = (("distinct surfaces", 1, 0.0), ("families of 10, 2% jitter", 10, 0.02))


def retrieval_report(args, ch, torch, workloads):
    """One-vs-many retrieval (the downstream experiment): collections of
    1000 d = 3 surface clouds of 1000..4000 points and 20 queries, each a
    resample of a member; l1, three scales, T = 50.  Two collections: every
    member its own random surface, and families of 10 members sharing a base
    surface with 2% parameter jitter (near neighbours).  For each k: recall@k
    (the true nearest cloud under exact symmetric CH among the k smallest
    estimates, i.e. top-1 accuracy after the exact re-rank) and the time of
    one retrieval, against brute force (exact symmetric CH to every cloud,
    one library call per cloud)."""
    m, queries, metric, eps, T, L = 1000, 20, 1, 0.2, 50, 3
    out = {"m": m, "n": [1000, 4000], "d": 3, "queries": queries, "metric": "l1", "eps": eps,
           "T": T, "L": L, "sets": []}
    for name, family, jitter in RETRIEVAL_SETS:
        clouds, qs, src = workloads.retrieval_collection(seed=args.seed, m=m, n_min=1000,
                                                         n_max=4000, queries=queries,
                                                         family=family, jitter=jitter)
        sizes = [c.shape[0] for c in clouds]
        Bs = torch.from_numpy(np.ascontiguousarray(np.concatenate(clouds), np.float32)).cuda()
        offs = np.concatenate([[0], np.cumsum(sizes)])
        views = [Bs[offs[i]:offs[i + 1]] for i in range(m)]
        Qs = [torch.from_numpy(np.ascontiguousarray(q, np.float32)).cuda() for q in qs]
        torch.cuda.synchronize()
        print(f"[bench] retrieval ({name}): {m} clouds, {int(offs[-1])} points, {queries} "
              "queries", file=sys.stderr, flush=True)

        truth, brute_ms = [], []
        for q in Qs:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            vals = [ch.chamfer_exact_symmetric(q, v, metric) for v in views]
            exact = torch.stack([v[0] for v in vals]).cpu().numpy()
            brute_ms.append((time.perf_counter() - t0) * 1e3)
            truth.append(int(np.argmin(exact)))
        print(f"[bench] retrieval: brute force {np.median(brute_ms):.1f} ms/query",
              file=sys.stderr, flush=True)

        ch.chamfer_retrieve_packed(Qs[0], Bs, sizes, metric, eps, T, 1, 1, n_scales=L)  # warm
        rows = []
        for k in RETRIEVAL_K:
            hits = 0
            times = []
            for qi, q in enumerate(Qs):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, top, _ = ch.chamfer_retrieve_packed(q, Bs, sizes, metric, eps, T, 1 + qi, k,
                                                       n_scales=L)
                times.append((time.perf_counter() - t0) * 1e3)
                hits += top[0] == truth[qi]
            rows.append({"k": k, "recall_at_k": hits / queries,
                         "ms_per_query": float(np.median(times))})
            print(f"[bench] retrieval k={k}: recall {hits}/{queries}, "
                  f"{rows[-1]['ms_per_query']:.2f} ms/query", file=sys.stderr, flush=True)
        out["sets"].append({"collection": name, "points": int(offs[-1]),
                            "brute_ms_per_query": float(np.median(brute_ms)),
                            "nearest_is_source": float(np.mean([t == int(s) for t, s in
                                                                zip(truth, src)])),
                            "rows": rows})
        del Bs, views, Qs
    return {"retrieval_report": out}


TARGET_WORKLOAD = "l2_1m_d128"


def target_point(args, ch, torch, workloads):
    """The speed-up target at 10^6 points: l2, |A| = |B| = 10^6, d = 128,
    1000-cluster mixture, eps = 0.1, T = 2000, L = 24.  Estimate ms per step
    (same timing as the headline), GPU brute force, their ratio, the
    estimate's relative error against the brute force, the stage split and
    the roofline of the exact pass over the draws."""
    gen, kw, metric, eps, T, L, desc = WORKLOADS[TARGET_WORKLOAD]
    A, B = getattr(workloads, gen)(seed=args.seed, **kw)
    n_a, d = A.shape
    n_b = B.shape[0]
    At = torch.from_numpy(A).cuda()
    Bt = torch.from_numpy(B).cuda()
    del A, B
    torch.cuda.synchronize()
    seed = 1
    steps = max(5, args.steps // 2)

    def step():
        return ch.chamfer_estimate(At, Bt, metric, eps, T, seed, n_scales=L, with_aux=False)

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    eta = float(out["eta"].item())
    ncalls = 10
    ev = HipEvents(ch.STAGE_EVENTS * ncalls)
    for s in range(ncalls):
        sub = ctypes.c_void_p(ctypes.addressof(ev.arr)
                              + s * ch.STAGE_EVENTS * ctypes.sizeof(ctypes.c_void_p))
        ch.chamfer_estimate(At, Bt, metric, eps, T, seed, n_scales=L, with_aux=False,
                            stage_events=sub)
    torch.cuda.synchronize()
    names = ["calibrate+tables", "bucket_B", "probe_A+D_a", "weights+draws", "exact_pass",
             "final"]
    stages = {n: float(np.mean([ev.ms(s * ch.STAGE_EVENTS + i, s * ch.STAGE_EVENTS + i + 1)
                                for s in range(ncalls)])) for i, n in enumerate(names)}
    ev.close()
    work = algorithmic_sample_pass(metric, T, n_b, d)
    kms = stages["exact_pass"]
    achieved = work["ops"] / (kms * 1e-3) / 1e12
    print(f"[bench] target {TARGET_WORKLOAD}: {dt * 1e3:.3f} ms/step", file=sys.stderr,
          flush=True)
    ch.chamfer_exact(At, Bt, metric, rows_out=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ex, _, _ = ch.chamfer_exact(At, Bt, metric, rows_out=False)
    torch.cuda.synchronize()
    bt = time.perf_counter() - t0
    exact = float(ex.item())
    print(f"[bench] target brute force {bt * 1e3:.1f} ms", file=sys.stderr, flush=True)
    del At, Bt
    torch.cuda.empty_cache()
    return {"workload": desc, "name": TARGET_WORKLOAD, "steps": steps,
            "estimate_ms": dt * 1e3, "points_per_s": (n_a + n_b) / dt,
            "brute_force_ms": bt * 1e3, "speedup": bt / dt,
            "rel_err": abs(eta - exact) / exact, "eta": eta, "CH": exact,
            "stages_ms": stages,
            "roofline": {"kernel": "exact pass over the T draws (the draws' split table, "
                                   "matrix-core record kernel, resolve, rescans)",
                         "bound": work["bound"], "achieved": achieved, "peak": work["peak"],
                         "unit": work["unit"], "frac": achieved / work["peak"],
                         "kernel_ms": kms}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="l2_100k_d128", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=42)
    ap.add_argument("--brute-steps", type=int, default=2)
    ap.add_argument("--no-brute", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-target", action="store_true",
                    help="skip the 10^6-point target measurement of the default run")
    ap.add_argument("--precision-report", action="store_true",
                    help="time exact CH and the estimator in FP32, BF16 and FP8 and report "
                         "their errors (l2 workloads)")
    ap.add_argument("--kw-report", action="store_true",
                    help="multi-probe CrudeNN: time, lambda_hat and the error of eta over "
                         "seeds for several (k structures, window W)")
    ap.add_argument("--sampling-report", action="store_true",
                    help="importance vs uniform sampling: error vs T over seeds and the time "
                         "to reach 2%% / 1%% on three synthetic cases")
    ap.add_argument("--reduction-report", action="store_true",
                    help="reduction to bounded aspect ratio: bounds, parts, time of the "
                         "reduction and of the estimate with it, errors over seeds")
    ap.add_argument("--retrieval-report", action="store_true",
                    help="one-vs-many retrieval over 1000 clouds: recall@k and time vs "
                         "brute force")
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark: Poisson stream of mixed requests through the "
                         "continuous-batching server, FP32 and BF16-refined")
    ap.add_argument("--requests", type=int, default=20000)
    ap.add_argument("--rate", type=float, default=500.0)
    ap.add_argument("--arena-gib", type=float, default=8.0)
    ap.add_argument("--lanes", type=int, default=4)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run --steps plain device-to-device copies of MIB MiB "
                         "(calibrates the FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: one GPU only; --gpus {args.gpus} is not supported (the path would "
              "shard A by rows with B replicated, and one GPU runs one shard's kernels).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe:
        # a plain device copy: calibrates the traffic counters, and its rate
        # (bytes read + written per second) is the HBM bandwidth this box
        # reaches with a library kernel
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / max(args.steps, 1)
        print(json.dumps({"copy_probe_bytes": n * 4, "copies": args.steps, "ms_per_copy": ms,
                          "hbm_tb_per_s": 2 * n * 4 / (ms * 1e-3) / 1e12}))
        return

    import paper_2307_03043_amd as ch
    import workloads

    if args.serve:
        print(json.dumps(serve_bench(args, ch, torch, workloads)))
        return
    if args.sampling_report:
        print(json.dumps(sampling_report(args, ch, torch, workloads)))
        return
    if args.reduction_report:
        print(json.dumps(reduction_report(args, ch, torch, workloads)))
        return
    if args.retrieval_report:
        print(json.dumps(retrieval_report(args, ch, torch, workloads)))
        return

    gen, kw, metric, eps, T, L, desc = WORKLOADS[args.workload]
    A, B = getattr(workloads, gen)(seed=args.seed, **kw)
    n_a, d = A.shape
    n_b = B.shape[0]
    dev = torch.device("cuda:0")
    At = torch.from_numpy(A).to(dev)
    Bt = torch.from_numpy(B).to(dev)
    torch.cuda.synchronize()
    seed = 1

    if args.precision_report:
        print(json.dumps(precision_report(args, ch, torch, A, B, At, Bt, metric, eps, T, L,
                                          desc)))
        return
    if args.kw_report:
        print(json.dumps(kw_report(args, ch, torch, At, Bt, metric, eps, T, L, desc)))
        return

    def step():
        return ch.chamfer_estimate(At, Bt, metric, eps, T, seed, n_scales=L, with_aux=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"[bench] {args.workload}: warmup done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    eta = float(out["eta"].item())
    print(f"[bench] timed {args.steps} steps: {dt * 1e3:.3f} ms/step", file=sys.stderr, flush=True)

    # per-stage times and per-step latency from the library's stage events
    # per-stage times and per-call latency over at least LATENCY_CALLS calls
    ncalls = max(args.steps, LATENCY_CALLS)
    ev = HipEvents(ch.STAGE_EVENTS * ncalls)
    for s in range(ncalls):
        sub = ctypes.c_void_p(ctypes.addressof(ev.arr)
                              + s * ch.STAGE_EVENTS * ctypes.sizeof(ctypes.c_void_p))
        last = ch.chamfer_estimate(At, Bt, metric, eps, T, seed, n_scales=L, with_aux=True,
                                   stage_events=sub)
    torch.cuda.synchronize()
    names = ["calibrate+tables", "bucket_B", "probe_A+D_a", "weights+draws", "exact_pass",
             "final"]
    stage = np.zeros((ncalls, len(names)))
    lat = np.zeros(ncalls)
    for s in range(ncalls):
        base = s * ch.STAGE_EVENTS
        for i in range(len(names)):
            stage[s, i] = ev.ms(base + i, base + i + 1)
        lat[s] = ev.ms(base, base + ch.STAGE_EVENTS - 1)
    ev.close()
    aux = last
    stages_ms = {n: float(stage[:, i].mean()) for i, n in enumerate(names)}
    dom = int(np.argmax(stage.mean(axis=0)))
    lam = float(aux["D"].item())

    # roofline of the exact pass over the draws (stage 4 -> 5: for l2 the
    # draws' split table, the record pass on the matrix cores and the
    # per-draw resolve kernel; B's split table is written by the kernel that
    # hashes B, in the bucket_B stage)
    work = algorithmic_sample_pass(metric, T, n_b, d)
    kernel_ms = stages_ms["exact_pass"]
    achieved = work["ops"] / (kernel_ms * 1e-3) / 1e12
    roofline = {"kernel": "k_nnmin (exact pass over the T draws)", "bound": work["bound"],
                "achieved": achieved, "peak": work["peak"], "unit": work["unit"],
                "frac": achieved / work["peak"],
                "traffic": measured_traffic(args.workload, kernel_ms), "kernel_ms": kernel_ms,
                "algorithmic": work["note"]}
    if "products" in work:
        roofline["kernel"] = ("k_split_rows of the draws + k_nnmin_l2_split record pass + "
                              "k_split_resolve (exact pass over the T draws; B's split table "
                              "is written while B is hashed, in bucket_B)")
        roofline["mfma_dtype"] = "bf16"
        roofline["frac_of_split_ceiling"] = achieved * work["products"] / work["peak"]

    result = {
        "metric": METRIC_NAME,
        "value": (n_a + n_b) / dt,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "name": args.workload, "n_a": n_a, "n_b": n_b, "d": d,
                   "metric": "l2" if metric == 2 else "l1", "eps": eps, "T": T, "L": L,
                   "seed": args.seed},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "calls": int(ncalls)},
        "stages_ms": stages_ms,
        "dominant_stage": names[dom],
        "roofline": roofline,
        "eta": eta,
        "D_normaliser": lam,
    }

    if not args.no_brute:
        ch.chamfer_exact(At, Bt, metric, rows_out=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.brute_steps):
            ex, _, _ = ch.chamfer_exact(At, Bt, metric, rows_out=False)
        torch.cuda.synchronize()
        bt = (time.perf_counter() - t0) / args.brute_steps
        exact = float(ex.item())
        result["brute_force"] = {"ms": bt * 1e3, "points_per_s": (n_a + n_b) / bt,
                                 "speedup_of_estimate": bt / dt, "CH": exact,
                                 "dtype": "f32", "kernel": "k_nnmin over all rows of A"}
        result["accuracy"] = {"rel_err": abs(eta - exact) / exact, "lambda_hat": lam / exact}
        print(f"[bench] brute force {bt * 1e3:.1f} ms", file=sys.stderr, flush=True)

    if args.workload == "l2_100k_d128" and not args.no_target:
        result["target_point"] = target_point(args, ch, torch, workloads)

    if not args.no_cpu:
        base, ref = cpu_baseline(args, A, B, metric, eps, T, L, seed)
        result["cpu_baseline"] = base
        if ref is not None:
            result["accuracy"] = dict(result.get("accuracy", {}), oracle_eta=ref["eta"],
                                      gpu_vs_oracle_rel=abs(eta - ref["eta"]) / ref["eta"])
        print(f"[bench] cpu oracle {base['seconds']:.2f} s", file=sys.stderr, flush=True)

    print(json.dumps(result))


if __name__ == "__main__":
    main()
