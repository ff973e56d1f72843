"""Write tests/golden/exact_ch.json: the float64 exact Chamfer distance of the
benchmark workloads, computed by the CPU oracle only (definition of CH in
the introduction; the oracle's brute force in double precision, summed
exactly).  The coverage test of the estimator compares GPU estimates over
many seeds with these values.

Run: python tests/golden/make_exact_ch.py  (about a minute per 10^5-point
workload on 8 cores)."""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

WORKLOADS = {
    # name: generator, kwargs, metric (seed 42)
    "l2_100k_d128": ("clusters_l2", dict(n=100_000, d=128, k=1000), 2),
    "l2_4k_d16": ("small_l2", dict(n=4096, d=16), 2),
}


def main():
    out = {"cite": "CH(A, B) = sum_a min_b d(a, b), not squared (definition of CH in the "
                   "introduction and its footnote); float64 brute force of the CPU oracle, "
                   "exactly rounded sum; inputs from workloads.py with seed 42."}
    for name, (gen, kw, metric) in WORKLOADS.items():
        A, B = getattr(workloads, gen)(seed=42, **kw)
        t = time.time()
        ch, _, _ = oracle.chamfer_exact(A, B, metric)
        out[name] = {"generator": gen, "kwargs": kw, "seed": 42, "metric": metric,
                     "ch": ch, "seconds": round(time.time() - t, 1)}
        print(name, ch, f"{time.time() - t:.1f} s", flush=True)
    with open(os.path.join(HERE, "exact_ch.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
