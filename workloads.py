"""Seeded synthetic point clouds for the Chamfer-distance workloads.

This module only draws input point sets.  It holds none of the estimator's
arithmetic (no hashing, no sampling, no distances), so both the CPU oracle and
the GPU library can be fed from it without sharing any of the method.

Every generator takes an explicit seed and uses numpy's PCG64
(`numpy.random.default_rng`).  The draw order inside each generator is fixed:
centres, then cluster assignments, then noise, then the second set.  Arrays
are float32, row-major ``[n, d]`` and C-contiguous.

The shapes and value distributions stand in for the regimes the paper
evaluates on (Table 1 of the experiments section): small low-dimensional
clouds, high-dimensional embedding clouds, an outlier cloud, and large
high-dimensional clouds.  None of the paper's datasets is reproduced.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

L1 = 1
L2 = 2


def _f32(x: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float32)


def mixture(rng: np.random.Generator, n: int, centres: np.ndarray,
            sigma: np.ndarray | float, noise: str = "normal") -> np.ndarray:
    """n points: a uniformly chosen centre plus i.i.d. per-coordinate noise."""
    k, d = centres.shape
    assign = rng.integers(0, k, size=n)
    sig = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (k,))[assign][:, None]
    if noise == "normal":
        eps = rng.standard_normal((n, d))
    elif noise == "laplace":
        eps = rng.laplace(0.0, 1.0, size=(n, d))
    else:
        raise ValueError(noise)
    return centres[assign] + sig * eps


def small_l2(seed: int = 42, n: int = 4096, d: int = 16):
    """Small plain-method case: 16 centres ~U[-10,10]^d, sigma=1.

    B comes from the same mixture with every centre moved by N(0, 0.5^2).
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-10.0, 10.0, size=(16, d))
    a = mixture(rng, n, centres, 1.0)
    centres_b = centres + 0.5 * rng.standard_normal(centres.shape)
    b = mixture(rng, n, centres_b, 1.0)
    return _f32(a), _f32(b)


def clusters_l2(seed: int = 42, n: int = 100_000, d: int = 128,
                k: int = 1000, n_b: int | None = None):
    """High-dimensional cluster clouds: centres ~N(0, 4^2 I), sigma_j ~U[0.2, 1].

    A and B are independent draws from the same mixture.
    """
    rng = np.random.default_rng(seed)
    centres = 4.0 * rng.standard_normal((k, d))
    sig = rng.uniform(0.2, 1.0, size=k)
    a = mixture(rng, n, centres, sig)
    b = mixture(rng, n if n_b is None else n_b, centres, sig)
    return _f32(a), _f32(b)


def mixed_l1(seed: int = 42, n: int = 1_000_000, d: int = 64, k: int = 5000,
             n_b: int | None = None):
    """l1 workload: 70% from a k-cluster mixture with Laplace(0, 0.5) noise,
    30% uniform in [-50, 50]^d.  Centres ~U[-50, 50]^d."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-50.0, 50.0, size=(k, d))

    def draw(m):
        n_cl = int(round(0.7 * m))
        pts = np.empty((m, d))
        pts[:n_cl] = mixture(rng, n_cl, centres, 0.5, noise="laplace")
        pts[n_cl:] = rng.uniform(-50.0, 50.0, size=(m - n_cl, d))
        return pts[rng.permutation(m)]

    a = draw(n)
    b = draw(n if n_b is None else n_b)
    return _f32(a), _f32(b)


def precision_l2(seed: int = 42, n: int = 1_000_000, d: int = 256,
                 k: int = 10_000, n_b: int | None = None):
    """Precision workload: 10,000 centres ~N(0, I), sigma = 0.3."""
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((k, d))
    a = mixture(rng, n, centres, 0.3)
    b = mixture(rng, n if n_b is None else n_b, centres, 0.3)
    return _f32(a), _f32(b)


def outlier_cloud(seed: int = 42, n: int = 50_000, d: int = 100):
    """Outlier scenario of the experiments section: A and B standard Gaussian
    clouds, plus one extra point of A at 0.5*n*(1,...,1)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, d))
    b = rng.standard_normal((n, d))
    a = np.vstack([a, np.full((1, d), 0.5 * n)])
    return _f32(a), _f32(b)


def uniform_cube(seed: int, n_a: int, n_b: int, d: int, lo=-1.0, hi=1.0):
    rng = np.random.default_rng(seed)
    return (_f32(rng.uniform(lo, hi, size=(n_a, d))),
            _f32(rng.uniform(lo, hi, size=(n_b, d))))


# --------------------------------------------------------------------------
# Serving stream: d=3 surface clouds (ellipsoids, tori) and d=128 clusters.
# --------------------------------------------------------------------------

def _rotation(rng: np.random.Generator) -> np.ndarray:
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    return q * np.sign(np.diag(r))


def surface_pair(rng: np.random.Generator, n_a: int, n_b: int):
    """Two independent samples of one random surface in R^3 with N(0, 0.01^2)
    noise.  Ellipsoid (semi-axes ~U[0.5, 2]) or torus (R~U[1,2], r~U[0.2,0.5]),
    randomly rotated; points use uniform angles (not area-uniform)."""
    kind = rng.integers(0, 2)
    rot = _rotation(rng)
    if kind == 0:
        axes = rng.uniform(0.5, 2.0, size=3)

        def draw(m):
            th = rng.uniform(0.0, math.pi, size=m)
            ph = rng.uniform(0.0, 2 * math.pi, size=m)
            p = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph),
                          np.cos(th)], axis=1) * axes
            return p
    else:
        big, small = rng.uniform(1.0, 2.0), rng.uniform(0.2, 0.5)

        def draw(m):
            u = rng.uniform(0.0, 2 * math.pi, size=m)
            v = rng.uniform(0.0, 2 * math.pi, size=m)
            p = np.stack([(big + small * np.cos(v)) * np.cos(u),
                          (big + small * np.cos(v)) * np.sin(u),
                          small * np.sin(v)], axis=1)
            return p
    a = draw(n_a) @ rot.T + 0.01 * rng.standard_normal((n_a, 3))
    b = draw(n_b) @ rot.T + 0.01 * rng.standard_normal((n_b, 3))
    return _f32(a), _f32(b)


def _jittered_pair(rng: np.random.Generator, base, jitter: float, n: int):
    """Two samples of size n of the base surface (kind, parameters, rotation)
    with every shape parameter scaled by an independent 1 + jitter N(0, 1)."""
    kind, params, rot = base
    p = params * (1.0 + jitter * rng.standard_normal(params.shape))

    def draw(m):
        if kind == 0:
            th = rng.uniform(0.0, math.pi, size=m)
            ph = rng.uniform(0.0, 2 * math.pi, size=m)
            return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph),
                             np.cos(th)], axis=1) * p
        u = rng.uniform(0.0, 2 * math.pi, size=m)
        v = rng.uniform(0.0, 2 * math.pi, size=m)
        return np.stack([(p[0] + p[1] * np.cos(v)) * np.cos(u),
                         (p[0] + p[1] * np.cos(v)) * np.sin(u), p[1] * np.sin(v)], axis=1)

    a = draw(n) @ rot.T + 0.01 * rng.standard_normal((n, 3))
    b = draw(n) @ rot.T + 0.01 * rng.standard_normal((n, 3))
    return _f32(a), _f32(b)


def retrieval_collection(seed: int = 42, m: int = 1000, n_min: int = 1000, n_max: int = 4000,
                         queries: int = 20, family: int = 1, jitter: float = 0.0):
    """A collection of m d=3 surface clouds (sizes uniform in [n_min, n_max])
    and `queries` query clouds, each an independent resample (same surface,
    same size) of a distinct member; returns (clouds, queries, source ids).
    family = 1: every member is its own random surface (as surface_pair).
    family > 1: members come in consecutive groups of `family` sharing one
    base surface (ellipsoid or torus, rotation) whose parameters each member
    scales by 1 + jitter N(0, 1): near neighbours that the estimate has to
    tell apart."""
    rng = np.random.default_rng(seed)
    src = rng.choice(m, size=queries, replace=False)
    slot = {int(s): q for q, s in enumerate(src)}
    clouds, qs = [], [None] * queries
    base = None
    for i in range(m):
        n = int(rng.integers(n_min, n_max + 1))
        if family <= 1:
            a, b = surface_pair(rng, n, n)
        else:
            if i % family == 0:
                kind = int(rng.integers(0, 2))
                params = (rng.uniform(0.5, 2.0, size=3) if kind == 0 else
                          np.array([rng.uniform(1.0, 2.0), rng.uniform(0.2, 0.5)]))
                base = (kind, params, _rotation(rng))
            a, b = _jittered_pair(rng, base, jitter, n)
        clouds.append(a)
        if i in slot:
            qs[slot[i]] = b
    return clouds, qs, src.astype(np.int64)


@dataclass
class Request:
    rid: int
    arrival_s: float
    kind: str          # "surface" (d=3) or "clusters" (d=128)
    n_a: int
    n_b: int
    d: int
    metric: int
    eps: float
    seed: int


def serving_stream(seed: int = 42, count: int = 20_000, rate_hz: float = 500.0,
                   n_min: int = 1000, n_max: int = 200_000):
    """Request descriptors: Poisson arrivals, sizes log-uniform in
    [n_min, n_max], 80% d=3 surfaces / 20% d=128 clusters, l2 70% / l1 30%,
    eps in {0.1, 0.2}.  Clouds are drawn lazily by `request_clouds`."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    lo, hi = math.log(n_min), math.log(n_max)
    for rid in range(count):
        t += rng.exponential(1.0 / rate_hz)
        kind = "surface" if rng.uniform() < 0.8 else "clusters"
        n_a = int(round(math.exp(rng.uniform(lo, hi))))
        n_b = int(round(math.exp(rng.uniform(lo, hi))))
        metric = L2 if rng.uniform() < 0.7 else L1
        eps = 0.1 if rng.uniform() < 0.5 else 0.2
        out.append(Request(rid, t, kind, n_a, n_b, 3 if kind == "surface" else 128,
                           metric, eps, seed + rid))
    return out


def request_clouds(req: Request):
    rng = np.random.default_rng(req.seed)
    if req.kind == "surface":
        return surface_pair(rng, req.n_a, req.n_b)
    centres = 4.0 * rng.standard_normal((64, req.d))
    sig = rng.uniform(0.2, 1.0, size=64)
    return _f32(mixture(rng, req.n_a, centres, sig)), _f32(mixture(rng, req.n_b, centres, sig))
