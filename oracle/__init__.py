"""CPU oracle for the near-linear Chamfer estimator.

TEST INFRASTRUCTURE ONLY: only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path
(the GPU library and its binding) never imports, links or calls it, and the
two share no code.

The arithmetic lives in ``chamfer_oracle.c`` (plain C, one IEEE operation per
written operation); this module builds it with gcc, loads it with ctypes and
composes the steps in the order of the paper's two algorithm figures:

* ``chamfer_exact``    -- CH(A,B) = sum_a min_b d(a,b) (introduction), in
  double precision, summed exactly with ``math.fsum``;
* ``crude_nn``         -- the CrudeNN figure (multi-scale grid hashing, first
  colliding scale, D_a = d(a, b) for the lowest-index colliding b);
* ``chamfer_estimate`` -- the Chamfer-Estimate figure (D = sum D_a, T i.i.d.
  draws x ~ D_a / D, eta = mean of (D / D_x) min_b d(x, b)), with the
  distribution held in 64-bit fixed point.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

L1 = 1
L2 = 2
DEFAULT_EMBED_DIM = 32

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chamfer_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

_F32 = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_F64 = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_U64 = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_I32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_VP = ctypes.c_void_p
_I64 = ctypes.c_int64
_INT = ctypes.c_int


def _host_has_fma() -> bool:
    try:
        with open("/proc/cpuinfo") as f:
            return " fma " in f.read()
    except OSError:
        return False


def build() -> str:
    """Compile the oracle with gcc (always recompiles).  With FMA3 on the
    host, fmaf becomes the hardware instruction (correctly rounded, the same
    result as the library call); -ffp-contract=off still forbids any fusion
    that the source does not spell out."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-o", _SO + ".tmp", _SRC, "-lm"]
    if _host_has_fma():
        cmd.insert(1, "-mfma")
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    L = ctypes.CDLL(_SO)
    L.or_threads.restype = _INT
    L.or_philox4x64.argtypes = [_U64, _U64, _U64]
    L.or_grid_tables.argtypes = [ctypes.c_uint64, _INT, _INT, _F32, _U64]
    L.or_grid_tables_rep.argtypes = [ctypes.c_uint64, ctypes.c_uint64, _INT, _INT, _F32, _U64]
    L.or_embedding.argtypes = [ctypes.c_uint64, _INT, _INT, _F32]
    L.or_default_scales.argtypes = [_I64, _I64, ctypes.c_double]
    L.or_default_scales.restype = _INT
    L.or_default_samples.argtypes = [_I64, ctypes.c_double]
    L.or_default_samples.restype = _I64
    L.or_calibrate.argtypes = [_F32, _I64, _F32, _I64, _INT, _F32, _F32,
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_INT)]
    L.or_hash_keys.argtypes = [_F32, _I64, _INT, _INT, _F32, _VP, _INT, _INT, _INT,
                               _F32, _U64, _U64]
    L.or_crude_nn.argtypes = [_U64, _I64, _U64, _I64, _INT, _F32, _F32, _INT, _INT,
                              _I32, _I32, _F32]
    L.or_crude_window.argtypes = [_U64, _I64, _U64, _I64, _INT, _INT, _F32, _F32, _INT, _INT,
                                  _I32, _I32, _F32]
    L.or_dist32.argtypes = [_F32, _F32, _INT, _INT]
    L.or_dist32.restype = ctypes.c_float
    L.or_nn_f64.argtypes = [_F32, _I64, _VP, _F32, _I64, _INT, _INT, _F64, _I32]
    L.or_nn_f32.argtypes = [_F32, _I64, _VP, _F32, _I64, _INT, _INT, _F32, _I32]
    L.or_weights.argtypes = [_F32, _I64, ctypes.POINTER(_INT), _U64, _U64,
                             ctypes.POINTER(ctypes.c_uint64)]
    L.or_weights.restype = _INT
    L.or_sample.argtypes = [ctypes.c_uint64, _U64, _I64, ctypes.c_uint64, _I64, _I32]
    _lib = L
    return L


def threads() -> int:
    """OpenMP threads of the parallel loops (exact nearest neighbours)."""
    return int(lib().or_threads())


def _f32(x):
    return np.ascontiguousarray(x, dtype=np.float32)


# --------------------------------------------------------------------------
# Random streams (Philox4x64-10) and the tables drawn from them.
# --------------------------------------------------------------------------

def philox4x64(counter, key) -> np.ndarray:
    """One Philox4x64-10 block (Salmon et al., SC 2011)."""
    out = np.zeros(4, np.uint64)
    lib().or_philox4x64(np.asarray(counter, np.uint64), np.asarray(key, np.uint64), out)
    return out


def grid_tables(seed: int, L: int, kh: int, rep: int = 0):
    """Shifts z'[L, kh] in cell units (U[0,1) on a 2^-24 lattice) and odd
    64-bit key multipliers M[L, kh], one independent pair per scale
    (appendix lemma on the grid hash at every scale); rep numbers the
    independent LSH structures of the repeated variant."""
    z = np.zeros((L, kh), np.float32)
    m = np.zeros((L, kh), np.uint64)
    if rep == 0:
        lib().or_grid_tables(seed, L, kh, z, m)
    else:
        lib().or_grid_tables_rep(seed, rep, L, kh, z, m)
    return z, m


def embedding(seed: int, d: int, ke: int = DEFAULT_EMBED_DIM) -> np.ndarray:
    """Scaled Gaussian matrix Z / (beta * ke), beta = sqrt(2/pi), [ke, d]
    (appendix theorem embedding l2 into l1)."""
    z = np.zeros((ke, d), np.float32)
    lib().or_embedding(seed, d, ke, z)
    return z


def default_scales(n_a: int, n_b: int, eps: float) -> int:
    """L = ceil(log2(max(n_A, n_B) / eps)) (CrudeNN figure: L = O(log(n/eps)))."""
    return int(lib().or_default_scales(n_a, n_b, eps))


def default_samples(n_a: int, eps: float) -> int:
    """T = ceil(ceil(log2 n_A) / eps^2) (main theorem: T = O(log(n)/eps^2))."""
    return int(lib().or_default_samples(n_a, eps))


# --------------------------------------------------------------------------
# CrudeNN
# --------------------------------------------------------------------------

def calibrate(A, B):
    A, B = _f32(A), _f32(B)
    d = A.shape[1]
    lo = np.zeros(d, np.float32)
    hi = np.zeros(d, np.float32)
    S = ctypes.c_double()
    e = _INT()
    lib().or_calibrate(A, A.shape[0], B, B.shape[0], d, lo, hi, ctypes.byref(S), ctypes.byref(e))
    return lo, hi, S.value, e.value


def hash_keys(X, metric, lo, Zs, L, e_top, zfrac, mult) -> np.ndarray:
    """keys[L, n] of every point of X (see ``bucket_key`` in the C source)."""
    X = _f32(X)
    n, d = X.shape
    keys = np.zeros((L, n), np.uint64)
    ke = 0 if Zs is None else Zs.shape[0]
    zp = None if Zs is None else Zs.ctypes.data
    lib().or_hash_keys(X, n, d, metric, lo, zp, ke, L, e_top, zfrac, mult, keys)
    return keys


def dist32(a, b, metric) -> np.float32:
    a, b = _f32(a), _f32(b)
    return np.float32(lib().or_dist32(a, b, a.shape[0], metric))


def crude_nn(A, B, metric, eps, seed, n_scales=0, embed_dim=DEFAULT_EMBED_DIM, window=1,
             reps=1):
    """CrudeNN figure.  Returns a dict with the per-point first colliding
    scale (L when none), the candidate b (lowest index in the bucket) and
    D_a = dist32(a, b), plus the intermediate keys and calibration.

    window W > 1 or reps k > 1: the variant of the large-scale experiments.
    Each of k independent LSH structures (grid stream rep = 0 .. k-1; the
    l2 embedding is the same for all) retrieves the first W distinct points
    of B from a's buckets, finest scale first; the candidate is the closest
    of the k W retrieved points (dist32, ties to the lower b) and the scale
    the finest first-collision scale over the structures.  The keys and
    tables returned are those of structure 0."""
    A, B = _f32(A), _f32(B)
    n_a, d = A.shape
    n_b = B.shape[0]
    L = n_scales if n_scales > 0 else default_scales(n_a, n_b, eps)
    lo, hi, S, e_top = calibrate(A, B)
    Zs = embedding(seed, d, embed_dim) if metric == L2 else None
    kh = d if metric == L1 else embed_dim
    out = None
    for r in range(reps):
        zfrac, mult = grid_tables(seed, L, kh, r)
        kA = hash_keys(A, metric, lo, Zs, L, e_top, zfrac, mult)
        kB = hash_keys(B, metric, lo, Zs, L, e_top, zfrac, mult)
        scale = np.zeros(n_a, np.int32)
        nn = np.zeros(n_a, np.int32)
        D = np.zeros(n_a, np.float32)
        if window == 1:
            lib().or_crude_nn(kA, n_a, kB, n_b, L, A, B, d, metric, scale, nn, D)
        else:
            lib().or_crude_window(kA, n_a, kB, n_b, L, window, A, B, d, metric, scale, nn, D)
        if out is None:
            out = dict(scale=scale, nn=nn, D=D, keys_a=kA, keys_b=kB, lo=lo, hi=hi, S=S,
                       e_top=e_top, L=L, embed=Zs, zfrac=zfrac, mult=mult)
            continue
        # the closest retrieved point over all structures, ties to the lower b
        better = (D < out["D"]) | ((D == out["D"]) & (nn < out["nn"]))
        out["D"] = np.where(better, D, out["D"])
        out["nn"] = np.where(better, nn, out["nn"])
        out["scale"] = np.minimum(out["scale"], scale)
    return out


# --------------------------------------------------------------------------
# Exact nearest neighbours and CH
# --------------------------------------------------------------------------

def nn_f64(X, B, metric, rows=None):
    X, B = _f32(X), _f32(B)
    nx = X.shape[0] if rows is None else len(rows)
    mind = np.zeros(nx, np.float64)
    arg = np.zeros(nx, np.int32)
    r = None
    if rows is not None:
        r = np.ascontiguousarray(rows, np.int32)
    lib().or_nn_f64(X, nx, None if r is None else r.ctypes.data, B, B.shape[0],
                    X.shape[1], metric, mind, arg)
    return mind, arg


def nn_f32(X, B, metric, rows=None):
    X, B = _f32(X), _f32(B)
    nx = X.shape[0] if rows is None else len(rows)
    mind = np.zeros(nx, np.float32)
    arg = np.zeros(nx, np.int32)
    r = None
    if rows is not None:
        r = np.ascontiguousarray(rows, np.int32)
    lib().or_nn_f32(X, nx, None if r is None else r.ctypes.data, B, B.shape[0],
                    X.shape[1], metric, mind, arg)
    return mind, arg


def chamfer_exact(A, B, metric):
    """CH(A, B) = sum_a min_b d(a, b), distances not squared; double
    precision, exactly rounded sum."""
    mind, arg = nn_f64(A, B, metric)
    return math.fsum(mind.tolist()), mind, arg


# --------------------------------------------------------------------------
# Chamfer-Estimate
# --------------------------------------------------------------------------

def weights(D):
    D = _f32(D)
    n = D.shape[0]
    w = np.zeros(n, np.uint64)
    P = np.zeros(n, np.uint64)
    s = _INT()
    W = ctypes.c_uint64()
    zero = lib().or_weights(D, n, ctypes.byref(s), w, P, ctypes.byref(W))
    return s.value, w, P, W.value, bool(zero)


def sample(seed, P, W, T):
    idx = np.zeros(T, np.int32)
    if T > 0 and W > 0:
        lib().or_sample(seed, np.ascontiguousarray(P, np.uint64), len(P), W, T, idx)
    return idx


SAMPLING_IMPORTANCE = 0
SAMPLING_UNIFORM = 1


def chamfer_estimate(A, B, metric, eps, T, seed, n_scales=0,
                     embed_dim=DEFAULT_EMBED_DIM, crude=None, window=1, reps=1,
                     sampling=SAMPLING_IMPORTANCE):
    """Chamfer-Estimate figure with the fixed-point distribution above.

    eta = (1/T) sum_l (W / w_{x_l}) * min_b d(x_l, b), the per-sample minima in
    double precision and the sum exactly rounded.  eta = 0 when every D_a is 0
    (then every min_b d(a, b) is 0 as well) and when A is empty.

    sampling=SAMPLING_UNIFORM is the uniform-sampling baseline of the
    uniform-vs-importance paragraph: the same steps with every D_a = 1, so
    every point has the same fixed-point weight w, the draw is uniform over A
    and (W / w) = n_A, i.e. eta = (n_A / T) sum_l min_b d(x_l, b)."""
    A, B = _f32(A), _f32(B)
    n_a = A.shape[0]
    if T <= 0:
        T = default_samples(max(n_a, 1), eps)
    if n_a == 0:
        return dict(eta=0.0, T=T, idx=np.zeros(0, np.int32), m=np.zeros(0), W=0, s=0,
                    D_norm=0.0, crude=None)
    if crude is None and sampling == SAMPLING_UNIFORM:
        crude = dict(D=np.ones(n_a, np.float32))
    if crude is None:
        crude = crude_nn(A, B, metric, eps, seed, n_scales, embed_dim, window, reps)
    s, w, P, W, zero = weights(crude["D"])
    if zero:
        return dict(eta=0.0, T=T, idx=np.zeros(T, np.int32), m=np.zeros(T), W=0, s=0,
                    D_norm=0.0, crude=crude, w=w, P=P)
    idx = sample(seed, P, W, T)
    m, arg = nn_f64(A, B, metric, rows=idx)
    terms = [(float(W) / float(w[i])) * float(mi) for i, mi in zip(idx.tolist(), m.tolist())]
    eta = math.fsum(terms) / T
    return dict(eta=eta, T=T, idx=idx, m=m, nn=arg, W=W, s=s, w=w, P=P,
                D_norm=math.ldexp(float(W), -s), crude=crude)


def chamfer_symmetric_exact(A, B, metric):
    """CH(A, B) + CH(B, A) (the symmetric form of the small-scale
    experiments); returns (sum, CH(A, B), CH(B, A))."""
    ab = chamfer_exact(A, B, metric)[0]
    ba = chamfer_exact(B, A, metric)[0]
    return ab + ba, ab, ba


def chamfer_symmetric_estimate(A, B, metric, eps, T, seed, **kw):
    """eta(A, B) + eta(B, A), both directions with the same seed and
    options; returns (sum, eta(A, B), eta(B, A))."""
    ab = chamfer_estimate(A, B, metric, eps, T, seed, **kw)["eta"]
    ba = chamfer_estimate(B, A, metric, eps, T, seed, **kw)["eta"]
    return ab + ba, ab, ba


def retrieve(A, clouds, metric, eps, T, seed, k, **kw):
    """One-vs-many retrieval (the downstream experiment: the nearest cloud
    under CH(A, B) + CH(B, A)): the symmetric estimate against every cloud,
    the k smallest (ties to the lower index), then their exact symmetric CH
    ranked ascending (ties to the lower index).  Returns (estimates, the k
    cloud indices, their exact values)."""
    est = np.array([chamfer_symmetric_estimate(A, B, metric, eps, T, seed, **kw)[0]
                    for B in clouds])
    cand = sorted(range(len(clouds)), key=lambda i: (est[i], i))[:k]
    ranked = sorted((chamfer_symmetric_exact(A, clouds[i], metric)[0], i) for i in cand)
    return est, [i for _, i in ranked], [v for v, _ in ranked]
