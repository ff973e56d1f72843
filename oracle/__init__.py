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
_I8 = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")
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
    L.or_set_threads.argtypes = [_INT]
    L.or_philox4x64.argtypes = [_U64, _U64, _U64]
    L.or_grid_tables.argtypes = [ctypes.c_uint64, _INT, _INT, _F32, _U64]
    L.or_grid_tables_rep.argtypes = [ctypes.c_uint64, ctypes.c_uint64, _INT, _INT, _F32, _U64]
    L.or_embedding.argtypes = [ctypes.c_uint64, _INT, _INT, _I8]
    L.or_default_scales.argtypes = [_I64, _I64, ctypes.c_double]
    L.or_default_scales.restype = _INT
    L.or_default_samples.argtypes = [_I64, ctypes.c_double]
    L.or_default_samples.restype = _I64
    L.or_calibrate.argtypes = [_F32, _I64, _F32, _I64, _INT, _F32, _F32,
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_INT)]
    L.or_hash_keys.argtypes = [_F32, _I64, _INT, _INT, _F32, _VP, _INT, _INT, _INT,
                               _F32, _U64, _U64]
    L.or_hashed_coords.argtypes = [_F32, _I64, _INT, _INT, _F32, _INT, _VP, _INT, _F32]
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
    L.or_sketch_direction.argtypes = [ctypes.c_uint64, _INT, _INT, _F64]
    L.or_project.argtypes = [_F32, _I64, _INT, _F64, _F64]
    L.or_part_tables.argtypes = [ctypes.c_uint64, _INT, _F32, _U64]
    L.or_part_keys.argtypes = [_F32, _I64, _INT, _INT, _F32, _INT, _VP, _INT, _INT, _F32, _U64,
                               _U64]
    L.or_pad.argtypes = [_F32, _I64, _INT, _INT, _INT, ctypes.c_uint64, ctypes.c_float, _F32]
    _lib = L
    return L


def threads() -> int:
    """OpenMP threads of the parallel loops (exact nearest neighbours)."""
    return int(lib().or_threads())


def set_threads(n: int) -> None:
    """Use n OpenMP threads in the parallel loops from now on."""
    lib().or_set_threads(int(n))


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
    """Quantised Gaussian matrix Zq = clamp(rint(32 g), -127, 127), int8
    [ke, d] (appendix theorem embedding l2 into l1; the scale 1 / (beta ke)
    with beta = sqrt(2/pi), and 1/32, is applied to the integer products)."""
    z = np.zeros((ke, d), np.int8)
    lib().or_embedding(seed, d, ke, z)
    return z


EMBED_SCALE = 32.0
EMBED_QBITS = 24


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


def hashed_coords(X, metric, lo, Zs, e_top) -> np.ndarray:
    """The coordinates the grid hash sees, Y[n, kh]: x - lo for l1 and, for
    l2, the embedding T(x - lo) of the appendix theorem embedding l2 into
    l1 in its finite-precision form: coordinates quantised to 24 bits of the
    span 2^e_top, an exact integer product with the quantised matrix, then
    scaled to float (see hashed_coords in the C source)."""
    X = _f32(X)
    n, d = X.shape
    kh = d if metric == 1 else Zs.shape[0]
    Y = np.zeros((n, kh), np.float32)
    Zs = None if Zs is None else np.ascontiguousarray(Zs, np.int8)
    zp = None if Zs is None else Zs.ctypes.data
    lib().or_hashed_coords(X, n, d, metric, _f32(lo), e_top, zp,
                           0 if Zs is None else Zs.shape[0], Y)
    return Y


def hash_keys(X, metric, lo, Zs, L, e_top, zfrac, mult) -> np.ndarray:
    """keys[L, n] of every point of X (see ``bucket_key`` in the C source)."""
    X = _f32(X)
    n, d = X.shape
    keys = np.zeros((L, n), np.uint64)
    Zs = None if Zs is None else np.ascontiguousarray(Zs, np.int8)
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


# --------------------------------------------------------------------------
# Reduction to bounded aspect ratio (lemma on the reduction to poly(n/eps)
# aspect ratio; its proof in the appendix: very crude estimate from a
# p-stable 1-D sketch, a coarse grid partition, appended random coordinates)
# --------------------------------------------------------------------------

REDUCE_NONE = 0
REDUCE_PARTITION = 1
REDUCE_PAD = 2


def ceil_log2(x: int) -> int:
    """Smallest k >= 0 with 2^k >= x (x >= 1)."""
    return max(0, (int(x) - 1).bit_length())


def sketch_direction(seed: int, d: int, metric: int) -> np.ndarray:
    """p-stable vector g: i.i.d. Cauchy entries for l1, Gaussian for l2."""
    g = np.zeros(d, np.float64)
    lib().or_sketch_direction(seed, d, metric, g)
    return g


def project(X, g) -> np.ndarray:
    """<x, g> per row, double precision, fused multiply-adds in ascending
    coordinate order."""
    X = _f32(X)
    p = np.zeros(X.shape[0], np.float64)
    lib().or_project(X, X.shape[0], X.shape[1], np.ascontiguousarray(g, np.float64), p)
    return p


def nearest_1d(pa, pb) -> np.ndarray:
    """t_a = min_b |pa - pb| by sorting pb and looking at the neighbours of
    each pa (the 1-D nearest-neighbour search of the proof); every
    difference is one IEEE subtraction."""
    s = np.sort(np.asarray(pb, np.float64))
    i = np.searchsorted(s, pa, side="left")
    t = np.full(len(pa), np.inf)
    has_succ = i < len(s)
    t[has_succ] = s[i[has_succ]] - pa[has_succ]
    has_pred = i > 0
    pred = pa[has_pred] - s[i[has_pred] - 1]
    t[has_pred] = np.minimum(t[has_pred], pred)
    return t


def pad_dims(n_a: int, n_b: int, d: int) -> int:
    """Padding coordinates: O(log n) of them, at least 3 ceil(log2 n), with
    d + m rounded up to the next of 16, 32, 64, 128 (a multiple of 16 above
    128)."""
    dp = d + 3 * ceil_log2(max(n_a, n_b, 2))
    if dp <= 128:
        w = 16
        while w < dp:
            w *= 2
        dp = w
    else:
        dp = -(-dp // 16) * 16
    return dp - d


def reduce_bounds(n_a: int, n_b: int, eps: float, max_t: float, d: int) -> dict:
    """Exponents and bounds from M = max_a t_a (one reading of the proof's
    constants, all powers of two so that both implementations agree):

    with n = max(n_A, n_B), a p-stable g' satisfies |g'| < t with probability
    at most t and |g'| > t with probability below 1/t (Cauchy; the Gaussian
    tail is lighter), so with probability at least 1 - 2/n
      k_hi = ceil(log2 n_A) + ceil(log2 n)                   (|g'| <= 2^k_hi)
      k_lo = ceil(log2 n_A) + ceil(log2 n_B) + ceil(log2 n)  (|g'| >= 2^-k_lo)
    give  eta_lo = 2^(e_M - k_hi) <= CH(A, B) <= eta_hi
                 = 2^(e_M + 1 + ceil(log2 n_A) + k_lo),  e_M = floor(log2 M).
    c = eta_hi / eta_lo; the partition side is 2^e_part >= c n eta_hi; the
    padding adds m = pad_dims(n_A, n_B, d) coordinates of magnitude
    q = eps eta_lo / (2 n m) (l1 norm of the padding vector eps eta_lo / (2n)).
    M = 0 (every a on top of a b in the projection): no partition, q = 0."""
    n = max(n_a, n_b, 2)
    la, lb, ln = ceil_log2(n_a), ceil_log2(n_b), ceil_log2(n)
    k_hi = la + ln
    k_lo = la + lb + ln
    m = pad_dims(n_a, n_b, d)
    if not max_t > 0.0:
        return dict(degenerate=True, e_M=0, k_hi=k_hi, k_lo=k_lo, e_part=0, m=m,
                    eta_lo=0.0, eta_hi=0.0, q=np.float32(0.0))
    e_M = math.frexp(max_t)[1] - 1
    e_hi = e_M + 1 + la + k_lo
    log2c = e_hi - (e_M - k_hi)
    e_part = log2c + ln + e_hi
    q = np.float32(math.ldexp(eps / float(2 * n * m), e_M - k_hi))
    return dict(degenerate=False, e_M=e_M, k_hi=k_hi, k_lo=k_lo, e_part=e_part, m=m,
                eta_lo=math.ldexp(1.0, e_M - k_hi), eta_hi=math.ldexp(1.0, e_hi), q=q)


def part_tables(seed: int, kh: int):
    z = np.zeros(kh, np.float32)
    m = np.zeros(kh, np.uint64)
    lib().or_part_tables(seed, kh, z, m)
    return z, m


def part_keys(X, metric, lo, e_top, Zs, e, zfrac, mult) -> np.ndarray:
    """Key of every point's cell of side 2^e (see or_part_keys)."""
    X = _f32(X)
    n, d = X.shape
    keys = np.zeros(n, np.uint64)
    Zs = None if Zs is None else np.ascontiguousarray(Zs, np.int8)
    ke = 0 if Zs is None else Zs.shape[0]
    zp = None if Zs is None else Zs.ctypes.data
    lib().or_part_keys(X, n, d, metric, lo, e_top, zp, ke, e, zfrac, mult, keys)
    return keys


def pad(X, m: int, side: int, seed: int, q) -> np.ndarray:
    """X with m appended coordinates +-q (signs from the counter (row, side,
    PAD))."""
    X = _f32(X)
    n, d = X.shape
    out = np.zeros((n, d + m), np.float32)
    lib().or_pad(X, n, d, m, side, seed, np.float32(q), out)
    return out


def aspect_reduce(A, B, metric, eps, seed, embed_dim=DEFAULT_EMBED_DIM):
    """The reduction's steps: g, projections, t_a, their sum (the 1-D
    Chamfer distance, a poly(n)-approximation of CH) and maximum, the bounds
    and exponents, and the partition keys of A and B (cells of side
    2^e_part of the grid hash on the hashed coordinates: x - lo for l1, the
    l2 -> l1 embedding for l2)."""
    A, B = _f32(A), _f32(B)
    d = A.shape[1]
    g = sketch_direction(seed, d, metric)
    pa, pb = project(A, g), project(B, g)
    t = nearest_1d(pa, pb)
    max_t = float(t.max()) if len(t) else 0.0
    out = reduce_bounds(A.shape[0], B.shape[0], eps, max_t, d)
    out.update(g=g, pa=pa, pb=pb, t=t, max_t=max_t, ch1=math.fsum(t.tolist()))
    lo, _, _, e_top = calibrate(A, B)
    Zs = embedding(seed, d, embed_dim) if metric == L2 else None
    kh = d if metric == L1 else Zs.shape[0]
    zf, mt = part_tables(seed, kh)
    if out["degenerate"]:
        out["keys_A"] = np.zeros(A.shape[0], np.uint64)
        out["keys_B"] = np.zeros(B.shape[0], np.uint64)
    else:
        out["keys_A"] = part_keys(A, metric, lo, e_top, Zs, out["e_part"], zf, mt)
        out["keys_B"] = part_keys(B, metric, lo, e_top, Zs, out["e_part"], zf, mt)
    return out


def parts(keys_A, keys_B):
    """The partition as lists of row indices per part, parts in ascending
    key order, rows ascending; None when some part of A has no point of B
    (the event the proof bounds by 1/n: the partition is then not used)."""
    ka = np.asarray(keys_A)
    kb = np.asarray(keys_B)
    out = []
    for k in np.unique(ka):
        ra = np.nonzero(ka == k)[0]
        rb = np.nonzero(kb == k)[0]
        if len(rb) == 0:
            return None
        out.append((ra, rb))
    return out


def chamfer_estimate_reduced(A, B, metric, eps, T, seed, reduction=REDUCE_PARTITION,
                             embed_dim=DEFAULT_EMBED_DIM, **kw):
    """The estimator applied after the reduction: partition A and B, pad
    (reduction = REDUCE_PAD: both sets get the m coordinates +-q before the
    estimate, rows keyed by their index in A or B), and sum the estimates
    of the parts in ascending key order (a trivial or unusable partition is
    one part: the plain estimate of the, possibly padded, sets)."""
    A, B = _f32(A), _f32(B)
    if A.shape[0] == 0:
        return dict(eta=0.0, parts=0, info=None)
    info = aspect_reduce(A, B, metric, eps, seed, embed_dim)
    if reduction == REDUCE_PAD:
        A = pad(A, info["m"], 0, seed, info["q"])
        B = pad(B, info["m"], 1, seed, info["q"])
    pl = parts(info["keys_A"], info["keys_B"])
    if pl is None or len(pl) == 1:
        r = chamfer_estimate(A, B, metric, eps, T, seed, embed_dim=embed_dim, **kw)
        return dict(eta=r["eta"], parts=1, info=info)
    eta = 0.0
    for ra, rb in pl:
        eta += chamfer_estimate(A[ra], B[rb], metric, eps, T, seed, embed_dim=embed_dim,
                                **kw)["eta"]
    return dict(eta=eta, parts=len(pl), info=info)
