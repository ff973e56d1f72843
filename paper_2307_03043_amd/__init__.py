"""Python binding of libchamfer (gfx950 / MI355X).

Thin ctypes marshalling over the C ABI declared in ``include/chamfer.h``:
every function here has the name of a C entry point, turns torch tensors
into device pointers, passes torch's current HIP stream and a cached
workspace, and returns torch tensors.  All computation happens in the HIP
kernels of ``libchamfer.so``; if the library is missing or was not built for
this machine, every call raises.

Point sets are float32 CUDA (HIP) tensors of shape [n, d], contiguous.
"""

from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_HERE, "libchamfer.so")

L1 = 1
L2 = 2
FP32, BF16, FP8 = 0, 1, 2

_STATUS = {0: "ok", -1: "invalid argument", -2: "workspace missing or too small",
           -3: "HIP launch or runtime error", -4: "input contains NaN or Inf",
           -5: "problem needs more workspace than the static scratch buffer holds"}


class ChamferError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {_STATUS.get(status, status)} (status {status})")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("n_scales", ctypes.c_int32), ("embed_dim", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("window", ctypes.c_int32),
                ("reps", ctypes.c_int32), ("sampling", ctypes.c_int32),
                ("reduction", ctypes.c_int32)]


REDUCE_NONE, REDUCE_PARTITION, REDUCE_PAD = 0, 1, 2


class Reduction(ctypes.Structure):
    """chamfer_reduction: the reduction's bounds and exponents."""
    _fields_ = [("ch1", ctypes.c_double), ("max_t", ctypes.c_double),
                ("eta_lo", ctypes.c_double), ("eta_hi", ctypes.c_double),
                ("e_M", ctypes.c_int32), ("e_part", ctypes.c_int32),
                ("pad_dims", ctypes.c_int32), ("pad_value", ctypes.c_float),
                ("degenerate", ctypes.c_int32), ("one_part", ctypes.c_int32)]


_AUX_ARRAYS = ("sample_idx", "sample_min", "sample_nn", "D", "W", "s", "status",
               "crude_D", "crude_nn", "crude_scale")
STAGE_EVENTS = 7


class Aux(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in _AUX_ARRAYS] + [("stage_events", ctypes.c_void_p)]


_lib = None
_lib_lock = threading.Lock()

_VP, _I64, _I32, _U64, _F64 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                              ctypes.c_uint64, ctypes.c_double)
_SIGS = {
    "chamfer_workspace_bytes": (ctypes.c_size_t, [_I64, _I64, _I32, _I32, _F64, _I64, _VP]),
    "chamfer_exact": (ctypes.c_int, [_VP, _VP, _I64, _I64, _I32, _I32, _VP, _VP, _VP, _VP, _VP,
                                     ctypes.c_size_t, _VP]),
    "crude_nn": (ctypes.c_int, [_VP, _VP, _I64, _I64, _I32, _I32, _F64, _U64, _VP, _VP, _VP,
                                _VP, _VP, ctypes.c_size_t, _VP]),
    "chamfer_estimate": (ctypes.c_int, [_VP, _VP, _I64, _I64, _I32, _I32, _F64, _I64, _U64,
                                        _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "chamfer_estimate_noalloc": (ctypes.c_int, [_VP, _VP, _I64, _I64, _I32, _I32, _F64, _I64,
                                                _U64, _VP, _VP, _VP, _VP]),
    "chamfer_hash_keys": (ctypes.c_int, [_VP, _VP, _I64, _I64, _I32, _I32, _F64, _U64, _VP,
                                         _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "chamfer_nn_min": (ctypes.c_int, [_VP, _VP, _I64, _VP, _I64, _I32, _I32, _VP, _VP, _VP,
                                      _VP, ctypes.c_size_t, _VP]),
    "chamfer_estimate_symmetric": (ctypes.c_int, [_VP, _VP, _I64, _I64, _I32, _I32, _F64, _I64,
                                                  _U64, _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "chamfer_exact_symmetric": (ctypes.c_int, [_VP, _VP, _I64, _I64, _I32, _I32, _VP, _VP, _VP,
                                               ctypes.c_size_t, _VP]),
    "chamfer_retrieve_workspace_bytes": (ctypes.c_size_t, [_I64, _VP, _I32, _I32, _I32, _F64,
                                                           _I64, _VP]),
    "chamfer_retrieve": (ctypes.c_int, [_VP, _I64, _VP, _VP, _I32, _I32, _I32, _F64, _I64, _U64,
                                        _I32, _VP, _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "chamfer_default_samples": (ctypes.c_int64, [_I64, _F64]),
    "chamfer_pad_dims": (ctypes.c_int32, [_I64, _I64, _I32]),
    "chamfer_reduce_workspace_bytes": (ctypes.c_size_t, [_I64, _I64, _I32, _I32, _VP]),
    "chamfer_aspect_reduce": (ctypes.c_int, [_VP, _VP, _I64, _I64, _I32, _I32, _F64, _U64, _VP,
                                             _VP, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_size_t,
                                             _VP]),
    "chamfer_default_scales": (ctypes.c_int32, [_I64, _I64, _F64]),
    "chamfer_embedding_matrix": (ctypes.c_int, [_U64, _I32, _I32, _VP]),
    "chamfer_split_score_bound": (ctypes.c_double, [_I32, _I32, ctypes.c_float, ctypes.c_float]),
    "chamfer_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "chamfer_server_create": (ctypes.c_int, [ctypes.c_size_t, _I32, _VP]),
    "chamfer_server_warm": (ctypes.c_int, [_VP, _I32, _I32, _I32, _I32]),
    "chamfer_server_submit": (ctypes.c_int, [_VP, _VP, _VP]),
    "chamfer_server_progress": (ctypes.c_int, [_VP]),
    "chamfer_server_results": (ctypes.c_int, [_VP, _VP, _I32]),
    "chamfer_server_stats": (ctypes.c_int, [_VP, _VP]),
    "chamfer_server_destroy": (ctypes.c_int, [_VP]),
}


def lib() -> ctypes.CDLL:
    """Load libchamfer.so (raises if it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(SO_PATH):
                raise RuntimeError(f"libchamfer.so not built ({SO_PATH}); run "
                                   "`python -c 'import __graft_entry__ as g; g.build()'`")
            L = ctypes.CDLL(SO_PATH)
            for name, (res, args) in _SIGS.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != 0:
        raise ChamferError(rc, where)


IMPORTANCE, UNIFORM = 0, 1  # enum chamfer_sampling


def _opts(n_scales=0, embed_dim=0, precision=0, window=0, reps=0, sampling=0,
          reduction=0) -> Opts:
    return Opts(n_scales, embed_dim, precision, window, reps, sampling, reduction)


# ----------------------------------------------------------- torch glue ---

def _torch():
    import torch
    return torch


def _points(x, name):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if x.dtype != torch.float32 or x.dim() != 2 or not x.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 [n, d] tensor")
    return x


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


_ws_cache: dict = {}


def _workspace(nbytes: int, device):
    """A cached uint8 device buffer per (device, stream) of at least nbytes."""
    torch = _torch()
    key = (device.index if device.index is not None else torch.cuda.current_device(),
           torch.cuda.current_stream(device).cuda_stream)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def release_workspaces():
    _ws_cache.clear()


# ------------------------------------------------------------- host API ---

def chamfer_workspace_bytes(n_a, n_b, d, metric, eps=0.5, T=0, n_scales=0, embed_dim=0,
                            precision=0, window=0, reps=0, sampling=0, reduction=0) -> int:
    o = _opts(n_scales, embed_dim, precision, window, reps, sampling, reduction)
    return int(lib().chamfer_workspace_bytes(n_a, n_b, d, metric, eps, T, ctypes.byref(o)))


def chamfer_default_samples(n_a: int, eps: float) -> int:
    return int(lib().chamfer_default_samples(n_a, eps))


def chamfer_default_scales(n_a: int, n_b: int, eps: float) -> int:
    return int(lib().chamfer_default_scales(n_a, n_b, eps))


def chamfer_split_score_bound(d: int, terms: int, xn2: float, b2max: float) -> float:
    """The certificate bound E of the l2 exact pass (host arithmetic only)."""
    return float(lib().chamfer_split_score_bound(d, terms, xn2, b2max))


def chamfer_embedding_matrix(seed: int, d: int, embed_dim: int = 32) -> np.ndarray:
    z = np.zeros((embed_dim, d), np.int8)
    _check(lib().chamfer_embedding_matrix(seed, d, embed_dim, z.ctypes.data),
           "chamfer_embedding_matrix")
    return z


# ----------------------------------------------------------- device API ---

def chamfer_exact(A, B, metric=L2, *, precision=0, rows_out=True):
    """Exact CH(A, B) (double, [1] tensor) and the per-row min / arg-min."""
    torch = _torch()
    A, B = _points(A, "A"), _points(B, "B")
    n_a, d = A.shape
    n_b = B.shape[0]
    if B.shape[1] != d:
        raise ValueError("A and B differ in dimension")
    dev = A.device
    o = _opts(precision=precision)
    nbytes = lib().chamfer_workspace_bytes(n_a, n_b, d, metric, 0.0, 0, ctypes.byref(o))
    if nbytes == 0:
        raise ChamferError(-1, "chamfer_exact")
    ws = _workspace(nbytes, dev)
    ch = torch.empty(1, dtype=torch.float64, device=dev)
    rmin = torch.empty(n_a, dtype=torch.float32, device=dev) if rows_out else None
    rnn = torch.empty(n_a, dtype=torch.int32, device=dev) if rows_out else None
    _check(lib().chamfer_exact(_ptr(A), _ptr(B), n_a, n_b, d, metric, _ptr(ch), _ptr(rmin),
                               _ptr(rnn), ctypes.byref(o), _ptr(ws), ws.numel(), _stream(dev)),
           "chamfer_exact")
    return ch, rmin, rnn


def chamfer_nn_min(X, B, metric=L2, rows=None, *, precision=0):
    """Nearest neighbour in B of rows of X (all rows, or X[rows])."""
    torch = _torch()
    X, B = _points(X, "X"), _points(B, "B")
    d = X.shape[1]
    if B.shape[1] != d:
        raise ValueError("X and B differ in dimension")
    if rows is not None:
        if rows.dtype != torch.int32 or not rows.is_cuda or not rows.is_contiguous():
            raise TypeError("rows must be a contiguous int32 CUDA tensor")
        n_x = rows.numel()
    else:
        n_x = X.shape[0]
    dev = X.device
    o = _opts(precision=precision)
    nbytes = lib().chamfer_workspace_bytes(n_x, B.shape[0], d, metric, 0.0, 0, ctypes.byref(o))
    if nbytes == 0:
        raise ChamferError(-1, "chamfer_nn_min")
    ws = _workspace(nbytes, dev)
    mn = torch.empty(n_x, dtype=torch.float32, device=dev)
    arg = torch.empty(n_x, dtype=torch.int32, device=dev)
    _check(lib().chamfer_nn_min(_ptr(X), _ptr(rows), n_x, _ptr(B), B.shape[0], d, metric,
                                _ptr(mn), _ptr(arg), ctypes.byref(o), _ptr(ws), ws.numel(),
                                _stream(dev)), "chamfer_nn_min")
    return mn, arg


def crude_nn(A, B, metric, eps, seed, *, n_scales=0, embed_dim=0, window=0, reps=0):
    """CrudeNN: D_a (float32), candidate b, first colliding scale."""
    torch = _torch()
    A, B = _points(A, "A"), _points(B, "B")
    n_a, d = A.shape
    dev = A.device
    o = _opts(n_scales, embed_dim, window=window, reps=reps)
    nbytes = lib().chamfer_workspace_bytes(n_a, B.shape[0], d, metric, eps, 0, ctypes.byref(o))
    if nbytes == 0:
        raise ChamferError(-1, "crude_nn")
    ws = _workspace(nbytes, dev)
    D = torch.empty(n_a, dtype=torch.float32, device=dev)
    nn = torch.empty(n_a, dtype=torch.int32, device=dev)
    sc = torch.empty(n_a, dtype=torch.int32, device=dev)
    _check(lib().crude_nn(_ptr(A), _ptr(B), n_a, B.shape[0], d, metric, eps, seed, _ptr(D),
                          _ptr(nn), _ptr(sc), ctypes.byref(o), _ptr(ws), ws.numel(),
                          _stream(dev)), "crude_nn")
    return D, nn, sc


def chamfer_estimate(A, B, metric, eps, T=0, seed=0, *, n_scales=0, embed_dim=0, precision=0,
                     window=0, reps=0, sampling=0, reduction=0,
                     with_aux=True, stage_events=None):
    """(1 +- eps) estimate of CH(A, B).  Returns a dict of device tensors:
    eta [1] double, and with_aux: sample_idx/min/nn [T], D, W, s, status,
    crude_D/nn/scale [n_A].  stage_events: optional ctypes array of
    STAGE_EVENTS hipEvent_t handles recorded at the stage boundaries.
    reduction (REDUCE_PARTITION / REDUCE_PAD): the estimate after the
    reduction to bounded aspect ratio (no aux outputs; synchronises once)."""
    torch = _torch()
    A, B = _points(A, "A"), _points(B, "B")
    n_a, d = A.shape
    n_b = B.shape[0]
    dev = A.device
    o = _opts(n_scales, embed_dim, precision, window, reps, sampling, reduction)
    if reduction:
        with_aux = False
    if T == 0 and 0.0 < eps < 1.0 and not reduction:
        T = chamfer_default_samples(max(n_a, 1), eps)
    nbytes = lib().chamfer_workspace_bytes(n_a, n_b, d, metric, eps, T, ctypes.byref(o))
    if nbytes == 0:
        raise ChamferError(-1, "chamfer_estimate")
    ws = _workspace(nbytes, dev)
    out = {"eta": torch.empty(1, dtype=torch.float64, device=dev), "T": T}
    aux = Aux()
    if with_aux:
        out.update(
            sample_idx=torch.empty(T, dtype=torch.int32, device=dev),
            sample_min=torch.empty(T, dtype=torch.float32, device=dev),
            sample_nn=torch.empty(T, dtype=torch.int32, device=dev),
            D=torch.empty(1, dtype=torch.float64, device=dev),
            W=torch.empty(1, dtype=torch.int64, device=dev),
            s=torch.empty(1, dtype=torch.int32, device=dev),
            status=torch.empty(1, dtype=torch.int32, device=dev),
            crude_D=torch.empty(n_a, dtype=torch.float32, device=dev),
            crude_nn=torch.empty(n_a, dtype=torch.int32, device=dev),
            crude_scale=torch.empty(n_a, dtype=torch.int32, device=dev),
        )
        for f in _AUX_ARRAYS:
            setattr(aux, f, out[f].data_ptr())
    if stage_events is not None:
        aux.stage_events = ctypes.cast(stage_events, ctypes.c_void_p)
    _check(lib().chamfer_estimate(_ptr(A), _ptr(B), n_a, n_b, d, metric, eps, T, seed,
                                  _ptr(out["eta"]), None if reduction else ctypes.byref(aux),
                                  ctypes.byref(o),
                                  _ptr(ws), ws.numel(), _stream(dev)), "chamfer_estimate")
    return out


def chamfer_estimate_noalloc(A, B, metric, eps, T=0, seed=0, *, n_scales=0, embed_dim=0,
                             precision=0, window=0, reps=0, sampling=0):
    """chamfer_estimate on the library's static scratch array instead of a
    workspace (no device allocation inside the call; the outputs below are
    allocated here, by the caller).  Same outputs as chamfer_estimate."""
    torch = _torch()
    A, B = _points(A, "A"), _points(B, "B")
    n_a, d = A.shape
    n_b = B.shape[0]
    dev = A.device
    o = _opts(n_scales, embed_dim, precision, window, reps, sampling)
    if T == 0 and 0.0 < eps < 1.0:
        T = chamfer_default_samples(max(n_a, 1), eps)
    out = {"eta": torch.empty(1, dtype=torch.float64, device=dev), "T": T}
    out.update(
        sample_idx=torch.empty(T, dtype=torch.int32, device=dev),
        sample_min=torch.empty(T, dtype=torch.float32, device=dev),
        sample_nn=torch.empty(T, dtype=torch.int32, device=dev),
        D=torch.empty(1, dtype=torch.float64, device=dev),
        W=torch.empty(1, dtype=torch.int64, device=dev),
        s=torch.empty(1, dtype=torch.int32, device=dev),
        status=torch.empty(1, dtype=torch.int32, device=dev),
        crude_D=torch.empty(n_a, dtype=torch.float32, device=dev),
        crude_nn=torch.empty(n_a, dtype=torch.int32, device=dev),
        crude_scale=torch.empty(n_a, dtype=torch.int32, device=dev),
    )
    aux = Aux()
    for f in _AUX_ARRAYS:
        setattr(aux, f, out[f].data_ptr())
    _check(lib().chamfer_estimate_noalloc(_ptr(A), _ptr(B), n_a, n_b, d, metric, eps, T, seed,
                                          _ptr(out["eta"]), ctypes.byref(aux), ctypes.byref(o),
                                          _stream(dev)), "chamfer_estimate_noalloc")
    return out


def chamfer_estimate_symmetric(A, B, metric, eps, T=0, seed=0, *, n_scales=0, embed_dim=0,
                               precision=0, window=0, reps=0, sampling=0):
    """eta(A, B) + eta(B, A): a float64 device tensor [sum, A->B, B->A]."""
    torch = _torch()
    A, B = _points(A, "A"), _points(B, "B")
    n_a, d = A.shape
    n_b = B.shape[0]
    dev = A.device
    o = _opts(n_scales, embed_dim, precision, window, reps, sampling)
    nbytes = max(lib().chamfer_workspace_bytes(n_a, n_b, d, metric, eps, T, ctypes.byref(o)),
                 lib().chamfer_workspace_bytes(n_b, n_a, d, metric, eps, T, ctypes.byref(o)))
    if nbytes == 0:
        raise ChamferError(-1, "chamfer_estimate_symmetric")
    ws = _workspace(nbytes, dev)
    out = torch.empty(3, dtype=torch.float64, device=dev)
    _check(lib().chamfer_estimate_symmetric(_ptr(A), _ptr(B), n_a, n_b, d, metric, eps, T, seed,
                                            _ptr(out), ctypes.byref(o), _ptr(ws), ws.numel(),
                                            _stream(dev)), "chamfer_estimate_symmetric")
    return out


def chamfer_exact_symmetric(A, B, metric, *, precision=0):
    """CH(A, B) + CH(B, A): a float64 device tensor [sum, A->B, B->A]."""
    torch = _torch()
    A, B = _points(A, "A"), _points(B, "B")
    n_a, d = A.shape
    n_b = B.shape[0]
    dev = A.device
    o = _opts(precision=precision)
    nbytes = max(lib().chamfer_workspace_bytes(n_a, n_b, d, metric, 0.0, 0, ctypes.byref(o)),
                 lib().chamfer_workspace_bytes(n_b, n_a, d, metric, 0.0, 0, ctypes.byref(o)))
    if nbytes == 0:
        raise ChamferError(-1, "chamfer_exact_symmetric")
    ws = _workspace(nbytes, dev)
    out = torch.empty(3, dtype=torch.float64, device=dev)
    _check(lib().chamfer_exact_symmetric(_ptr(A), _ptr(B), n_a, n_b, d, metric, _ptr(out),
                                         ctypes.byref(o), _ptr(ws), ws.numel(), _stream(dev)),
           "chamfer_exact_symmetric")
    return out


def chamfer_pad_dims(n_a: int, n_b: int, d: int) -> int:
    return int(lib().chamfer_pad_dims(n_a, n_b, d))


def chamfer_aspect_reduce(A, B, metric, eps, seed=0, *, embed_dim=0, pad=False):
    """The reduction to bounded aspect ratio (chamfer_aspect_reduce): a dict
    with the host copy of chamfer_reduction (`info`), t [n_A] float64, the
    partition keys of A and B (int64 views of the uint64 keys) and, with
    pad=True, the padded copies [n, d + m]."""
    torch = _torch()
    A, B = _points(A, "A"), _points(B, "B")
    n_a, d = A.shape
    n_b = B.shape[0]
    if B.shape[1] != d:
        raise ValueError("A and B differ in dimension")
    dev = A.device
    o = _opts(embed_dim=embed_dim)
    nbytes = lib().chamfer_reduce_workspace_bytes(n_a, n_b, d, metric, ctypes.byref(o))
    if nbytes == 0:
        raise ChamferError(-1, "chamfer_aspect_reduce")
    ws = _workspace(nbytes, dev)
    info = torch.zeros(ctypes.sizeof(Reduction), dtype=torch.uint8, device=dev)
    out = {"t": torch.empty(n_a, dtype=torch.float64, device=dev),
           "keys_A": torch.empty(n_a, dtype=torch.int64, device=dev),
           "keys_B": torch.empty(n_b, dtype=torch.int64, device=dev)}
    m = chamfer_pad_dims(n_a, n_b, d)
    if pad:
        out["A_pad"] = torch.empty(n_a, d + m, dtype=torch.float32, device=dev)
        out["B_pad"] = torch.empty(n_b, d + m, dtype=torch.float32, device=dev)
    _check(lib().chamfer_aspect_reduce(_ptr(A), _ptr(B), n_a, n_b, d, metric, eps, seed,
                                       ctypes.byref(o), _ptr(info), _ptr(out["t"]),
                                       _ptr(out["keys_A"]), _ptr(out["keys_B"]),
                                       _ptr(out.get("A_pad")), _ptr(out.get("B_pad")), _ptr(ws),
                                       ws.numel(), _stream(dev)), "chamfer_aspect_reduce")
    r = Reduction.from_buffer_copy(bytes(info.cpu().numpy()))
    out["info"] = {f: getattr(r, f) for f, _ in Reduction._fields_}
    return out


def chamfer_retrieve(A, clouds, metric, eps, T=0, seed=0, k=10, **kw):
    """Nearest clouds to A under CH(A, B) + CH(B, A): `clouds` is a list of
    [n_i, d] device tensors (concatenated here; chamfer_retrieve_packed
    takes them already packed).  Returns (est [m] float64 device tensor of
    symmetric estimates, top-k cloud indices ranked by exact symmetric CH,
    their exact values)."""
    torch = _torch()
    Bs = torch.cat([_points(B, "B") for B in clouds]).contiguous()
    return chamfer_retrieve_packed(A, Bs, [int(B.shape[0]) for B in clouds], metric, eps, T,
                                   seed, k, **kw)


def chamfer_retrieve_packed(A, Bs, sizes, metric, eps, T=0, seed=0, k=10, *, n_scales=0,
                            embed_dim=0, precision=0):
    """As chamfer_retrieve, with the m clouds back to back in one [sum n_i,
    d] device tensor `Bs` and their sizes in `sizes`."""
    torch = _torch()
    A, Bs = _points(A, "A"), _points(Bs, "Bs")
    n_a, d = A.shape
    dev = A.device
    offsets = np.zeros(len(sizes) + 1, np.int64)
    offsets[1:] = np.cumsum(sizes)
    if offsets[-1] != Bs.shape[0] or Bs.shape[1] != d:
        raise ValueError("chamfer_retrieve: sizes do not match Bs")
    m = len(sizes)
    o = _opts(n_scales, embed_dim, precision)
    nbytes = lib().chamfer_retrieve_workspace_bytes(n_a, offsets.ctypes.data, m, d, metric, eps,
                                                    T, ctypes.byref(o))
    if nbytes == 0:
        raise ChamferError(-1, "chamfer_retrieve")
    ws = _workspace(nbytes, dev)
    est = torch.empty(m, dtype=torch.float64, device=dev)
    top = np.zeros(k, np.int32)
    vals = np.zeros(k, np.float64)
    _check(lib().chamfer_retrieve(_ptr(A), n_a, _ptr(Bs), offsets.ctypes.data, m, d, metric, eps,
                                  T, seed, k, ctypes.byref(o), _ptr(est), top.ctypes.data,
                                  vals.ctypes.data, _ptr(ws), ws.numel(), _stream(dev)),
           "chamfer_retrieve")
    return est, top.tolist(), vals.tolist()


def chamfer_hash_keys(A, B, metric, eps, seed, *, n_scales=0, embed_dim=0):
    """Bucket keys [L, n_A], [L, n_B] (int64 holding the uint64 keys < 2^63)
    and e_top."""
    torch = _torch()
    A, B = _points(A, "A"), _points(B, "B")
    n_a, d = A.shape
    n_b = B.shape[0]
    dev = A.device
    o = _opts(n_scales, embed_dim)
    L = n_scales if n_scales else chamfer_default_scales(n_a, n_b, eps)
    nbytes = lib().chamfer_workspace_bytes(n_a, n_b, d, metric, eps, 0, ctypes.byref(o))
    if nbytes == 0:
        raise ChamferError(-1, "chamfer_hash_keys")
    ws = _workspace(nbytes, dev)
    ka = torch.empty((L, n_a), dtype=torch.int64, device=dev)
    kb = torch.empty((L, n_b), dtype=torch.int64, device=dev)
    et = torch.empty(1, dtype=torch.int32, device=dev)
    _check(lib().chamfer_hash_keys(_ptr(A), _ptr(B), n_a, n_b, d, metric, eps, seed, _ptr(ka),
                                   _ptr(kb), _ptr(et), ctypes.byref(o), _ptr(ws), ws.numel(),
                                   _stream(dev)), "chamfer_hash_keys")
    return ka, kb, et


# -------------------------------------------------------------- serving ---

class Request(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("n_A", ctypes.c_int64),
                ("n_B", ctypes.c_int64), ("d", ctypes.c_int32), ("metric", ctypes.c_int32),
                ("eps", ctypes.c_double), ("T", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("opts", Opts)]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int32), ("s", ctypes.c_int32),
                ("eta", ctypes.c_double), ("D", ctypes.c_double), ("W", ctypes.c_uint64),
                ("submit_s", ctypes.c_double), ("admit_s", ctypes.c_double),
                ("done_s", ctypes.c_double), ("footprint", ctypes.c_size_t)]


class ServerStat(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int64), ("in_flight", ctypes.c_int32),
                ("lanes_busy", ctypes.c_int32),
                ("arena_bytes", ctypes.c_size_t), ("arena_used", ctypes.c_size_t),
                ("arena_peak", ctypes.c_size_t), ("batches", ctypes.c_int64),
                ("batched", ctypes.c_int64), ("graphs", ctypes.c_int64),
                ("stalls", ctypes.c_int64)]


def chamfer_server_create(arena_bytes: int, lanes: int = 4):
    h = ctypes.c_void_p()
    _check(lib().chamfer_server_create(arena_bytes, lanes, ctypes.byref(h)),
           "chamfer_server_create")
    return h


class ChamferServer:
    """Continuous-batching server (see chamfer_server_* in chamfer.h).

    Host point sets are numpy float32 arrays or CPU torch tensors (pinned
    tensors make the copy-in asynchronous); they are kept alive here until the
    request's result has been drained."""

    def __init__(self, arena_bytes: int, lanes: int = 4):
        self.h = chamfer_server_create(arena_bytes, lanes)
        self._keep = {}

    @staticmethod
    def _host_ptr(x, name):
        if hasattr(x, "data_ptr"):
            if x.is_cuda or x.dtype.__str__() != "torch.float32" or not x.is_contiguous():
                raise TypeError(f"{name} must be a contiguous float32 CPU tensor")
            return x.data_ptr(), x.shape
        x = np.ascontiguousarray(x)
        if x.dtype != np.float32:
            raise TypeError(f"{name} must be float32")
        return x.ctypes.data, x.shape

    def submit(self, A, B, metric, eps, T=0, seed=0, *, n_scales=0, embed_dim=0, precision=0):
        pa, sa = self._host_ptr(A, "A")
        pb, sb = self._host_ptr(B, "B")
        if len(sa) != 2 or len(sb) != 2 or sa[1] != sb[1]:
            raise ValueError("A and B must be [n, d] with the same d")
        req = Request(pa, pb, sa[0], sb[0], sa[1], metric, eps, T, seed,
                      _opts(n_scales, embed_dim, precision))
        rid = ctypes.c_uint64()
        _check(lib().chamfer_server_submit(self.h, ctypes.byref(req), ctypes.byref(rid)),
               "chamfer_server_submit")
        self._keep[rid.value] = (A, B)
        return rid.value

    def warm(self, d, metric, *, embed_dim=0, precision=0):
        """Instantiate the graph of a request class on every lane now."""
        _check(lib().chamfer_server_warm(self.h, d, metric, embed_dim, precision),
               "chamfer_server_warm")

    def progress(self) -> int:
        n = lib().chamfer_server_progress(self.h)
        if n < 0:
            raise ChamferError(n, "chamfer_server_progress")
        return n

    def results(self, max_n: int = 1024):
        buf = (Result * max_n)()
        n = lib().chamfer_server_results(self.h, buf, max_n)
        if n < 0:
            raise ChamferError(n, "chamfer_server_results")
        out = []
        for i in range(n):
            r = buf[i]
            self._keep.pop(r.id, None)
            out.append({f: getattr(r, f) for f, _ in Result._fields_})
        return out

    def stats(self):
        st = ServerStat()
        _check(lib().chamfer_server_stats(self.h, ctypes.byref(st)), "chamfer_server_stats")
        return {f: getattr(st, f) for f, _ in ServerStat._fields_}

    def close(self):
        if self.h is not None:
            lib().chamfer_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
