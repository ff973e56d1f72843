"""CPU-side checks of the C ABI (no device work): the library loads and
exports every function declared in include/chamfer.h, the host helpers agree
with the oracle, and argument errors are rejected before any launch."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_2307_03043_amd as ch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chamfer.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("chamfer_exact", "crude_nn", "chamfer_estimate", "chamfer_workspace_bytes",
                     "chamfer_strerror", "chamfer_hash_keys", "chamfer_nn_min"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ch.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
        ctypes.cast(getattr(lib, name), ctypes.c_void_p)


def test_strerror():
    lib = ch.lib()
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.chamfer_strerror(code)
    assert lib.chamfer_strerror(0) == b"ok"


def test_default_parameters_match_oracle(orc):
    for n_a, n_b, eps in [(100000, 100000, 0.1), (4096, 4096, 0.2), (1, 1, 0.5),
                          (10**6, 10**6, 0.1), (12345, 77, 0.3), (2**20, 2**20, 0.25)]:
        assert ch.chamfer_default_scales(n_a, n_b, eps) == orc.default_scales(n_a, n_b, eps)
        assert ch.chamfer_default_samples(n_a, eps) == orc.default_samples(n_a, eps)
    assert ch.chamfer_default_samples(10, 0.0) == -1
    assert ch.chamfer_default_scales(10, 10, 1.0) == -1


@pytest.mark.parametrize("d,ke,seed", [(16, 32, 7), (128, 32, 42), (3, 8, 1), (256, 64, 2**40 + 3)])
def test_embedding_matrix_bit_exact(orc, d, ke, seed):
    """The library's host-drawn embedding equals the oracle's, bit for bit."""
    z = ch.chamfer_embedding_matrix(seed, d, ke)
    ref = orc.embedding(seed, d, ke)
    assert z.dtype == np.int8 and np.array_equal(z, ref)


def test_embedding_rejects_bad_dims():
    with pytest.raises(ch.ChamferError):
        ch.chamfer_embedding_matrix(1, 16, 12)
    with pytest.raises(ch.ChamferError):
        ch.chamfer_embedding_matrix(1, 0, 32)


def test_workspace_bytes():
    full = ch.chamfer_workspace_bytes(100000, 100000, 128, 2, 0.1, 2000)
    exact_only = ch.chamfer_workspace_bytes(100000, 100000, 128, 2, 0.0, 0)
    assert full > exact_only > 0
    # per-scale tables: L = 20 scales of 2^18 16-byte buckets dominate
    assert full >= 20 * (1 << 18) * 16
    assert ch.chamfer_workspace_bytes(10, 0, 3, 2, 0.1, 0) == 0      # empty B
    assert ch.chamfer_workspace_bytes(10, 10, 0, 2, 0.1, 0) == 0     # d = 0
    assert ch.chamfer_workspace_bytes(10, 10, 3, 3, 0.1, 0) == 0     # bad metric
    assert ch.chamfer_workspace_bytes(10, 10, 3, 2, 0.1, 0, embed_dim=12) == 0
    assert ch.chamfer_workspace_bytes(10, 10, 3, 2, 0.1, 0, n_scales=65) == 0


def _raw_estimate(lib, n_a=10, n_b=10, d=3, metric=2, eps=0.1, T=0, ws_bytes=1 << 20, opts=None):
    dummy = ctypes.c_void_p(16)   # never dereferenced: the call must fail first
    eta = ctypes.c_void_p(16)
    return lib.chamfer_estimate(dummy, dummy, n_a, n_b, d, metric, eps, T, 1, eta, None,
                                opts, ctypes.c_void_p(256) if ws_bytes else None, ws_bytes, None)


def test_argument_errors_are_host_side():
    """Invalid arguments return EINVAL/EWORKSPACE before anything is
    launched (these calls run without a GPU)."""
    lib = ch.lib()
    assert _raw_estimate(lib, d=0) == -1
    assert _raw_estimate(lib, metric=3) == -1
    assert _raw_estimate(lib, n_b=0) == -1
    assert _raw_estimate(lib, n_a=-1) == -1
    assert _raw_estimate(lib, eps=0.0) == -1
    assert _raw_estimate(lib, eps=1.0) == -1
    assert _raw_estimate(lib, T=-5) == -1
    assert _raw_estimate(lib, ws_bytes=0) == -2
    assert _raw_estimate(lib, ws_bytes=64) == -2
    for bad in (ch.Opts(0, 12, 0, 0, 0, 0, 0), ch.Opts(0, 0, 7, 0, 0, 0, 0),
                ch.Opts(0, 0, 0, 33, 0, 0, 0), ch.Opts(0, 0, 0, -1, 0, 0, 0),
                ch.Opts(0, 0, 0, 0, 65, 0, 0), ch.Opts(0, 0, 0, 0, 0, 2, 0),
                ch.Opts(0, 0, 0, 0, 0, 0, 3), ch.Opts(0, 0, 0, 0, 0, 0, -1)):
        assert _raw_estimate(lib, opts=ctypes.byref(bad)) == -1
    # CrudeNN needs its tables: uniform sampling is an estimator option only
    uni = ch.Opts(0, 0, 0, 0, 0, 1, 0)
    dummy = ctypes.c_void_p(16)
    assert lib.crude_nn(dummy, dummy, 5, 5, 3, 2, 0.5, 0, dummy, dummy, None, ctypes.byref(uni),
                        dummy, 1 << 30, None) == -1
    # symmetric forms need both sets non-empty and a workspace for both directions
    out = ctypes.c_void_p(64)
    assert lib.chamfer_estimate_symmetric(dummy, dummy, 0, 5, 3, 2, 0.5, 0, 1, out, None, dummy,
                                          1 << 30, None) == -1
    assert lib.chamfer_exact_symmetric(dummy, dummy, 5, 0, 3, 2, out, None, dummy, 1 << 30,
                                       None) == -1
    small = min(lib.chamfer_workspace_bytes(10, 1000, 3, 2, 0.5, 0, None),
                lib.chamfer_workspace_bytes(1000, 10, 3, 2, 0.5, 0, None))
    assert lib.chamfer_estimate_symmetric(dummy, dummy, 10, 1000, 3, 2, 0.5, 0, 1, out, None,
                                          dummy, small, None) == -2
    dummy = ctypes.c_void_p(16)
    assert lib.chamfer_exact(dummy, dummy, 5, 0, 3, 2, dummy, None, None, None, dummy, 1 << 20,
                             None) == -1
    assert lib.crude_nn(dummy, dummy, 5, 5, 3, 2, 1.5, 0, dummy, dummy, None, None, dummy,
                        1 << 20, None) == -1
    assert lib.chamfer_nn_min(dummy, None, -1, dummy, 5, 3, 2, None, None, None, dummy, 1 << 20,
                              None) == -1


def orc_pad(n, d):
    """The padding-width rule written out (next of 16/32/64/128, else a
    multiple of 16, of d + 3 ceil(log2 n))."""
    dp = d + 3 * max(1, (n - 1).bit_length())
    nxt = [w for w in (16, 32, 64, 128) if w >= dp]
    return (nxt[0] if nxt else -(-dp // 16) * 16) - d


def test_reduction_argument_errors_are_host_side():
    """The reduction: pad dimension rule, workspace sizes, and argument
    errors before any device work; the other entry points reject it."""
    lib = ch.lib()
    # at least 3 ceil(log2 n), d + m on a width the exact pass specialises
    assert lib.chamfer_pad_dims(1, 1, 1) == 15 and lib.chamfer_pad_dims(1000, 5, 3) == 61
    assert lib.chamfer_pad_dims(1 << 20, 7, 64) == 64 and lib.chamfer_pad_dims(1 << 20, 7, 100) == 60
    assert lib.chamfer_pad_dims(3, (1 << 20) + 1, 128) == 64 and lib.chamfer_pad_dims(5, 5, 0) == -1
    for n in (2, 100, 10 ** 6):
        for d in (1, 3, 16, 37, 64, 100, 128, 129, 300, 2000):
            m = lib.chamfer_pad_dims(n, n, d)
            assert m == orc_pad(n, d) and m >= 3 * max(1, (n - 1).bit_length())
    assert lib.chamfer_reduce_workspace_bytes(100, 200, 3, 1, None) > 0
    assert lib.chamfer_reduce_workspace_bytes(0, 200, 3, 1, None) == 0
    assert lib.chamfer_reduce_workspace_bytes(100, 200, 3, 3, None) == 0
    assert lib.chamfer_reduce_workspace_bytes(100, 200, 4096, 1, None) == 0
    part, padded = ch._opts(reduction=1), ch._opts(reduction=2)
    plain = lib.chamfer_workspace_bytes(1000, 2000, 16, 2, 0.2, 0, None)
    red = lib.chamfer_workspace_bytes(1000, 2000, 16, 2, 0.2, 0, ctypes.byref(part))
    pad = lib.chamfer_workspace_bytes(1000, 2000, 16, 2, 0.2, 0, ctypes.byref(padded))
    assert plain < red < pad
    # d + m must stay within 2048 for the padded estimate
    assert lib.chamfer_workspace_bytes(1000, 1000, 2040, 1, 0.2, 0, ctypes.byref(padded)) == 0
    assert lib.chamfer_workspace_bytes(1000, 1000, 2040, 1, 0.2, 0, ctypes.byref(part)) > 0
    dummy = ctypes.c_void_p(256)
    aux = ch.Aux()
    out = ctypes.c_void_p(64)
    # aux outputs are not available with the reduction
    assert lib.chamfer_estimate(dummy, dummy, 10, 10, 3, 2, 0.2, 0, 1, out, ctypes.byref(aux),
                                ctypes.byref(part), dummy, 1 << 40, None) == -1
    assert lib.chamfer_estimate(dummy, dummy, 10, 10, 3, 2, 0.2, 0, 1, out, None,
                                ctypes.byref(part), dummy, red // 1000, None) == -2
    assert lib.chamfer_estimate(dummy, dummy, 10, 10, 3, 2, 1.5, 0, 1, out, None,
                                ctypes.byref(part), dummy, 1 << 40, None) == -1
    # chamfer_aspect_reduce
    rb = lib.chamfer_reduce_workspace_bytes(10, 10, 3, 2, None)
    call = lambda **k: lib.chamfer_aspect_reduce(
        k.get("A", dummy), dummy, k.get("n_a", 10), 10, 3, 2, k.get("eps", 0.2), 1, None, None,
        None, None, None, None, None, dummy, k.get("ws", rb - 1), None)
    assert call(n_a=0) == -1 and call(A=None) == -1 and call(eps=0.0) == -1
    assert call() == -2
    # every other entry point rejects a reduction
    assert lib.crude_nn(dummy, dummy, 5, 5, 3, 2, 0.5, 0, dummy, dummy, None, ctypes.byref(part),
                        dummy, 1 << 30, None) == -1
    assert lib.chamfer_exact(dummy, dummy, 5, 5, 3, 2, dummy, None, None, ctypes.byref(part),
                             dummy, 1 << 30, None) == -1


def test_retrieve_argument_errors_are_host_side():
    """Retrieval rejects bad collections, k, options and workspaces before
    any device work (no GPU here: a launch would fail with EHIP)."""
    import numpy as np
    lib = ch.lib()
    dummy = ctypes.c_void_p(256)
    top = np.zeros(8, np.int32)
    vals = np.zeros(8, np.float64)

    def offs(*o):
        return np.array(o, np.int64)

    def size(o, m=None, n_a=10, d=3, metric=2, opts=None):
        return lib.chamfer_retrieve_workspace_bytes(n_a, o.ctypes.data, len(o) - 1 if m is None
                                                    else m, d, metric, 0.2, 0,
                                                    None if opts is None else ctypes.byref(opts))

    def call(o, k=1, m=None, ws_bytes=None, n_a=10, d=3, opts=None, A=dummy):
        m = len(o) - 1 if m is None else m
        if ws_bytes is None:
            ws_bytes = 1 << 40
        return lib.chamfer_retrieve(A, n_a, dummy, o.ctypes.data, m, d, 2, 0.2, 0, 1, k, opts,
                                    None, top.ctypes.data, vals.ctypes.data, dummy, ws_bytes, None)

    good = offs(0, 5, 9, 30)
    assert size(good) > 0
    assert size(good, n_a=0) == 0
    assert size(offs(0, 5, 5, 9)) == 0          # empty cloud
    assert size(offs(1, 5, 9)) == 0             # offsets[0] != 0
    assert size(good, m=0) == 0
    assert size(good, d=4096) == 0
    assert size(good, opts=ch._opts(0, 0, 0, window=4)) == 0
    assert size(good, opts=ch._opts(0, 0, 0, sampling=ch.UNIFORM)) == 0
    # the slots are sized for the largest cloud in either direction
    assert size(offs(0, 5, 9, 3000)) > size(offs(0, 5, 9, 30))
    assert call(good, k=0) == -1
    assert call(good, k=4) == -1                # k > m
    assert call(offs(0, 5, 5, 9)) == -1
    assert call(good, A=None) == -1
    assert call(good, ws_bytes=size(good) - 1) == -2


def test_server_argument_errors_are_host_side():
    lib = ch.lib()
    h = ctypes.c_void_p()
    assert lib.chamfer_server_create(1 << 20, 0, ctypes.byref(h)) == -1
    assert lib.chamfer_server_create(1 << 20, 1000, ctypes.byref(h)) == -1
    assert lib.chamfer_server_create(16, 4, ctypes.byref(h)) == -1
    assert lib.chamfer_server_submit(None, None, None) == -1
    assert lib.chamfer_server_warm(None, 3, 2, 0, 0) == -1
    assert lib.chamfer_server_progress(None) == -1
    assert lib.chamfer_server_destroy(None) == -1


def test_noalloc_checks_before_launch():
    """chamfer_estimate_noalloc refuses bad arguments and sizes beyond its
    static scratch array on the host, before it touches a device."""
    lib = ch.lib()
    n, d = 100_000, 128
    assert ch.chamfer_workspace_bytes(n, n, d, 2, 0.1) > 64 << 20
    rc = lib.chamfer_estimate_noalloc(None, None, n, n, d, 2, 0.1, 2000, 1, None, None, None,
                                      None)
    assert rc == -5
    assert b"static scratch" in lib.chamfer_strerror(-5)
    rc = lib.chamfer_estimate_noalloc(None, None, 10, 10, 0, 2, 0.1, 20, 1, None, None, None,
                                      None)
    assert rc == -1
    o = ch.Opts(reduction=1)
    rc = lib.chamfer_estimate_noalloc(None, None, 10, 10, 3, 2, 0.1, 20, 1, None, None,
                                      ctypes.byref(o), None)
    assert rc == -1
