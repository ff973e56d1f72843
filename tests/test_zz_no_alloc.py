"""chamfer_estimate_noalloc (the estimate on the library's static scratch
array, for callers that cannot allocate) against chamfer_estimate with a
caller workspace on the same inputs: the same kernels run on the same data,
so every output is identical -- bit-exact indices, crude distances and
sampled minima, and eta equal (within 1e-5 relative is the bar).  Two calls
in a row, the second smaller, show that the array's leftover contents from
the first call do not leak into the second; a size beyond the array is
refused before any launch."""

import math

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_03043_amd as lib
    lib.lib()
    return lib


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


FIELDS = ["sample_idx", "sample_min", "sample_nn", "W", "s", "status", "crude_D", "crude_nn",
          "crude_scale"]


def compare(ch, A, B, metric, eps, T, seed):
    print(f"[case] noalloc n_a={A.shape[0]} n_b={B.shape[0]} d={A.shape[1]} metric={metric} "
          f"eps={eps} T={T} seed={seed}", flush=True)
    At, Bt = dev(A), dev(B)
    got = ch.chamfer_estimate_noalloc(At, Bt, metric, eps, T, seed)
    torch.cuda.synchronize()
    got = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in got.items()}
    ref = ch.chamfer_estimate(At, Bt, metric, eps, T, seed)
    torch.cuda.synchronize()
    ref = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in ref.items()}
    assert int(got["status"][0]) == 0
    for f in FIELDS:
        assert np.array_equal(got[f].view(np.uint8), ref[f].view(np.uint8)), f
    eta, eta_ref = float(got["eta"][0]), float(ref["eta"][0])
    assert math.isclose(eta, eta_ref, rel_tol=1e-5), (eta, eta_ref)
    assert eta == eta_ref
    return eta


def test_noalloc_two_calls_second_smaller(ch):
    A, B = workloads.clusters_l2(seed=5, n=20_000, d=128, k=200)
    e1 = compare(ch, A, B, 2, 0.1, 2000, 11)
    A2, B2 = workloads.small_l2(seed=6, n=3001, d=16)
    e2 = compare(ch, A2, B2[:2500], 2, 0.2, 512, 12)
    assert e1 > 0 and e2 > 0
    # l1 after l2, smaller again, on a ragged size
    A3 = workloads.uniform_cube(7, 777, 1201, 5)
    compare(ch, A3[0], A3[1], 1, 0.2, 300, 13)


def test_noalloc_refuses_too_large(ch):
    n, d = 100_000, 128
    need = ch.chamfer_workspace_bytes(n, n, d, 2, 0.1)
    assert need > 64 << 20
    A = torch.zeros((n, d), dtype=torch.float32, device="cuda:0")
    with pytest.raises(ch.ChamferError) as ei:
        ch.chamfer_estimate_noalloc(A, A, 2, 0.1, 2000, 1)
    assert ei.value.status == -5
    # the library still works after the refusal
    A2, B2 = workloads.small_l2(seed=8, n=1500, d=16)
    compare(ch, A2, B2, 2, 0.2, 256, 14)
