"""The allocation-free entry point sk_sketch_noalloc against sk_sketch.

sk_sketch_noalloc runs the same plan and kernels as sk_sketch with the
library's fixed per-device array as the workspace, so its A_hat must be
bitwise the one sk_sketch writes with a caller-owned workspace.  Two calls
in a row, the second on a smaller input, check that nothing a call leaves in
the shared array leaks into the next one.
"""
import numpy as np
import pytest

from paper_2310_15419_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    from paper_2310_15419_amd import binding
    binding.lib()
    return binding


CASES = [
    # (m, n, nnz, d, dist, seed, values): the first is the larger call
    (60_000, 300, 90_000, 600, "uniform", 11, "uniform"),
    (5_000, 40, 6_000, 100, "gaussian", 12, "normal"),
]


def _pair(B, A, d, dist, seed, prec=0, tune=None):
    import torch
    dA = B.DeviceCsc.from_host(A, dtype=np.float32 if A.vals.dtype != np.float64 else None)
    # (n, d) row-major: column-major A_hat with ld = d, like `out`
    ref = B.sketch(dA, d, dist, seed, prec=prec, tune=tune).t().contiguous()
    out = torch.full((A.n, d), float("nan"), dtype=torch.float32, device="cuda")
    B.sketch_noalloc_into(dA, d, dist, seed, out, prec=prec, tune=tune)
    torch.cuda.synchronize()
    ref, got = ref.cpu().numpy(), out.cpu().numpy()
    assert ref.shape == got.shape == (A.n, d)
    return ref, got


def test_noalloc_bitwise_equal_to_sketch_two_calls(B, oracle_lib):
    for (m, n, nnz, d, dist, seed, vals) in CASES:
        print(f"noalloc m={m} n={n} d={d} {dist}", flush=True)
        A = inputs.uniform_positions(m, n, nnz, seed, vals, np.float32)
        ref, got = _pair(B, A, d, dist, seed)
        assert np.array_equal(ref.view(np.uint32), got.view(np.uint32))
        # and the oracle's bar for the FP32 path
        o = oracle_lib.sketch(A.m, A.n, A.colptr, A.rowidx, A.vals.astype(np.float64), d, dist,
                              seed)
        err = np.linalg.norm(got.T.astype(np.float64) - o) / np.linalg.norm(o)
        assert err <= 1e-5, err


def test_noalloc_matrix_core_path_then_smaller(B):
    # +-1 S in BF16 on the matrix cores, then a smaller sparse call
    A = inputs.uniform_positions(4000, 150, 30_000, 9, "uniform", np.float32)
    print("noalloc bf16 matrix cores", flush=True)
    ref, got = _pair(B, A, 300, "rademacher", 5, prec=B.PREC_BF16, tune={"dense_min_pct": 1})
    assert np.array_equal(ref.view(np.uint32), got.view(np.uint32))
    A2 = inputs.uniform_positions(900, 30, 1500, 3, "uniform", np.float32)
    print("noalloc small rademacher", flush=True)
    ref, got = _pair(B, A2, 64, "rademacher", 6)
    assert np.array_equal(ref.view(np.uint32), got.view(np.uint32))


def test_noalloc_rejects_oversize(B):
    import torch
    from paper_2310_15419_amd.binding import SketchError
    # 64 MiB cannot hold the workspace of this shape: refused on the host
    # before any device work
    m, n = 2_000_000, 2000
    A = B.DeviceCsc(m, n, torch.zeros(n + 1, dtype=torch.int64, device="cuda"),
                    torch.zeros(20_000_000, dtype=torch.int32, device="cuda"),
                    torch.zeros(20_000_000, dtype=torch.float32, device="cuda"))
    out = torch.empty((n, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(SketchError) as e:
        B.sketch_noalloc_into(A, 16, "uniform", 1, out)
    assert e.value.code == -4
