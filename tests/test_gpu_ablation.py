"""The distribution-cost ablation's generator modes (through the C-ABI).

The integer-scaled (-1,1) mode and the stored-S product compute the same
A_hat as the product path, bit for bit (the same sums in the same order; the
scaled mode's S differs by the exact factor 2^24); the junk generator runs
the same kernel with a cheap, non-random hash; the generator-throughput probe
folds exactly the generator's words.
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


def _run(B, A, d, dist, seed, tune):
    import torch
    dA = B.DeviceCsc.from_host(A)
    ws = B.alloc_workspace(B.workspace_bytes(dA, d, dist, tune=tune))
    out = torch.empty((A.n, d), dtype=torch.float32, device="cuda")
    B.sketch_into(dA, d, dist, seed, out, ws, tune=tune)
    torch.cuda.synchronize()
    return dA, ws, out


@pytest.mark.parametrize("variant,shape", [(3, (30_000, 900, 60_000, 300)),
                                           (6, (20_000, 150, 30_000, 203)),
                                           (9, (30_000, 900, 60_000, 300))])
def test_scaled_and_stored_equal_product(B, oracle_lib, variant, shape):
    import torch
    m, n, nnz, d = shape
    A = inputs.uniform_positions(m, n, nnz, 17, "uniform", np.float32)
    base = {"variant": variant, "dense_min_pct": 101, "col_split": 1}
    print(f"ablation modes, variant {variant}", flush=True)
    dA, ws, ref = _run(B, A, d, "uniform", 21, base)
    _, _, scaled = _run(B, A, d, "uniform", 21, dict(base, rng_mode=3))
    assert torch.equal(ref, scaled)
    # stored S: materialise S (d x m, leading dimension a multiple of 128)
    lds = -(-d // 128) * 128
    S = torch.zeros((m, lds), dtype=torch.float32, device="cuda")
    B.lib().sk_materialize_s(0, d, 0, m, 1, 21, S.data_ptr(), lds,
                             B._stream(None))
    out = torch.empty_like(ref)
    B.sketch_stored_into(dA, S, out, ws, tune=base)
    torch.cuda.synchronize()
    assert torch.equal(ref, out)
    got = ref.t().cpu().numpy().astype(np.float64)
    o = oracle_lib.sketch(A.m, A.n, A.colptr, A.rowidx, A.vals.astype(np.float64), d,
                          "uniform", 21)
    p = oracle_lib.parity(got, o, A.colptr, A.vals, "uniform")
    assert p["normwise"] <= 1e-5 and p["max_elem_scaled"] <= oracle_lib.ELEM_TOL, p


@pytest.mark.parametrize("dist", ["rademacher", "uniform", "gaussian"])
def test_junk_generator_runs(B, dist):
    import torch
    A = inputs.uniform_positions(20_000, 900, 40_000, 5, "uniform", np.float32)
    tune = {"variant": 3, "dense_min_pct": 101, "rng_mode": 1}
    print(f"junk generator {dist}", flush=True)
    _, _, a = _run(B, A, 256, dist, 3, tune)
    _, _, b = _run(B, A, 256, dist, 3, tune)
    assert torch.isfinite(a).all() and torch.equal(a, b)
    _, _, p = _run(B, A, 256, dist, 3, dict(tune, rng_mode=0))
    assert not torch.equal(a, p)


def test_ablation_modes_refused_where_absent(B):
    import torch
    A = inputs.uniform_positions(5_000, 40, 3_000, 1, "uniform", np.float32)
    dA = B.DeviceCsc.from_host(A)
    out = torch.empty((40, 64), dtype=torch.float32, device="cuda")
    ws = B.alloc_workspace(B.workspace_bytes(dA, 64, "gaussian"))
    with pytest.raises(B.SketchError):  # the scaled mode is (-1,1) only
        B.sketch_into(dA, 64, "gaussian", 1, out, ws, tune={"variant": 3, "rng_mode": 3})
    with pytest.raises(B.SketchError):  # no ablation form of this shape
        B.sketch_into(dA, 64, "gaussian", 1, out, ws, tune={"variant": 1, "rng_mode": 1})


def test_throughput_probe_folds_generator_words(B, oracle_lib):
    import torch
    blocks, calls, seed = 2, 5, 0xABCDEF0123
    sink = torch.zeros(blocks * 256, dtype=torch.int32, device="cuda")
    B.rng_throughput("rademacher", 0, calls, blocks, seed, sink)
    got = sink.cpu().numpy().view(np.uint32)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    for t in (0, 1, 255, 300, 511):
        want = 0
        for c in range(calls):
            w = oracle_lib.philox((c, t, 0, 0), key)
            want ^= int(w[0] ^ w[1] ^ w[2] ^ w[3])
        assert int(got[t]) == want, t
    for dist in ("uniform", "gaussian"):
        for gen in (0, 1):
            B.rng_throughput(dist, gen, calls, blocks, seed, sink)
    torch.cuda.synchronize()
