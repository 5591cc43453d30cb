"""Pins for the oracle's generator and transforms (CPU only).

Philox4x32-10 is checked against PyTorch's independent header engine; the
word -> S-row mapping and the +-1 / (-1,1) transforms against those
independent words; the FP32 Gaussian against FP64 libm Box-Muller on the same
uniforms (which checks the polynomials, not only agreement).
"""
import numpy as np
import pytest

from tests import refgen


def test_philox_matches_independent_engine(oracle_lib):
    rng = np.random.default_rng(123)
    pairs = [((0, 0), (0, 0, 0, 0)),
             ((0xFFFFFFFF, 0xFFFFFFFF), (0xFFFFFFFF,) * 4),
             ((0xA4093822, 0x299F31D0), (0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344))]
    for _ in range(300):
        k = rng.integers(0, 2**32, size=2, dtype=np.uint64)
        c = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        pairs.append(((int(k[0]), int(k[1])), tuple(int(v) for v in c)))
    ref = refgen.torch_philox(pairs)
    got = np.array([oracle_lib.philox(c, k) for k, c in pairs], dtype=np.uint32)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("seed", [1, 0x1234_5678_9ABC_DEF0])
def test_rademacher_bits_map_to_rows(oracle_lib, seed):
    # rows 128g + 32w + b take bit b of word w; bit 0 -> +1, bit 1 -> -1
    j_list = [0, 5, 99_999, 2**31 - 1, 2**33 + 17]
    S = np.stack([oracle_lib.materialize_s("rademacher", seed, 0, 300, j, 1)[:, 0]
                  for j in j_list], axis=1)
    for c, j in enumerate(j_list):
        for g in range(3):
            x = refgen.words_for(seed, g, j)
            for w in range(4):
                for b in range(32):
                    i = 128 * g + 32 * w + b
                    if i >= 300:
                        continue
                    assert S[i, c] == (-1.0 if (x[w] >> b) & 1 else 1.0)


def test_uniform_words_and_exactness(oracle_lib):
    seed = 21
    d, cols = 64, 40
    j0 = 1_999_980
    S = oracle_lib.materialize_s("uniform", seed, 0, d, j0, cols)
    scaled = S * 2.0**24
    # exact odd integers strictly inside (-2^24, 2^24): open interval, FP32-exact
    assert np.all(scaled == np.round(scaled))
    assert np.all(np.abs(scaled) < 2**24)
    assert np.all(np.mod(scaled, 2) == 1)
    for c in range(cols):
        j = j0 + c
        for g in range(d // 4):
            x = refgen.words_for(seed, g, j).view(np.int32).astype(np.int64)
            expect = (2 * (x >> 8) + 1).astype(np.float64)
            assert np.array_equal(scaled[4 * g:4 * g + 4, c], expect)


def test_uniform_row0_offsets_consistent(oracle_lib):
    full = oracle_lib.materialize_s("uniform", 5, 0, 37, 10, 3)
    part = oracle_lib.materialize_s("uniform", 5, 13, 24, 10, 3)
    assert np.array_equal(full[13:], part)
    fullg = oracle_lib.materialize_s("gaussian", 5, 0, 37, 10, 3)
    partg = oracle_lib.materialize_s("gaussian", 5, 13, 24, 10, 3)
    assert np.array_equal(fullg[13:], partg)
    fullr = oracle_lib.materialize_s("rademacher", 5, 0, 300, 10, 3)
    partr = oracle_lib.materialize_s("rademacher", 5, 131, 169, 10, 3)
    assert np.array_equal(fullr[131:], partr)


def test_uniform_moments(oracle_lib):
    S = oracle_lib.materialize_s("uniform", 77, 0, 400, 0, 2500).ravel()
    n = S.size
    assert abs(S.mean()) < 5 * np.sqrt(1 / 3 / n)
    var = 1 / 3 - 1 / (3 * 2.0**48)
    # var of s^2 for U(-1,1) is 4/45
    assert abs(S.var() - var) < 5 * np.sqrt(4 / 45 / n)
    assert S.min() > -1.0 and S.max() < 1.0


def test_rademacher_balance(oracle_lib):
    S = oracle_lib.materialize_s("rademacher", 3, 0, 512, 0, 2000).ravel()
    assert set(np.unique(S)) == {-1.0, 1.0}
    assert abs(S.mean()) < 5 / np.sqrt(S.size)


def test_gaussian_against_fp64_box_muller(oracle_lib):
    rng = np.random.default_rng(5)
    xe = rng.integers(0, 2**32, size=200_000, dtype=np.uint64).astype(np.uint32)
    xo = rng.integers(0, 2**32, size=200_000, dtype=np.uint64).astype(np.uint32)
    # special words: u1 = 1 (r = 0), u1 = 2^-24 (largest r), quadrant edges, f near sqrt 2
    special_e = [0xFFFFFFFF, 0x000000FF, 0x00000000, 0x6A09E600, 0x6A09E700, 0x7FFFFF00,
                 0x80000000, 0x00000100, 0xB504F300]
    special_o = [0x00000000, 0x3FFFFF00, 0x40000000, 0x7FFFFFFF, 0x80000000, 0xBFFFFFFF,
                 0xC0000000, 0xFFFFFFFF, 0x12345678]
    xe = np.concatenate([xe, np.array(special_e, np.uint32)])
    xo = np.concatenate([xo, np.array(special_o, np.uint32)])
    z0, z1 = oracle_lib.gauss_words(xe, xo)
    r0, r1, r = refgen.box_muller_f64(xe, xo)
    tol = 2.0**-20 * np.maximum(r, 1.0)
    assert np.all(np.abs(z0.astype(np.float64) - r0) <= tol)
    assert np.all(np.abs(z1.astype(np.float64) - r1) <= tol)


def test_gaussian_words_map_to_rows(oracle_lib):
    seed, j = 31, 3_999_999
    S = oracle_lib.materialize_s("gaussian", seed, 0, 12, j, 1)[:, 0]
    for g in range(3):
        x = refgen.words_for(seed, g, j)
        z0, z1 = oracle_lib.gauss_words(x[[0, 2]], x[[1, 3]])
        assert S[4 * g] == z0[0] and S[4 * g + 1] == z1[0]
        assert S[4 * g + 2] == z0[1] and S[4 * g + 3] == z1[1]
        r0, r1, _ = refgen.box_muller_f64(x[[0, 2]], x[[1, 3]])
        assert np.allclose(S[4 * g:4 * g + 4], [r0[0], r1[0], r0[1], r1[1]], atol=1e-5)


def test_gaussian_moments_and_ks(oracle_lib):
    from scipy import stats
    S = oracle_lib.materialize_s("gaussian", 11, 0, 1000, 0, 10_000).ravel()
    n = S.size
    assert abs(S.mean()) < 5 / np.sqrt(n)
    assert abs(S.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    kurt = np.mean(S**4) / np.mean(S**2) ** 2
    assert abs(kurt - 3.0) < 5 * np.sqrt(96.0 / n)
    ks = stats.kstest(S[:2_000_000], "norm")
    assert ks.pvalue > 1e-6


def test_coefficient_tables_from_their_definition(oracle_lib):
    import math
    t = oracle_lib.tables()
    assert np.array_equal(t["log"], np.array([1 / 3, 1 / 5, 1 / 7, 1 / 9, 1 / 11], np.float32))
    h = math.pi / 2
    sin_ref = [(-1) ** k * h ** (2 * k + 1) / math.factorial(2 * k + 1) for k in range(7)]
    cos_ref = [(-1) ** k * h ** (2 * k) / math.factorial(2 * k) for k in range(8)]
    assert np.array_equal(t["sin"], np.array(sin_ref, np.float32))
    assert np.array_equal(t["cos"], np.array(cos_ref, np.float32))
    hi, lo, s2 = t["misc"]
    assert float(hi) == 22713 / 32768 and abs(float(hi) + float(lo) - math.log(2)) < 1e-12
    assert s2 == np.float32(math.sqrt(2))


@pytest.mark.parametrize("seed", [31, 0xFEDC_BA98_7654_3210])
def test_s_entry_against_independent_words(oracle_lib, seed):
    # S(i, j) one entry at a time, pinned on words from the independent engine:
    # +-1 and (-1,1) exactly, the Gaussian against FP64 libm Box-Muller
    cases = [(0, 0), (127, 3), (128, 3), (255, 2**31 - 1), (4001, 2**31 + 5), (9, 2**40 + 1)]
    for i, j in cases:
        x = refgen.words_for(seed, i // 128, j)
        b = (int(x[(i % 128) // 32]) >> (i % 32)) & 1
        assert oracle_lib.s_entry("rademacher", seed, i, j) == (-1.0 if b else 1.0)
        x = refgen.words_for(seed, i // 4, j)
        t = int(np.int32(np.uint32(x[i % 4]))) >> 8
        assert oracle_lib.s_entry("uniform", seed, i, j) == (2 * t + 1) * 2.0**-24
        pair = (x[0], x[1]) if i % 4 < 2 else (x[2], x[3])
        z0, z1, r = refgen.box_muller_f64(np.array([pair[0]], np.uint32),
                                          np.array([pair[1]], np.uint32))
        z = (z0 if i % 2 == 0 else z1)[0]
        got = oracle_lib.s_entry("gaussian", seed, i, j)
        assert abs(got - z) <= 2.0**-20 * max(r[0], 1.0), (i, j, got, z)


@pytest.mark.gpu
@pytest.mark.parametrize("seed", [0, 1, 0x0123456789ABCDEF, 0xFFFFFFFFFFFFFFFF])
@pytest.mark.parametrize("offset_calls", [0, 12345, (1 << 32) - 3])
def test_philox_against_rocrand(oracle_lib, seed, offset_calls):
    """A second independent Philox4x32-10: rocRAND's host generator (it needs
    the HIP runtime, hence a device).  Its output 4k + w is word w of the
    block function at counter (k_lo, k_hi, 0, 0) with key (seed_lo, seed_hi);
    an offset of 4 (2^32 - 3) calls crosses the carry into the second counter
    word."""
    import ctypes
    import torch
    assert torch.cuda.is_available(), "the HIP runtime needs a device"
    try:
        L = ctypes.CDLL("/opt/rocm/lib/librocrand.so")
    except OSError:
        pytest.skip("rocRAND is not installed")
    gen = ctypes.c_void_p()
    assert L.rocrand_create_generator_host_blocking(ctypes.byref(gen), 404) == 0  # PHILOX4_32_10
    try:
        assert L.rocrand_set_seed(gen, ctypes.c_ulonglong(seed)) == 0
        assert L.rocrand_set_offset(gen, ctypes.c_ulonglong(4 * offset_calls)) == 0
        n = 4 * 1024
        out = np.zeros(n, dtype=np.uint32)
        assert L.rocrand_generate(gen, out.ctypes.data_as(ctypes.c_void_p), ctypes.c_size_t(n)) == 0
    finally:
        L.rocrand_destroy_generator(gen)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    for k in range(1024):
        c = offset_calls + k
        want = oracle_lib.philox((c & 0xFFFFFFFF, c >> 32, 0, 0), key)
        assert [int(x) for x in out[4 * k:4 * k + 4]] == [int(x) for x in want], k
