"""Pins of the oracle's random sources and sketches against independent
definitions (not against the oracle itself)."""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

from conftest import read_golden
from oracle import hashes, sketches


def test_philox_known_answers():
    for row in read_golden("philox4x32_10_kat.txt"):
        vals = [int(t, 16) for t in row]
        ctr = np.array([vals[0:4]], dtype=np.uint32)
        out = hashes.philox4x32_10(ctr, (vals[4], vals[5]))[0]
        assert [int(v) for v in out] == vals[6:10]


def test_murmur3_matches_sklearn():
    from sklearn.utils import murmurhash3_32  # independent implementation
    rng = np.random.default_rng(5)
    keys = np.concatenate([np.arange(0, 300), rng.integers(0, 2**31 - 1, size=700)])
    for seed in (0, 1, 7, 0x9E3779B9 + 8, 2**32 - 1):
        ours = hashes.murmur3_32(keys, seed)
        ref = np.array([murmurhash3_32(int(k), seed & 0xFFFFFFFF, positive=True) for k in keys],
                       dtype=np.uint64).astype(np.uint32)
        assert np.array_equal(ours, ref)


def test_murmur3_high_keys_match_sklearn_int32_view():
    from sklearn.utils import murmurhash3_32
    keys = np.array([2**31, 2**31 + 5, 2**32 - 1, 3_000_000_000], dtype=np.uint64)
    ours = hashes.murmur3_32(keys, 11)
    # sklearn takes the same 4 bytes as a signed int32
    ref = [murmurhash3_32(int(np.uint32(k).view(np.int32)), 11, positive=True) for k in keys]
    assert [int(v) for v in ours] == ref


def test_box_muller_is_standard_normal():
    z = hashes.gaussian_entries(123, 0, np.arange(400_000))
    assert abs(z.mean()) < 5 / math.sqrt(len(z))
    assert abs(z.var() - 1.0) < 0.02
    ks = scipy.stats.kstest(z[:100_000], "norm")
    assert ks.pvalue > 1e-3
    # lanes of one Philox block are distinct and streams differ
    assert len(np.unique(hashes.gaussian_entries(1, 0, np.arange(8)))) == 8
    assert not np.allclose(hashes.gaussian_entries(1, 0, np.arange(8)),
                           hashes.gaussian_entries(1, 1, np.arange(8)))


def test_fwht_equals_sylvester_hadamard():
    rng = np.random.default_rng(0)
    for n in (1, 2, 8, 64, 1024):
        X = rng.standard_normal((n, 3))
        H = scipy.linalg.hadamard(n).astype(np.float64)  # Sylvester construction
        assert np.allclose(sketches.fwht_rows(X), H @ X, atol=1e-11 * n)
        assert np.allclose(H.T @ H, n * np.eye(n))
    k = np.arange(64)[:, None]
    i = np.arange(64)[None, :]
    assert np.array_equal(sketches.hadamard_entry(k, i), scipy.linalg.hadamard(64))


def test_srht_dense_definition_and_isometry():
    rng = np.random.default_rng(1)
    n, d, m, seed = 256, 5, 32, 17
    A = rng.standard_normal((n, d))
    H = scipy.linalg.hadamard(n).astype(np.float64)
    D = sketches.srht_signs(n, seed)
    rows = sketches.srht_rows(m, n, seed)
    S = H[rows] * D[None, :] / math.sqrt(m)
    assert np.allclose(sketches.srht_sketch(A, m, seed), S @ A, atol=1e-12)
    for k in (0, 7, m - 1):
        assert np.allclose(sketches.srht_entry(A, m, seed, k, [0, 3]), (S @ A)[k, [0, 3]])
    # E[S^T S] = I: averaging the rank-one term over every possible sampled row is exact
    HD = H * D[None, :]
    assert np.allclose(HD.T @ HD / n, np.eye(n))
    # signs and samples: bit 31 of the hash, low bits of the shifted-seed hash
    h = hashes.murmur3_32(np.arange(n), seed)
    assert np.array_equal(D < 0, (h >> 31) == 1)
    hp = hashes.murmur3_32(np.arange(m), (seed + 0x9E3779B9) & 0xFFFFFFFF)
    assert np.array_equal(rows, hp & (n - 1))


def test_countsketch_brute_force():
    rng = np.random.default_rng(2)
    n, d, m, seed = 300, 4, 16, 9
    A = rng.standard_normal((n, d))
    S = np.zeros((m, n))
    for i in range(n):  # one nonzero per column, written out entry by entry
        h = int(hashes.murmur3_32(np.array([i]), seed)[0])
        S[h % m, i] = -1.0 if h >> 31 else 1.0
    assert np.array_equal(S, sketches.countsketch_matrix(n, m, seed))
    assert np.allclose(sketches.countsketch(A, m, seed), S @ A, atol=1e-13)
    assert np.array_equal(np.diag(S.T @ S), np.ones(n))


def test_gaussian_sketch_is_matrix_product_and_isotropic():
    rng = np.random.default_rng(3)
    n, d, m = 200, 6, 40
    A = rng.standard_normal((n, d))
    S = sketches.gaussian_matrix(m, n, 21)
    assert np.allclose(sketches.gaussian_sketch(A, m, 21), S @ A, atol=1e-12)
    # E[S^T S] = I: diagonal mean 1 within Monte Carlo error, entries var 1/m
    G = S.T @ S
    assert abs(np.mean(np.diag(G)) - 1.0) < 0.05
    assert abs(S.var() * m - 1.0) < 0.05


def test_count_gauss_composition():
    rng = np.random.default_rng(4)
    n, d, m1, m2 = 512, 3, 64, 16
    A = rng.standard_normal((n, d))
    C = sketches.countsketch_matrix(n, m1, 5)
    G = sketches.gaussian_matrix(m2, m1, 5, stream=1)
    assert np.allclose(sketches.count_gauss_sketch(A, m1, m2, 5), G @ (C @ A), atol=1e-12)


def test_bf16_round_matches_torch_on_float32_inputs():
    """On float32-representable inputs torch's float32 -> bfloat16 conversion is a
    single round-to-nearest-even, so it pins the oracle's rounding."""
    import torch
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(200_000) * np.exp(rng.uniform(-30, 30, 200_000)))
    x = x.astype(np.float32).astype(np.float64)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).double().numpy()
    assert np.array_equal(sketches.bf16_round(x), ref)
    # ties go to even
    t = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8])
    assert np.array_equal(sketches.bf16_round(t), [1.0, 1.0 + 4 * 2.0 ** -8])
