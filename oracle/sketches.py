"""Oracle: the three sketch families of Lemma 3, written out densely or row by row.

TEST INFRASTRUCTURE ONLY (CPU, numpy float64); the product path never imports it.

All sketches satisfy E[S^T S] = I_n (Section 3.1 states it with a subscript m,
read here as n since S is m x n), so:

* Gaussian (Lemma 3(iv), sub-Gaussian):  S_ij = z_ij / sqrt(m), z_ij ~ N(0,1);
* SRHT (Lemma 3(iii)):  S = (1/sqrt(m)) P H D with D = diag(+-1), H the
  unnormalised Sylvester Walsh-Hadamard matrix (H[k,i] = (-1)^popcount(k & i),
  n a power of two) and P picking m rows uniformly *with replacement*;
* CountSketch (Lemma 3(i), one nonzero per column):  column i of S has a single
  +-1 in row h(i); no scaling.

Random choices come from the counter-based generators in `oracle.hashes`:

* SRHT: D_ii = -1 iff bit 31 of murmur3(i, seed) is set; sampled row k is
  murmur3(k, seed + 0x9E3779B9 mod 2^32) & (n - 1);
* CountSketch: h = murmur3(i, seed); bucket h mod m; sign -1 iff bit 31 of h;
* Gaussian: z_ij = gaussian_entries(seed, stream, i * n + j).
"""
from __future__ import annotations

import math

import numpy as np

from .hashes import gaussian_entries, murmur3_32

SRHT_SAMPLE_SEED_OFFSET = 0x9E3779B9


# ----------------------------------------------------------------------------
# Gaussian (Lemma 3(iv))
# ----------------------------------------------------------------------------
def gaussian_matrix(m: int, n: int, seed: int, stream: int = 0) -> np.ndarray:
    """Dense S (m x n) with entries N(0, 1/m)."""
    idx = np.arange(m * n, dtype=np.int64)
    return (gaussian_entries(seed, stream, idx) / math.sqrt(m)).reshape(m, n)


def gaussian_sketch(A: np.ndarray, m: int, seed: int, stream: int = 0) -> np.ndarray:
    n = A.shape[0]
    out = np.zeros((m, A.shape[1]), dtype=np.float64)
    A64 = A.astype(np.float64, copy=False)
    # row blocks of S to bound memory; S itself is a plain matrix product
    blk = max(1, (1 << 24) // max(n, 1))
    for i0 in range(0, m, blk):
        i1 = min(m, i0 + blk)
        idx = (np.arange(i0, i1, dtype=np.int64)[:, None] * n + np.arange(n, dtype=np.int64)[None, :])
        S = gaussian_entries(seed, stream, idx) / math.sqrt(m)
        out[i0:i1] = S @ A64
    return out


# ----------------------------------------------------------------------------
# SRHT (Lemma 3(iii))
# ----------------------------------------------------------------------------
def srht_signs(n: int, seed: int) -> np.ndarray:
    h = murmur3_32(np.arange(n, dtype=np.uint64), seed)
    return np.where((h >> np.uint32(31)) != 0, -1.0, 1.0)


def rademacher_probes(d: int, T: int, seed: int) -> np.ndarray:
    """Algorithm 5's probe vectors v^1..v^T in {-1, +1}^d as a d x T matrix:
    entry (j, l) is -1 iff bit 31 of murmur3(l * d + j, seed) is set (the same
    counter-based rule as the SRHT signs)."""
    idx = (np.arange(T, dtype=np.uint64)[None, :] * np.uint64(d)
           + np.arange(d, dtype=np.uint64)[:, None])
    h = murmur3_32(idx.ravel(), seed).reshape(d, T)
    return np.where((h >> np.uint32(31)) != 0, -1.0, 1.0)


def srht_rows(m: int, n: int, seed: int) -> np.ndarray:
    if n & (n - 1):
        raise ValueError("SRHT needs n to be a power of two")
    h = murmur3_32(np.arange(m, dtype=np.uint64), (seed + SRHT_SAMPLE_SEED_OFFSET) & 0xFFFFFFFF)
    return (h & np.uint32(n - 1)).astype(np.int64)


def hadamard_entry(k: np.ndarray, i: np.ndarray) -> np.ndarray:
    """Sylvester Walsh-Hadamard entry (-1)^popcount(k & i)."""
    v = np.bitwise_and(np.asarray(k, dtype=np.int64), np.asarray(i, dtype=np.int64))
    par = np.zeros(v.shape, dtype=np.int64)
    while np.any(v):
        par ^= v & 1
        v = v >> 1
    return 1.0 - 2.0 * par


def fwht_rows(X: np.ndarray) -> np.ndarray:
    """Unnormalised fast Walsh-Hadamard transform along axis 0 (Sylvester order), radix 2."""
    Y = np.array(X, dtype=np.float64, copy=True)
    n = Y.shape[0]
    if n & (n - 1):
        raise ValueError("length must be a power of two")
    h = 1
    while h < n:
        Y = Y.reshape(n // (2 * h), 2, h, *Y.shape[1:])
        a = Y[:, 0].copy()
        b = Y[:, 1]
        Y[:, 0] = a + b
        Y[:, 1] = a - b
        Y = Y.reshape(n, *Y.shape[3:])
        h *= 2
    return Y


def srht_sketch(A: np.ndarray, m: int, seed: int) -> np.ndarray:
    """SA = (1/sqrt(m)) P H D A via a full FWHT (small n only)."""
    n = A.shape[0]
    D = srht_signs(n, seed)
    Y = fwht_rows(D[:, None] * A.astype(np.float64))
    return Y[srht_rows(m, n, seed)] / math.sqrt(m)


def srht_entry(A: np.ndarray, m: int, seed: int, k: int, cols) -> np.ndarray:
    """One sampled output row SA[k, cols], summed directly over all n rows (O(n) per entry)."""
    n = A.shape[0]
    idx = int(srht_rows(m, n, seed)[k])
    D = srht_signs(n, seed)
    Hrow = hadamard_entry(np.full(n, idx), np.arange(n))
    w = Hrow * D
    return (w @ A[:, cols].astype(np.float64)) / math.sqrt(m)


# ----------------------------------------------------------------------------
# CountSketch (Lemma 3(i))
# ----------------------------------------------------------------------------
def countsketch_hash(n: int, m: int, seed: int):
    h = murmur3_32(np.arange(n, dtype=np.uint64), seed)
    bucket = (h % np.uint32(m)).astype(np.int64)
    sign = np.where((h >> np.uint32(31)) != 0, -1.0, 1.0)
    return bucket, sign


def countsketch_matrix(n: int, m: int, seed: int) -> np.ndarray:
    bucket, sign = countsketch_hash(n, m, seed)
    S = np.zeros((m, n))
    S[bucket, np.arange(n)] = sign
    return S


def countsketch(A: np.ndarray, m: int, seed: int) -> np.ndarray:
    """CA[h(i)] += s(i) A[i], rows taken in ascending i."""
    bucket, sign = countsketch_hash(A.shape[0], m, seed)
    out = np.zeros((m, A.shape[1]), dtype=np.float64)
    np.add.at(out, bucket, sign[:, None] * A.astype(np.float64))
    return out


def count_gauss_sketch(A: np.ndarray, m1: int, m2: int, seed: int) -> np.ndarray:
    """Two-stage sketch G (C A): CountSketch to m1 rows, then a Gaussian m2 x m1
    (Philox stream 1).  E[(GC)^T (GC)] = E[C^T E[G^T G] C] = I."""
    CA = countsketch(A, m1, seed)
    return gaussian_sketch(CA, m2, seed, stream=1)


# ----------------------------------------------------------------------------
# Mixed-precision reading of the Gaussian stage: S and A rounded to BF16
# (round to nearest, ties to even, of the exact value), products summed exactly
# enough (float64) to stand for an FP32-accumulated matrix-core product.
# ----------------------------------------------------------------------------
def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float64 values to the nearest BF16 value (8 significant bits, ties
    to even), returned as float64.  Normal-range inputs only."""
    b = np.ascontiguousarray(x, dtype=np.float64).view(np.uint64)
    shift = np.uint64(45)                       # 52 - 7 explicit mantissa bits
    lsb = (b >> shift) & np.uint64(1)
    bias = (np.uint64(1) << np.uint64(44)) - np.uint64(1) + lsb
    r = ((b + bias) >> shift) << shift
    return r.view(np.float64).reshape(np.shape(x))


def gaussian_sketch_bf16(A: np.ndarray, m: int, seed: int, stream: int = 0) -> np.ndarray:
    n = A.shape[0]
    S = gaussian_entries(seed, stream, np.arange(m * n, dtype=np.int64)).reshape(m, n)
    S = bf16_round(S * (1.0 / math.sqrt(m)))
    return S @ bf16_round(A.astype(np.float64))


def sketch(A: np.ndarray, kind: str, m: int, seed: int, m2: int = 0) -> np.ndarray:
    if kind == "gaussian":
        return gaussian_sketch(A, m, seed)
    if kind == "srht":
        return srht_sketch(A, m, seed)
    if kind == "countsketch":
        return countsketch(A, m, seed)
    if kind == "count_gauss":
        return count_gauss_sketch(A, m, m2, seed)
    raise ValueError(kind)
