"""Oracle: counter-based random sources the sketches draw from (CPU, numpy).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module; it
exists so tests, the smoke check and the CPU baseline can compute the expected
values independently of the GPU library.

The paper leaves the random sketch draw to "RP_fun" (Algorithm 1) and only
requires E[S^T S] = I (Section 3.1).  To make the GPU and the oracle draw the
*same* S without passing it in, both sides implement two published
counter-based generators from their definitions:

* MurmurHash3_x86_32 (Appleby, SMHasher; public domain) on one 4-byte
  little-endian key.  Used for CountSketch buckets/signs (Lemma 3(i)) and for
  the SRHT sign diagonal and row samples (Lemma 3(iii)).
* Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC'11).  Used, with the Box-Muller transform, for the Gaussian
  sketch (Lemma 3(iv)).
"""
from __future__ import annotations

import numpy as np

_U32 = np.uint32


def _rotl32(x: np.ndarray, r: int) -> np.ndarray:
    return (x << _U32(r)) | (x >> _U32(32 - r))


def murmur3_32(keys, seed: int) -> np.ndarray:
    """MurmurHash3_x86_32 of each uint32 key taken as its 4-byte little-endian encoding."""
    k = np.asarray(keys).astype(np.uint32, copy=True)
    with np.errstate(over="ignore"):
        h = np.full(k.shape, seed & 0xFFFFFFFF, dtype=np.uint32)
        k *= _U32(0xCC9E2D51)
        k = _rotl32(k, 15)
        k *= _U32(0x1B873593)
        h ^= k
        h = _rotl32(h, 13)
        h = h * _U32(5) + _U32(0xE6546B64)
        h ^= _U32(4)                      # total length in bytes
        h ^= h >> _U32(16)
        h *= _U32(0x85EBCA6B)
        h ^= h >> _U32(13)
        h *= _U32(0xC2B2AE35)
        h ^= h >> _U32(16)
    return h


_PH_M0 = 0xD2511F53
_PH_M1 = 0xCD9E8D57
_PH_W0 = 0x9E3779B9
_PH_W1 = 0xBB67AE85


def philox4x32_10(ctr: np.ndarray, key) -> np.ndarray:
    """Philox-4x32 with 10 rounds.  ctr: (..., 4) uint32; key: two uint32 words
    (scalars or arrays broadcastable to ctr[..., 0]).  Returns (..., 4) uint32."""
    c = np.asarray(ctr, dtype=np.uint64) & np.uint64(0xFFFFFFFF)
    c0, c1, c2, c3 = (c[..., j].copy() for j in range(4))
    k0 = np.asarray(key[0], dtype=np.uint64) & np.uint64(0xFFFFFFFF)
    k1 = np.asarray(key[1], dtype=np.uint64) & np.uint64(0xFFFFFFFF)
    mask = np.uint64(0xFFFFFFFF)
    with np.errstate(over="ignore"):
        for rnd in range(10):
            if rnd:
                k0 = (k0 + np.uint64(_PH_W0)) & mask
                k1 = (k1 + np.uint64(_PH_W1)) & mask
            p0 = c0 * np.uint64(_PH_M0)          # exact: both factors < 2^32
            p1 = c2 * np.uint64(_PH_M1)
            hi0, lo0 = p0 >> np.uint64(32), p0 & mask
            hi1, lo1 = p1 >> np.uint64(32), p1 & mask
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def gaussian_entries(seed: int, stream: int, index) -> np.ndarray:
    """Standard normal draws N(0,1) for flat element indices `index` (int64).

    Element e takes Philox block e // 4 (counter = (lo32(e//4), hi32(e//4),
    lo32(stream), hi32(stream)), key = (seed, 0)).  The block's four words give
    u_j = (w_j + 1/2) / 2^32 in (0,1); Box-Muller maps (u0,u1) to
    sqrt(-2 ln u0) * (cos, sin)(2 pi u1) for lanes 0,1 and (u2,u3) likewise for
    lanes 2,3.  All arithmetic in float64.
    """
    e = np.asarray(index, dtype=np.int64)
    blk = (e >> 2).astype(np.uint64)
    lane = (e & 3).astype(np.int64)
    ctr = np.empty(e.shape + (4,), dtype=np.uint64)
    ctr[..., 0] = blk & np.uint64(0xFFFFFFFF)
    ctr[..., 1] = blk >> np.uint64(32)
    ctr[..., 2] = np.uint64(stream & 0xFFFFFFFF)
    ctr[..., 3] = np.uint64((stream >> 32) & 0xFFFFFFFF)
    w = philox4x32_10(ctr, (seed & 0xFFFFFFFF, 0)).astype(np.float64)
    u = (w + 0.5) * (2.0 ** -32)
    pair = lane >> 1
    ua = np.where(pair == 0, u[..., 0], u[..., 2])
    ub = np.where(pair == 0, u[..., 1], u[..., 3])
    r = np.sqrt(-2.0 * np.log(ua))
    th = (2.0 * np.pi) * ub
    return np.where((lane & 1) == 0, r * np.cos(th), r * np.sin(th))
