// Counter-based random sources of the sketches, written from their published
// definitions:
//  - MurmurHash3_x86_32 (A. Appleby, SMHasher, public domain) of a single
//    4-byte little-endian key;
//  - Philox-4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11) and the
//    Box-Muller transform for N(0,1) draws.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace mihs {

constexpr uint32_t kSrhtSampleSeedOffset = 0x9E3779B9u;

__device__ __forceinline__ uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

__device__ __forceinline__ uint32_t murmur3_u32(uint32_t key, uint32_t seed) {
  uint32_t k = key * 0xCC9E2D51u;
  k = rotl32(k, 15);
  k *= 0x1B873593u;
  uint32_t h = seed ^ k;
  h = rotl32(h, 13);
  h = h * 5u + 0xE6546B64u;
  h ^= 4u;  // key length in bytes
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

struct U32x4 {
  uint32_t v[4];
};

__device__ __forceinline__ U32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint32_t hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
    const uint32_t hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  U32x4 o;
  o.v[0] = c0;
  o.v[1] = c1;
  o.v[2] = c2;
  o.v[3] = c3;
  return o;
}

// The four N(0,1) draws of Philox block `blk` (elements 4*blk .. 4*blk+3).
__device__ __forceinline__ void gaussian_block(uint32_t seed, uint64_t stream, uint64_t blk,
                                               double out[4]) {
  const U32x4 w = philox4x32_10((uint32_t)blk, (uint32_t)(blk >> 32), (uint32_t)stream,
                                (uint32_t)(stream >> 32), seed, 0u);
  const double two32inv = 2.3283064365386963e-10;  // 2^-32
  const double twopi = 6.283185307179586;           // 2 pi rounded to double
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const double ua = ((double)w.v[2 * p] + 0.5) * two32inv;
    const double ub = ((double)w.v[2 * p + 1] + 0.5) * two32inv;
    const double rad = sqrt(-2.0 * log(ua));
    double s, c;
    sincos(twopi * ub, &s, &c);
    out[2 * p] = rad * c;
    out[2 * p + 1] = rad * s;
  }
}

// The same four draws in FP32 for the mixed path, whose Gaussian entries are
// rounded to BF16 (8 significant bits) afterwards: the uniforms as above,
// rad = sqrt(-2 ln 2 log2(u_a)) and (cos, sin)(2 pi u_b) on the hardware's
// log2 / sine / cosine units (v_sin_f32 and v_cos_f32 take their argument in
// revolutions).  Relative error a few units of 2^-24, so the BF16 value equals
// the rounding of the FP64 draw except where the FP64 draw lies within that
// error of a BF16 rounding boundary (about one entry in 10^4, off by one BF16
// unit).
__device__ __forceinline__ void gaussian_block_f32(uint32_t seed, uint64_t stream, uint64_t blk,
                                                   float out[4]) {
  const U32x4 w = philox4x32_10((uint32_t)blk, (uint32_t)(blk >> 32), (uint32_t)stream,
                                (uint32_t)(stream >> 32), seed, 0u);
  const float two32inv = 2.3283064365386963e-10f;  // 2^-32
  const float m2ln2 = -1.3862943611198906f;        // -2 ln 2
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    // u = (w + 1/2) 2^-32 in (0, 1]; float(w) keeps 24 bits, plenty for BF16
    const float ua = ((float)w.v[2 * p] + 0.5f) * two32inv;
    const float ub = ((float)w.v[2 * p + 1] + 0.5f) * two32inv;
    const float rad = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(ua));
    out[2 * p] = rad * __builtin_amdgcn_cosf(ub);
    out[2 * p + 1] = rad * __builtin_amdgcn_sinf(ub);
  }
}

}  // namespace mihs
