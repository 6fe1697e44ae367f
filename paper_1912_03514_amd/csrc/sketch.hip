// Sketch kernels (Lemma 3): SRHT via a blocked fast Walsh-Hadamard transform,
// CountSketch via a deterministic bucket sort + segmented sums, Gaussian via
// counter-based generation and a matrix-core GEMM (FP64 MFMA for the plain
// path, BF16 MFMA with FP32 accumulation for the mixed path).
#include <math.h>

#include "device_util.hpp"
#include "internal.hpp"
#include "rng.hpp"

namespace mihs {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// BF16 rounding (round to nearest even of the exact value).  A double is first
// narrowed to float with round-to-odd (truncate, then set the sticky bit if
// inexact) so the second rounding to BF16 is a single correct rounding.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t bf16_rne_from_float(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ uint16_t bf16_rne(double x) {
  float f = __double2float_rz(x);
  if ((double)f != x) f = __uint_as_float(__float_as_uint(f) | 1u);
  return bf16_rne_from_float(f);
}
__device__ __forceinline__ uint16_t bf16_rne(float x) { return bf16_rne_from_float(x); }

// ---------------------------------------------------------------------------
// SRHT:  SA = (1/sqrt(m)) P H D A with H = H_hi (x) H_lo (Sylvester order):
// row index i = i_hi * B + i_lo.  Stage 1 applies D and the length-B transform
// over i_lo inside each block of B consecutive rows (in LDS).  Stage 2 forms
// each sampled row k = (k_hi, k_lo) as sum_{i_hi} (-1)^{popc(k_hi & i_hi)}
// Y[i_hi * B + k_lo], reading each needed row of Y once per column block.
// ---------------------------------------------------------------------------
__global__ void srht_rows_kernel(int* idx, int64_t m, int64_t n, uint32_t seed) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) idx[k] = (int)(murmur3_u32((uint32_t)k, seed + kSrhtSampleSeedOffset) & (uint32_t)(n - 1));
}

constexpr int kFwhtW = 16;  // columns per stage-1 tile

template <typename TA, typename TY>
__global__ __launch_bounds__(kBlock) void srht_stage1(const TA* __restrict__ A, int64_t lda,
                                                      int64_t d, int logB, uint32_t seed,
                                                      TY* __restrict__ Y, int64_t ldy) {
  extern __shared__ unsigned char smem_raw[];
  TY* T = (TY*)smem_raw;  // B x kFwhtW
  const int B = 1 << logB;
  const int64_t row0 = (int64_t)blockIdx.y * B;
  const int64_t c0 = (int64_t)blockIdx.x * kFwhtW;
  for (int e = threadIdx.x; e < B * kFwhtW; e += kBlock) {
    const int r = e / kFwhtW, c = e % kFwhtW;
    const int64_t gr = row0 + r, gc = c0 + c;
    TY v = TY(0);
    if (gc < d) {
      v = (TY)A[gr * lda + gc];
      if (murmur3_u32((uint32_t)gr, seed) >> 31) v = -v;
    }
    T[e] = v;
  }
  __syncthreads();
  for (int h = 1; h < B; h <<= 1) {
    for (int p = threadIdx.x; p < (B / 2) * kFwhtW; p += kBlock) {
      const int c = p % kFwhtW, q = p / kFwhtW;
      const int i = (q / h) * 2 * h + (q % h);
      const TY u = T[i * kFwhtW + c], v = T[(i + h) * kFwhtW + c];
      T[i * kFwhtW + c] = u + v;
      T[(i + h) * kFwhtW + c] = u - v;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < B * kFwhtW; e += kBlock) {
    const int r = e / kFwhtW, c = e % kFwhtW;
    const int64_t gc = c0 + c;
    if (gc < d) Y[(row0 + r) * ldy + gc] = T[e];
  }
}

// Stage 1 for blocks of 512 rows: the 9 butterfly levels of H_512 split as
// 4 levels in registers on rows s + 32 i (i = 0..15, bits 5..8 of the row),
// one transpose through LDS, then 5 levels in registers on rows 32 g + i
// (i = 0..31, bits 0..4).  W columns per workgroup (16 for FP64 A, 32 for
// FP32 A, i.e. 128-byte row segments).
template <typename T, int N>
__device__ __forceinline__ void fwht_regs(T (&x)[N]) {
#pragma unroll
  for (int h = 1; h < N; h <<= 1) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      if ((j & h) == 0) {
        const T a = x[j], b = x[j + h];
        x[j] = a + b;
        x[j + h] = a - b;
      }
    }
  }
}

template <typename TA, typename TY>
__global__ __launch_bounds__(kBlock) void srht_stage1_b512(const TA* __restrict__ A, int64_t lda,
                                                           int64_t d, uint32_t seed,
                                                           TY* __restrict__ Y, int64_t ldy) {
  // 32 columns when the transform runs in FP32 (256-byte row segments of FP64 A),
  // else 16 (the LDS tile stays at ~66 KiB either way)
  constexpr int W = sizeof(TY) == 4 ? 32 : 16;
  constexpr int C1 = W / 8;   // columns per thread, phase 1
  constexpr int C2 = W / 16;  // columns per thread, phase 2
  constexpr int PAD = 1;
  __shared__ TY T[512][W + PAD];
  const int64_t row0 = (int64_t)blockIdx.y * 512;  // column blocks vary fastest, so
  const int64_t c0 = (int64_t)blockIdx.x * W;       // concurrent workgroups cover whole rows
  const int t = threadIdx.x;
  {
    const int cp = t % 8, sl = t / 8;  // column group, row slot 0..31
    TY x[C1][16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int64_t gr = row0 + sl + 32 * i;
      const TA* src = A + gr * lda + c0 + C1 * cp;
      TA v[C1];
      if (c0 + C1 * cp + C1 <= d) {
        VecLoad<TA, C1, true>::run(src, v);  // one 16-byte load
      } else {
#pragma unroll
        for (int q = 0; q < C1; ++q) v[q] = (c0 + C1 * cp + q < d) ? src[q] : TA(0);
      }
      const bool neg = (murmur3_u32((uint32_t)gr, seed) >> 31) != 0;
#pragma unroll
      for (int q = 0; q < C1; ++q) x[q][i] = neg ? -(TY)v[q] : (TY)v[q];
    }
#pragma unroll
    for (int q = 0; q < C1; ++q) fwht_regs<TY, 16>(x[q]);
#pragma unroll
    for (int i = 0; i < 16; ++i)
#pragma unroll
      for (int q = 0; q < C1; ++q) T[sl + 32 * i][C1 * cp + q] = x[q][i];
  }
  __syncthreads();
  {
    const int c = C2 * (t % 16), g = t / 16;  // first column (C2 adjacent), row group 0..15
    TY y[C2][32];
#pragma unroll
    for (int i = 0; i < 32; ++i)
#pragma unroll
      for (int q = 0; q < C2; ++q) y[q][i] = T[32 * g + i][c + q];
#pragma unroll
    for (int q = 0; q < C2; ++q) fwht_regs<TY, 32>(y[q]);
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      TY* dst = Y + (row0 + 32 * g + i) * ldy + c0 + c;
      if (c0 + c + C2 <= d) {
#pragma unroll
        for (int q = 0; q < C2; ++q) dst[q] = y[q][i];
      } else {
#pragma unroll
        for (int q = 0; q < C2; ++q)
          if (c0 + c + q < d) dst[q] = y[q][i];
      }
    }
  }
}

constexpr int kS2Cols = 64;    // columns per stage-2 workgroup
constexpr int kS2Chunk = 8;    // samples accumulated together
constexpr int kS2Cap = 512;    // sample list capacity

template <typename TY, typename TS>
__global__ __launch_bounds__(kBlock) void srht_stage2(const TY* __restrict__ Y, int64_t ldy,
                                                      int64_t d, int logB, int64_t nhi,
                                                      const int* __restrict__ idx, int64_t m,
                                                      TS* __restrict__ SA, int64_t ldsa,
                                                      double scale) {
  __shared__ int s_list[kS2Cap];
  __shared__ int s_wcnt[kWavesPerBlock];
  __shared__ TY s_red[kWavesPerBlock][kS2Chunk][kS2Cols];
  const int B = 1 << logB;
  const int klo = blockIdx.y;  // column blocks vary fastest (whole rows of Y in flight)
  const int64_t col = (int64_t)blockIdx.x * kS2Cols + (threadIdx.x & (kS2Cols - 1));
  const int rg = threadIdx.x >> 6;  // row group = wave
  const int lane = lane_id();
  int cnt = 0;

  auto process = [&](int count) {
    for (int s0 = 0; s0 < count; s0 += kS2Chunk) {
      const int ns = min(kS2Chunk, count - s0);
      int khi[kS2Chunk];
      TY acc[kS2Chunk];
#pragma unroll
      for (int s = 0; s < kS2Chunk; ++s) {
        khi[s] = (s < ns) ? (idx[s_list[s0 + s]] >> logB) : 0;
        acc[s] = TY(0);
      }
      if (col < d) {
        constexpr int U = 8;  // rows loaded together per thread
        for (int64_t ih0 = rg; ih0 < nhi; ih0 += (int64_t)U * kWavesPerBlock) {
          TY y[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int64_t ih = ih0 + (int64_t)u * kWavesPerBlock;
            y[u] = (ih < nhi) ? Y[(ih * B + klo) * ldy + col] : TY(0);
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const unsigned ih = (unsigned)(ih0 + (int64_t)u * kWavesPerBlock);
#pragma unroll
            for (int s = 0; s < kS2Chunk; ++s) {
              if (s < ns) {  // uniform: the chunk's sample count
                const int par = __popc((unsigned)khi[s] & ih) & 1;
                acc[s] += par ? -y[u] : y[u];
              }
            }
          }
        }
      }
#pragma unroll
      for (int s = 0; s < kS2Chunk; ++s) s_red[rg][s][lane] = acc[s];
      __syncthreads();
      if (rg == 0 && col < d) {
        for (int s = 0; s < ns; ++s) {
          TY t = s_red[0][s][lane];
#pragma unroll
          for (int g = 1; g < kWavesPerBlock; ++g) t += s_red[g][s][lane];
          SA[(int64_t)s_list[s0 + s] * ldsa + col] = (TS)((double)t * scale);
        }
      }
      __syncthreads();
    }
  };

  for (int64_t w0 = 0; w0 < m; w0 += kBlock) {
    const int64_t k = w0 + threadIdx.x;
    const bool match = (k < m) && ((idx[k] & (B - 1)) == klo);
    const unsigned long long ball = __ballot(match);
    const int before = __popcll(ball & ((1ull << lane) - 1ull));
    if (lane == 0) s_wcnt[rg] = __popcll(ball);
    __syncthreads();
    int off = 0, total = 0;
    for (int g = 0; g < kWavesPerBlock; ++g) {
      if (g < rg) off += s_wcnt[g];
      total += s_wcnt[g];
    }
    if (cnt + total > kS2Cap) {
      process(cnt);
      cnt = 0;
    }
    if (match) s_list[cnt + off + before] = (int)k;
    cnt += total;
    __syncthreads();
  }
  if (cnt > 0) process(cnt);
}

// ---------------------------------------------------------------------------
// SRHT in one read of A.  A workgroup of 512 threads owns a strip of 16
// columns and a range of blocks of B = 2^LOGB consecutive rows.  For each block
// i_hi it applies D and the length-B transform over i_lo (registers, one LDS
// transpose), leaving T[k_lo] = sum_{i_lo} (-1)^{popc(k_lo & i_lo)} (D A)[i_hi B + i_lo]
// in LDS, and then adds every sampled row k = (k_hi, k_lo) with its sign:
//     acc_k += (-1)^{popc(k_hi & i_hi)} T[k_lo],
// so that after all blocks acc_k = ((H D A)[idx_k]) restricted to the strip.
// Thread (c, g), c = t % 16, g = t / 16, owns column c of samples
// g * NACC .. g * NACC + NACC - 1 in registers.  The next block's rows are
// loaded while the current one is transformed and accumulated.  Each sample's
// row offset in T and block index k_hi share one 32-bit word in LDS (one read
// per sample and block; with two, the FP32 form used 236 VGPRs and the FP64
// form spilled, against 204 and 210 now).  The partial
// sums of the workgroup's block range go to P[part] (or, with one range per
// strip, scaled straight to SA).
// ---------------------------------------------------------------------------
// Mixed CountSketch -> Gaussian: the FP32 bucket sums CA enter the Gaussian
// stage as three BF16 terms (hi + mid + lo), so that the BF16 products keep
// CA's FP32 accuracy; rounding CA itself to BF16 (2^-9 relative) perturbs
// the sketched Hessian by more than lambda on ill-conditioned problems.
constexpr int kCountGaussTerms = 3;

constexpr int kFusedThreads = 512;
constexpr int kBufferRsrcWord3 = 0x00020000;  // raw 32-bit buffer data (gfx9 family)
constexpr int kBufferNt = 2;                  // cache policy: non-temporal
constexpr int kFusedW = 16;       // columns per strip
constexpr int kFusedLdt = kFusedW + 1;

// sign words: bit j of word w is set iff D_{32 w + j} = -1
__global__ void srht_sign_words_kernel(uint32_t* words, int64_t nwords, uint32_t seed) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nwords) return;
  uint32_t v = 0u;
  for (int j = 0; j < 32; ++j)
    v |= (murmur3_u32((uint32_t)(w * 32 + j), seed) >> 31) << j;
  words[w] = v;
}

template <typename TA, typename TY, int LOGB, int NACC, typename TS>
__global__ __launch_bounds__(kFusedThreads) void srht_fused_kernel(
    const TA* __restrict__ A, int64_t lda, int64_t d, const uint32_t* __restrict__ signw,
    const int* __restrict__ idx, int64_t m, int64_t nblk, int nparts, TY* __restrict__ P,
    int64_t ldp, TS* __restrict__ SA, int64_t ldsa, double scale) {
  constexpr int B = 1 << LOGB;
  constexpr int R = B * kFusedW / kFusedThreads;  // rows per thread per phase (16 or 32)
  static_assert(R == 16 || R == 32, "block shape");
  extern __shared__ unsigned char smem_raw[];
  TY* T = (TY*)smem_raw;                                   // B x kFusedLdt
  // per sample: its row offset in T (low 16 bits) and k_hi (high 16 bits), one
  // LDS read per sample and block
  uint32_t* s_smp = (uint32_t*)(T + (size_t)B * kFusedLdt);  // 32 * NACC
  const int t = threadIdx.x;
  const int c = t % kFusedW, g = t / kFusedW;              // g in [0, 32)
  const int strip = blockIdx.x % (int)((d + kFusedW - 1) / kFusedW);
  const int part = blockIdx.x / (int)((d + kFusedW - 1) / kFusedW);
  const int64_t col = (int64_t)strip * kFusedW + c;
  const bool col_ok = col < d;
  const int64_t b0 = nblk * part / nparts, b1 = nblk * (part + 1) / nparts;

  for (int k = t; k < 32 * NACC; k += kFusedThreads) {
    const int v = k < m ? idx[k] : 0;
    const uint32_t khi = k < m ? (uint32_t)(v >> LOGB) : 0u;
    s_smp[k] = (uint32_t)((v & (B - 1)) * kFusedLdt) | (khi << 16);
  }
  TY acc[NACC];
#pragma unroll
  for (int j = 0; j < NACC; ++j) acc[j] = TY(0);

  // rows g + 32 i of block b, this thread's column, as buffer loads: the
  // block's base in a buffer resource, row 32 i's byte offset in a scalar
  // register and one per-lane byte offset, so that the row addresses do not
  // each occupy a pair of vector registers.  Non-temporal: A is read once.
  // Every offset stays below the block's B rows (checked against num_records).
  TA xa[R];
  const uint32_t lane_off = (uint32_t)(((int64_t)g * lda + (col_ok ? col : 0)) * sizeof(TA));
  const int32_t row32 = (int32_t)(32 * lda * (int64_t)sizeof(TA));  // bytes between rows g + 32 i
  const int32_t blk_bytes = (int32_t)(B * lda * (int64_t)sizeof(TA));
  auto load_block = [&](int64_t b) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(A + b * B * lda), (short)0, blk_bytes, kBufferRsrcWord3);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if constexpr (sizeof(TA) == 8) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, lane_off, i * row32, kBufferNt);
        xa[i] = __builtin_bit_cast(TA, v);
      } else {
        const auto v = __builtin_amdgcn_raw_buffer_load_b32(rs, lane_off, i * row32, kBufferNt);
        xa[i] = __builtin_bit_cast(TA, v);
      }
    }
  };
  if (b0 < b1) load_block(b0);
  for (int64_t b = b0; b < b1; ++b) {
    // phase 1: D, then the butterflies of row bits 5 .. LOGB-1 (register index bits)
    TY x[R];
    const uint32_t* sw = signw + b * (B / 32);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const bool neg = (sw[i] >> g) & 1u;
      x[i] = neg ? -(TY)xa[i] : (TY)xa[i];
    }
    // the next block's rows as soon as this block's are in x
    if (b + 1 < b1) load_block(b + 1);
    fwht_regs<TY, R>(x);
    __syncthreads();  // the previous block's accumulation has read T
#pragma unroll
    for (int i = 0; i < R; ++i) T[(g + 32 * i) * kFusedLdt + c] = x[i];
    __syncthreads();
    // phase 2: the butterflies of row bits 0 .. log2(R)-1 on rows R g + i
    {
      TY y[R];
#pragma unroll
      for (int i = 0; i < R; ++i) y[i] = T[(R * g + i) * kFusedLdt + c];
      fwht_regs<TY, R>(y);
      if constexpr (R == 16) {
        // row bit 4: rows 16 g + i and 16 (g ^ 1) + i live in threads t and t ^ 16
        // (the same wave)
        const bool upper = (g & 1) != 0;
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const TY other = __shfl_xor(y[i], kFusedW, kWave);
          y[i] = upper ? other - y[i] : y[i] + other;
        }
      }
#pragma unroll
      for (int i = 0; i < R; ++i) T[(R * g + i) * kFusedLdt + c] = y[i];
    }
    __syncthreads();
    // every owned sample: acc_k += (-1)^{popc(k_hi & b)} T[k_lo][c], eight
    // samples at a time (the empty asm keeps the compiler from hoisting every
    // sample's LDS reads at once, which would not fit in the registers)
    const uint32_t bb = (uint32_t)b;
    const TY* Tc = T + c;
#pragma unroll
    for (int j0 = 0; j0 < NACC; j0 += 8) {
      asm volatile("" ::: "memory");
#pragma unroll
      for (int j = j0; j < j0 + 8; ++j) {
        const int k = g * NACC + j;
        const uint32_t smp = s_smp[k];
        const TY v = Tc[smp & 0xFFFFu];
        const bool neg = (__popc((smp >> 16) & bb) & 1) != 0;
        acc[j] += neg ? -v : v;
      }
    }
  }
  if (!col_ok) return;
  if (nparts == 1) {
#pragma unroll
    for (int j = 0; j < NACC; ++j) {
      const int64_t k = (int64_t)g * NACC + j;
      if (k < m) SA[k * ldsa + col] = (TS)((double)acc[j] * scale);
    }
  } else {
    TY* Pp = P + (int64_t)part * m * ldp;
#pragma unroll
    for (int j = 0; j < NACC; ++j) {
      const int64_t k = (int64_t)g * NACC + j;
      if (k < m) Pp[k * ldp + col] = acc[j];
    }
  }
}

// SA[k][col] = scale * sum_{part} P[part][k][col], parts in order.
template <typename TY, typename TS>
__global__ void srht_parts_sum_kernel(const TY* __restrict__ P, int nparts, int64_t m, int64_t d,
                                      int64_t ldp, TS* __restrict__ SA, int64_t ldsa, double scale) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * d) return;
  const int64_t k = e / d, col = e - k * d;
  TY s = P[k * ldp + col];
  for (int q = 1; q < nparts; ++q) s += P[((int64_t)q * m + k) * ldp + col];
  SA[k * ldsa + col] = (TS)((double)s * scale);
}

__global__ void zero_u32_kernel(unsigned* p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// CountSketch: h = murmur3(i, seed), bucket = h mod m, sign = -1 iff bit 31.
// Rows are bucketed by a counting sort, each bucket's row list is sorted
// ascending, then each (bucket, column block) sums its rows in that order, so
// the result does not depend on scheduling.
// ---------------------------------------------------------------------------
__global__ void cs_hash_kernel(int64_t n, int64_t m, uint32_t seed, unsigned* code,
                               unsigned* hist) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t h = murmur3_u32((uint32_t)i, seed);
  const unsigned bucket = h % (uint32_t)m;
  code[i] = bucket | (h & 0x80000000u);
  atomicAdd(&hist[bucket], 1u);
}

// Exclusive scan of hist[0..m) into off[0..m]; one workgroup.
__global__ __launch_bounds__(kBlock) void cs_scan_kernel(const unsigned* hist, int64_t m,
                                                         unsigned* off, unsigned* cursor) {
  __shared__ unsigned s_part[kBlock];
  const int64_t per = (m + kBlock - 1) / kBlock;
  const int64_t b0 = threadIdx.x * per, b1 = min(m, b0 + per);
  unsigned s = 0;
  for (int64_t i = b0; i < b1; ++i) s += hist[i];
  s_part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned run = 0;
    for (int t = 0; t < kBlock; ++t) {
      const unsigned v = s_part[t];
      s_part[t] = run;
      run += v;
    }
    off[m] = run;
  }
  __syncthreads();
  unsigned run = s_part[threadIdx.x];
  for (int64_t i = b0; i < b1; ++i) {
    off[i] = run;
    cursor[i] = run;
    run += hist[i];
  }
}

__global__ void cs_scatter_kernel(int64_t n, const unsigned* code, int64_t m, unsigned* cursor,
                                  unsigned* perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned c = code[i];
  const unsigned pos = atomicAdd(&cursor[c & 0x7FFFFFFFu], 1u);
  perm[pos] = (unsigned)i;  // row index (n < 2^31)
}

constexpr int kSortCap = 2048;

// Sort each bucket's row list ascending (bitonic in LDS; a serial fallback for
// oversized buckets keeps the result well defined).
__global__ __launch_bounds__(kBlock) void cs_sort_kernel(const unsigned* off, unsigned* perm) {
  __shared__ unsigned s[kSortCap];
  const unsigned b0 = off[blockIdx.x], b1 = off[blockIdx.x + 1];
  const int cnt = (int)(b1 - b0);
  if (cnt <= 1) return;
  if (cnt > kSortCap) {
    if (threadIdx.x == 0) {
      for (int i = 1; i < cnt; ++i) {
        const unsigned v = perm[b0 + i];
        int j = i - 1;
        while (j >= 0 && perm[b0 + j] > v) {
          perm[b0 + j + 1] = perm[b0 + j];
          --j;
        }
        perm[b0 + j + 1] = v;
      }
    }
    return;
  }
  int P = 1;
  while (P < cnt) P <<= 1;
  for (int i = threadIdx.x; i < P; i += kBlock) s[i] = (i < cnt) ? perm[b0 + i] : 0xFFFFFFFFu;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += kBlock) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const unsigned a = s[i], b = s[ixj];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            s[i] = b;
            s[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < cnt; i += kBlock) perm[b0 + i] = s[i];
}

template <typename TA, typename TAcc, typename TOut>
__global__ __launch_bounds__(kBlock) void cs_accum_kernel(const TA* __restrict__ A, int64_t lda,
                                                          int64_t d, const unsigned* off,
                                                          const unsigned* perm,
                                                          const unsigned* code,
                                                          TOut* __restrict__ out, int64_t ldo) {
  const unsigned bucket = blockIdx.x;
  const int64_t col = (int64_t)blockIdx.y * kBlock + threadIdx.x;
  const unsigned b0 = off[bucket], b1 = off[bucket + 1];
  TAcc acc = TAcc(0);
  if (col < d) {
    unsigned p = b0;
    for (; p + 4 <= b1; p += 4) {
      TAcc v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const unsigned row = perm[p + t];
        const TAcc a = (TAcc)__builtin_nontemporal_load(&A[(int64_t)row * lda + col]);
        v[t] = (code[row] & 0x80000000u) ? -a : a;
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) acc += v[t];
    }
    for (; p < b1; ++p) {
      const unsigned row = perm[p];
      const TAcc a = (TAcc)__builtin_nontemporal_load(&A[(int64_t)row * lda + col]);
      acc += (code[row] & 0x80000000u) ? -a : a;
    }
    out[(int64_t)bucket * ldo + col] = (TOut)acc;
  }
}

// ---------------------------------------------------------------------------
// Gaussian:  S (M x K, row stride lds) with S_ij = N(0,1) * scale drawn from
// Philox element i*K + j; stored as double (plain) or BF16 bits (mixed).
// Columns K..lds-1 are zero.
// ---------------------------------------------------------------------------
template <typename TSel>
__global__ void gauss_gen_kernel(TSel* S, int64_t M, int64_t K, int64_t lds, uint32_t seed,
                                 uint64_t stream, double scale) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // one Philox block each
  const int64_t total = M * K;
  const int64_t first = e * 4;
  if (first >= total) return;
  // FP64 draws for the FP64 sketch; FP32 draws for the BF16 sketch (rounded to
  // 8 significant bits anyway)
  double z[4];
  float zf[4];
  if constexpr (sizeof(TSel) == 8)
    gaussian_block(seed, stream, (uint64_t)e, z);
  else
    gaussian_block_f32(seed, stream, (uint64_t)e, zf);
  const float scale_f = (float)scale;
  // row and column of the first element (one 64-bit division per thread), then
  // step along the row with wrap-around
  int64_t i = first / K, j = first - i * K;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (first + t < total) {
      if constexpr (sizeof(TSel) == 8) {
        S[i * lds + j] = z[t] * scale;
      } else {
        S[i * lds + j] = bf16_rne(zf[t] * scale_f);
      }
    }
    if (++j == K) {
      j = 0;
      ++i;
    }
  }
}

__global__ void zero_pad_cols(void* S, int elem, int64_t M, int64_t K, int64_t lds) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t padw = lds - K;
  if (padw <= 0 || e >= M * padw) return;
  const int64_t i = e / padw, j = K + e % padw;
  if (elem == 8)
    ((double*)S)[i * lds + j] = 0.0;
  else
    ((uint16_t*)S)[i * lds + j] = 0;
}

// P[z] (M x N) = S[:, kz] B[kz, :] in FP64 on the matrix cores
// (v_mfma_f64_16x16x4: A operand lane l = row l%16, k l/16; B operand lane l =
// col l%16, k l/16; result register r of lane l is row l/16 + 4r, column l%16).
template <typename TS, typename TB>
__global__ __launch_bounds__(kBlock) void gemm_f64_kernel(const TS* __restrict__ S, int64_t lds,
                                                          int64_t M, int64_t K,
                                                          const TB* __restrict__ B, int64_t ldb,
                                                          int64_t N, int64_t kchunk,
                                                          double* __restrict__ P) {
  constexpr int BM = 64, BN = 64, BK = 16;
  __shared__ double Ss[BM][BK + 1];
  __shared__ double Bs[BK][BN + 1];
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  const int64_t kb = (int64_t)blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  const int lane = lane_id(), wave = wave_id();
  const int wr = wave >> 1, wc = wave & 1;
  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (f64x4){0.0, 0.0, 0.0, 0.0};
  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
    for (int e = threadIdx.x; e < BM * BK; e += kBlock) {
      const int r = e / BK, c = e % BK;
      const int64_t gr = m0 + r, gk = k0 + c;
      Ss[r][c] = (gr < M && gk < ke) ? (double)S[gr * lds + gk] : 0.0;
    }
    for (int e = threadIdx.x; e < BK * BN; e += kBlock) {
      const int r = e / BN, c = e % BN;
      const int64_t gk = k0 + r, gc = n0 + c;
      Bs[r][c] = (gk < ke && gc < N) ? (double)B[gk * ldb + gc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = Ss[wr * 32 + i * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk + (lane >> 4)][wc * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  double* Pz = P + (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + wr * 32 + i * 16 + (lane >> 4) + 4 * r;
        const int64_t col = n0 + wc * 32 + j * 16 + (lane & 15);
        if (row < M && col < N) Pz[row * N + col] = acc[i][j][r];
      }
}

// Bt (N x ldbt, BF16 bits) = B^T rounded to BF16 (round to nearest even of the
// exact value), zero for k in [K, ldbt): the sketch GEMM's right operand with k
// contiguous, made once per sketch so that the GEMM streams 2-byte values
// instead of re-reading (and re-rounding) B for every 128-row tile of S.
// 64 x 64 tiles through LDS: reads along n, writes along k.
template <typename TB>
__global__ __launch_bounds__(kBlock) void bf16_transpose_kernel(const TB* __restrict__ B,
                                                                int64_t K, int64_t N, int64_t ldb,
                                                                uint16_t* __restrict__ Bt,
                                                                int64_t ldbt) {
  __shared__ uint16_t tile[64][66];
  const int64_t k0 = (int64_t)blockIdx.y * 64, n0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int kk = ty + 4 * i;
    const int64_t gk = k0 + kk, gn = n0 + tx;
    tile[kk][tx] = (gk < K && gn < N) ? bf16_rne(B[gk * ldb + gn]) : (uint16_t)0;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int nn = ty + 4 * i;
    const int64_t gn = n0 + nn, gk = k0 + tx;
    if (gn < N && gk < ldbt) Bt[gn * ldbt + gk] = tile[tx][nn];
  }
}

// The three-term BF16 split of B^T for products that must keep B's FP32
// accuracy: Bt_t (t = 0, 1, 2; stride part_stride) holds hi, mid, lo with
// hi = bf16(v), mid = bf16(v - hi), lo = bf16(v - hi - mid) for v = B[k, n]
// (each difference is exact in FP32), so that hi + mid + lo equals v to about
// 2^-24 relative and S (hi + mid + lo) is S B to FP32 accuracy.
__global__ __launch_bounds__(kBlock) void bf16_split3_transpose_kernel(
    const float* __restrict__ B, int64_t K, int64_t N, int64_t ldb, uint16_t* __restrict__ Bt,
    int64_t ldbt, int64_t part_stride) {
  __shared__ uint16_t tile[3][64][66];
  const int64_t k0 = (int64_t)blockIdx.y * 64, n0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
#pragma unroll 4
  for (int i = 0; i < 16; ++i) {
    const int kk = ty + 4 * i;
    const int64_t gk = k0 + kk, gn = n0 + tx;
    uint16_t h = 0, mi = 0, lo = 0;
    if (gk < K && gn < N) {
      const float v = B[gk * ldb + gn];
      h = bf16_rne(v);
      const float r1 = v - __uint_as_float((uint32_t)h << 16);
      mi = bf16_rne(r1);
      const float r2 = r1 - __uint_as_float((uint32_t)mi << 16);
      lo = bf16_rne(r2);
    }
    tile[0][kk][tx] = h;
    tile[1][kk][tx] = mi;
    tile[2][kk][tx] = lo;
  }
  __syncthreads();
#pragma unroll 4
  for (int i = 0; i < 16; ++i) {
    const int nn = ty + 4 * i;
    const int64_t gn = n0 + nn, gk = k0 + tx;
    if (gn < N && gk < ldbt) {
      Bt[gn * ldbt + gk] = tile[0][tx][nn];
      Bt[part_stride + gn * ldbt + gk] = tile[1][tx][nn];
      Bt[2 * part_stride + gn * ldbt + gk] = tile[2][tx][nn];
    }
  }
}

// P[z] (M x N) = S[:, kz] B[kz, :] with BF16 inputs and FP32 accumulation, B
// given as Bt = B^T in BF16 (both operands k-contiguous)
// (v_mfma_f32_16x16x32_bf16: lane l holds 8 consecutive k, 8(l/16)..+7, of
// row l%16 (A) / column l%16 (B); result register r of lane l is row
// 4(l/16) + r, column l%16).  128 x 128 tiles, 64 k per step; the global loads
// of step t + 1 are in flight in registers while step t is multiplied from LDS.
__global__ __launch_bounds__(kBlock) void gemm_bf16_kernel(const uint16_t* __restrict__ S,
                                                           int64_t lds, int64_t M, int64_t K,
                                                           const uint16_t* __restrict__ Bt,
                                                           int64_t ldbt, int64_t N,
                                                           int64_t kchunk, float* __restrict__ P) {
  constexpr int BM = 128, BN = 128, BK = 64, PAD = 8;
  constexpr int Q = BM * (BK / 8) / kBlock;  // 16-byte chunks per operand, thread and step
  static_assert(BM == BN && Q == 4, "tile shape");
  __shared__ __attribute__((aligned(16))) uint16_t As[BM][BK + PAD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN][BK + PAD];
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  const int64_t kb = (int64_t)blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  const int lane = lane_id(), wave = wave_id();
  const int wr = wave >> 1, wc = wave & 1;
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
  uint4 sreg[Q], breg[Q];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int t = 0; t < Q; ++t) {
      const int e = (int)threadIdx.x + t * kBlock;
      const int r = e / (BK / 8), q = e % (BK / 8);
      const int64_t gk = k0 + 8 * q;
      uint4 v = make_uint4(0u, 0u, 0u, 0u), w = make_uint4(0u, 0u, 0u, 0u);
      if (gk < ke) {
        const int64_t gr = m0 + r, gn = n0 + r;
        if (gr < M) {
          v = *(const uint4*)(S + gr * lds + gk);
          if (gk + 8 > ke) {  // zero the k's beyond this split's end (in S only)
            union {
              uint4 u;
              uint16_t h[8];
            } x;
            x.u = v;
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (gk + u >= ke) x.h[u] = 0;
            v = x.u;
          }
        }
        if (gn < N) w = *(const uint4*)(Bt + gn * ldbt + gk);
      }
      sreg[t] = v;
      breg[t] = w;
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int t = 0; t < Q; ++t) {
      const int e = (int)threadIdx.x + t * kBlock;
      const int r = e / (BK / 8), q = e % (BK / 8);
      *(uint4*)&As[r][8 * q] = sreg[t];
      *(uint4*)&Bs[r][8 * q] = breg[t];
    }
  };
  if (kb < ke) gload(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
    __syncthreads();  // the previous step's products are done with As / Bs
    lstore();
    __syncthreads();
    if (k0 + BK < ke) gload(k0 + BK);  // in flight during this step's products
#pragma unroll
    for (int kk = 0; kk < BK; kk += 32) {
      bf16x8 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        a[i] = *(const bf16x8*)&As[wr * 64 + i * 16 + (lane & 15)][kk + 8 * (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        b[j] = *(const bf16x8*)&Bs[wc * 64 + j * 16 + (lane & 15)][kk + 8 * (lane >> 4)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  float* Pz = P + (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + wr * 64 + i * 16 + 4 * (lane >> 4) + r;
        const int64_t col = n0 + wc * 64 + j * 16 + (lane & 15);
        if (row < M && col < N) Pz[row * N + col] = acc[i][j][r];
      }
}

// out (M x N, row stride ldo) = sum_z P[z] in order z = 0..splits-1
template <typename TP, typename TOut>
__global__ void splitk_reduce_kernel(const TP* P, int splits, int64_t M, int64_t N, TOut* out,
                                     int64_t ldo) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * N) return;
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += (double)P[(int64_t)z * M * N + e];
  out[(e / N) * ldo + (e % N)] = (TOut)s;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline bool hip_ok() { return hipGetLastError() == hipSuccess; }

// ---- Gaussian sketch driver -------------------------------------------------
struct GaussPlan {
  int64_t lds;     // padded row stride of S
  int splits;
  int64_t kchunk;
  int64_t ldbt;    // row stride of the BF16 transpose of B (mixed)
  int terms;       // BF16 terms of B (mixed): 1, or 3 for the FP32-accurate split
  size_t s_bytes, p_bytes, bt_bytes;
  size_t total() const { return s_bytes + p_bytes + bt_bytes; }
};

GaussPlan gauss_plan(const mihs_handle* h, int64_t M, int64_t K, int64_t N, int mixed,
                     int terms = 1) {
  GaussPlan g;
  g.terms = mixed ? terms : 1;
  const int BM = mixed ? 128 : 64, BN = mixed ? 128 : 64, BK = mixed ? 64 : 16;
  g.lds = (K + 7) / 8 * 8;
  const int64_t tiles = ceil_div(M, BM) * ceil_div(N, BN);
  int64_t want = ceil_div(2 * (int64_t)h->num_cu, tiles);
  const int64_t kmax = ceil_div(K, 8 * BK);  // keep >= 8 k-steps per split
  if (want > kmax) want = kmax;
  if (want < 1) want = 1;
  if (want > 64) want = 64;
  g.kchunk = ceil_div(ceil_div(K, want), BK) * BK;
  g.splits = (int)ceil_div(K, g.kchunk);
  g.s_bytes = align_up((size_t)M * g.lds * (mixed ? 2 : 8), 256);
  g.p_bytes = align_up((size_t)g.terms * g.splits * M * N * (mixed ? 4 : 8), 256);
  g.ldbt = (K + 7) / 8 * 8;
  g.bt_bytes = mixed ? align_up((size_t)g.terms * N * g.ldbt * 2, 256) : 0;
  return g;
}

// SA (M x N, row stride ldo, TOut) = G B with G = N(0,1)/sqrt(M) (M x K) from
// Philox stream `stream`; B is K x N (row stride ldb, TB).
template <typename TB>
int run_gauss(const mihs_handle* h, const TB* B, int64_t K, int64_t N, int64_t ldb, int64_t M,
              uint32_t seed, uint64_t stream_id, int mixed, void* out, int64_t ldo, char* ws,
              size_t ws_bytes, hipStream_t st, int terms = 1) {
  const GaussPlan g = gauss_plan(h, M, K, N, mixed, terms);
  if (ws_bytes < g.total()) return MIHS_ERR_WORKSPACE;
  void* S = ws;
  void* P = ws + g.s_bytes;
  const double scale = 1.0 / sqrt((double)M);
  const int64_t nblk = ceil_div(M * K, 4);
  if (mixed)
    hipLaunchKernelGGL(gauss_gen_kernel<uint16_t>, dim3((unsigned)ceil_div(nblk, 256)), dim3(256),
                       0, st, (uint16_t*)S, M, K, g.lds, seed, stream_id, scale);
  else
    hipLaunchKernelGGL(gauss_gen_kernel<double>, dim3((unsigned)ceil_div(nblk, 256)), dim3(256), 0,
                       st, (double*)S, M, K, g.lds, seed, stream_id, scale);
  if (g.lds > K)
    hipLaunchKernelGGL(zero_pad_cols, dim3((unsigned)ceil_div(M * (g.lds - K), 256)), dim3(256), 0,
                       st, S, mixed ? 2 : 8, M, K, g.lds);
  if (!hip_ok()) return MIHS_ERR_HIP;
  if (mixed) {
    uint16_t* Bt = (uint16_t*)(ws + g.s_bytes + g.p_bytes);
    const dim3 tgrid((unsigned)ceil_div(N, 64), (unsigned)ceil_div(g.ldbt, 64));
    const int64_t part = N * g.ldbt;  // elements of one BF16 term of B^T
    if constexpr (sizeof(TB) == 4) {
      if (g.terms == 3)
        hipLaunchKernelGGL(bf16_split3_transpose_kernel, tgrid, dim3(kBlock), 0, st, B, K, N,
                           ldb, Bt, g.ldbt, part);
      else
        hipLaunchKernelGGL(bf16_transpose_kernel<TB>, tgrid, dim3(kBlock), 0, st, B, K, N, ldb,
                           Bt, g.ldbt);
    } else {
      if (g.terms != 1) return MIHS_ERR_UNSUPPORTED;
      hipLaunchKernelGGL(bf16_transpose_kernel<TB>, tgrid, dim3(kBlock), 0, st, B, K, N, ldb, Bt,
                         g.ldbt);
    }
    // one GEMM per term into its own split-K partials; the reduction adds them
    // all in a fixed order
    dim3 grid((unsigned)ceil_div(N, 128), (unsigned)ceil_div(M, 128), (unsigned)g.splits);
    for (int t = 0; t < g.terms; ++t)
      hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(kBlock), 0, st, (const uint16_t*)S, g.lds,
                         M, K, (const uint16_t*)(Bt + t * part), g.ldbt, N, g.kchunk,
                         (float*)P + (int64_t)t * g.splits * M * N);
    hipLaunchKernelGGL((splitk_reduce_kernel<float, float>), dim3((unsigned)ceil_div(M * N, 256)),
                       dim3(256), 0, st, (const float*)P, g.terms * g.splits, M, N, (float*)out,
                       ldo);
  } else {
    dim3 grid((unsigned)ceil_div(N, 64), (unsigned)ceil_div(M, 64), (unsigned)g.splits);
    hipLaunchKernelGGL((gemm_f64_kernel<double, TB>), grid, dim3(kBlock), 0, st, (const double*)S, g.lds, M,
                       K, B, ldb, N, g.kchunk, (double*)P);
    hipLaunchKernelGGL((splitk_reduce_kernel<double, double>), dim3((unsigned)ceil_div(M * N, 256)),
                       dim3(256), 0, st, (const double*)P, g.splits, M, N, (double*)out, ldo);
  }
  return hip_ok() ? MIHS_OK : MIHS_ERR_HIP;
}

// ---- CountSketch driver -------------------------------------------------------
struct CsPlan {
  size_t code, perm, hist, off, cursor, total;
};
CsPlan cs_plan(int64_t n, int64_t m) {
  CsPlan p;
  size_t o = 0;
  p.code = o; o = align_up(o + (size_t)n * 4, 256);
  p.perm = o; o = align_up(o + (size_t)n * 4, 256);
  p.hist = o; o = align_up(o + (size_t)m * 4, 256);
  p.off = o; o = align_up(o + (size_t)(m + 1) * 4, 256);
  p.cursor = o; o = align_up(o + (size_t)m * 4, 256);
  p.total = o;
  return p;
}

template <typename TA, typename TAcc, typename TOut>
int run_countsketch(const TA* A, int64_t n, int64_t d, int64_t lda, int64_t m, uint32_t seed,
                    TOut* out, int64_t ldo, char* ws, size_t ws_bytes, hipStream_t st) {
  const CsPlan p = cs_plan(n, m);
  if (ws_bytes < p.total) return MIHS_ERR_WORKSPACE;
  unsigned* code = (unsigned*)(ws + p.code);
  unsigned* perm = (unsigned*)(ws + p.perm);
  unsigned* hist = (unsigned*)(ws + p.hist);
  unsigned* off = (unsigned*)(ws + p.off);
  unsigned* cursor = (unsigned*)(ws + p.cursor);
  // the histogram starts from zero (a kernel, not a memset: a caller may
  // capture this sequence in a graph)
  hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, hist, m);
  hipLaunchKernelGGL(cs_hash_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, n, m,
                     seed, code, hist);
  hipLaunchKernelGGL(cs_scan_kernel, dim3(1), dim3(kBlock), 0, st, hist, m, off, cursor);
  hipLaunchKernelGGL(cs_scatter_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, n, code,
                     m, cursor, perm);
  hipLaunchKernelGGL(cs_sort_kernel, dim3((unsigned)m), dim3(kBlock), 0, st, off, perm);
  hipLaunchKernelGGL((cs_accum_kernel<TA, TAcc, TOut>), dim3((unsigned)m, (unsigned)ceil_div(d, kBlock)),
                     dim3(kBlock), 0, st, A, lda, d, off, perm, code, out, ldo);
  return hip_ok() ? MIHS_OK : MIHS_ERR_HIP;
}

// ---- SRHT driver ----------------------------------------------------------------
int srht_logB(int64_t n) {
  int lb = 0;
  while ((1LL << (lb + 1)) <= n && lb < 9) ++lb;
  return lb;
}

// The one-read SRHT: block size (B = 2^logb rows), samples per thread, and the
// number of block ranges per strip (enough workgroups for one per CU).  Used
// when n >= B and m <= 2048; else the two-stage transform below.
struct SrhtFusedPlan {
  bool ok = false;
  int logb = 0, nacc = 0, nparts = 1;
  int64_t nblk = 0, strips = 0;
  size_t idx_bytes = 0, sign_bytes = 0, part_bytes = 0, lds = 0;
  size_t total() const { return idx_bytes + sign_bytes + part_bytes; }
};

SrhtFusedPlan srht_fused_plan(const mihs_handle* h, int64_t n, int64_t d, int64_t m, int ty_bytes) {
  SrhtFusedPlan F;
  F.logb = ty_bytes == 4 ? 10 : 9;
  if (n < (1LL << F.logb) || (n & (n - 1)) != 0 || m > 2048 || m < 1) return F;
  // a sample's block index k_hi is kept in 16 bits
  if ((n >> F.logb) > 65536) return F;
  F.ok = true;
  F.nacc = m <= 512 ? 16 : (m <= 1024 ? 32 : 64);
  F.nblk = n >> F.logb;
  F.strips = (d + kFusedW - 1) / kFusedW;
  int64_t parts = (h->num_cu + F.strips - 1) / F.strips;
  if (parts > F.nblk) parts = F.nblk;
  if (parts < 1) parts = 1;
  F.nparts = (int)parts;
  F.idx_bytes = align_up((size_t)m * 4, 256);
  F.sign_bytes = align_up((size_t)(n / 32) * 4, 256);
  F.part_bytes = F.nparts > 1 ? align_up((size_t)F.nparts * m * d * ty_bytes, 256) : 0;
  F.lds = (size_t)(1 << F.logb) * kFusedLdt * ty_bytes + 32 * (size_t)F.nacc * 4;
  return F;
}

template <typename TA, typename TY, int LOGB, typename TS>
int launch_srht_fused(const SrhtFusedPlan& F, const TA* A, int64_t lda, int64_t d, int64_t m,
                      const uint32_t* signw, const int* idx, TY* P, TS* SA, int64_t ldsa,
                      double scale, hipStream_t st) {
  const dim3 grid((unsigned)(F.strips * F.nparts));
  auto go = [&](auto kern) -> int {
    if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)F.lds) != hipSuccess)
      return MIHS_ERR_HIP;
    hipLaunchKernelGGL(kern, grid, dim3(kFusedThreads), F.lds, st, A, lda, d, signw, idx, m,
                       F.nblk, F.nparts, P, d, SA, ldsa, scale);
    return MIHS_OK;
  };
  int rc;
  if (F.nacc == 16) rc = go(srht_fused_kernel<TA, TY, LOGB, 16, TS>);
  else if (F.nacc == 32) rc = go(srht_fused_kernel<TA, TY, LOGB, 32, TS>);
  else rc = go(srht_fused_kernel<TA, TY, LOGB, 64, TS>);
  if (rc) return rc;
  if (F.nparts > 1)
    hipLaunchKernelGGL((srht_parts_sum_kernel<TY, TS>), dim3((unsigned)ceil_div(m * d, 256)),
                       dim3(256), 0, st, P, F.nparts, m, d, d, SA, ldsa, scale);
  return MIHS_OK;
}

template <typename TA, typename TY, typename TS>
int run_srht(const mihs_handle* h, const TA* A, int64_t n, int64_t d, int64_t lda, int64_t m,
             uint32_t seed, TS* SA, int64_t ldsa, char* ws, size_t ws_bytes, hipStream_t st) {
  SrhtFusedPlan F = srht_fused_plan(h, n, d, m, (int)sizeof(TY));
  // a block's bytes must fit the 32-bit buffer range of the row loads
  if (F.ok && (double)(1LL << F.logb) * (double)lda * sizeof(TA) >= 2147483647.0) F.ok = false;
  if (F.ok) {
    if (ws_bytes < F.total()) return MIHS_ERR_WORKSPACE;
    int* idx = (int*)ws;
    uint32_t* signw = (uint32_t*)(ws + F.idx_bytes);
    TY* P = (TY*)(ws + F.idx_bytes + F.sign_bytes);
    hipLaunchKernelGGL(srht_rows_kernel, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, idx,
                       m, n, seed);
    hipLaunchKernelGGL(srht_sign_words_kernel, dim3((unsigned)ceil_div(n / 32, 256)), dim3(256),
                       0, st, signw, n / 32, seed);
    const double scale = 1.0 / sqrt((double)m);
    int rc;
    if constexpr (sizeof(TY) == 4)
      rc = launch_srht_fused<TA, TY, 10, TS>(F, A, lda, d, m, signw, idx, P, SA, ldsa, scale, st);
    else
      rc = launch_srht_fused<TA, TY, 9, TS>(F, A, lda, d, m, signw, idx, P, SA, ldsa, scale, st);
    if (rc) return rc;
    return hip_ok() ? MIHS_OK : MIHS_ERR_HIP;
  }
  const size_t idx_bytes = align_up((size_t)m * 4, 256);
  const int64_t ldy = (d + 3) / 4 * 4;
  const size_t y_bytes = align_up((size_t)n * ldy * sizeof(TY), 256);
  if (ws_bytes < idx_bytes + y_bytes) return MIHS_ERR_WORKSPACE;
  int* idx = (int*)ws;
  TY* Y = (TY*)(ws + idx_bytes);
  const int logB = srht_logB(n);
  const int B = 1 << logB;
  const int64_t nhi = n >> logB;
  hipLaunchKernelGGL(srht_rows_kernel, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, idx, m, n,
                     seed);
  if (logB == 9) {
    constexpr int W = sizeof(TY) == 4 ? 32 : 16;
    hipLaunchKernelGGL((srht_stage1_b512<TA, TY>), dim3((unsigned)ceil_div(d, W), (unsigned)nhi),
                       dim3(kBlock), 0, st, A, lda, d, seed, Y, ldy);
  } else {
    const size_t sh1 = (size_t)B * kFwhtW * sizeof(TY);
    if (hipFuncSetAttribute((const void*)srht_stage1<TA, TY>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh1) != hipSuccess)
      return MIHS_ERR_HIP;
    hipLaunchKernelGGL((srht_stage1<TA, TY>), dim3((unsigned)ceil_div(d, kFwhtW), (unsigned)nhi),
                       dim3(kBlock), sh1, st, A, lda, d, logB, seed, Y, ldy);
  }
  hipLaunchKernelGGL((srht_stage2<TY, TS>), dim3((unsigned)ceil_div(d, kS2Cols), (unsigned)B),
                     dim3(kBlock), 0, st, Y, ldy, d, logB, nhi, idx, m, SA, ldsa,
                     1.0 / sqrt((double)m));
  return hip_ok() ? MIHS_OK : MIHS_ERR_HIP;
}

__global__ __launch_bounds__(kBlock) void neg_dot_kernel(const double* X, const double* W,
                                                         int64_t count, double lam, double* out,
                                                         double* out_log) {
  __shared__ double s_red[kWavesPerBlock];
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += kBlock) v += X[i] * W[i];
  v = block_sum(v, s_red);
  if (threadIdx.x == 0) {
    *out = -v;
    if (out_log) *out_log = lam * -v;  // chain rule through lambda = exp(log lambda)
  }
}

__global__ void fill_kernel(double* p, double v, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

}  // namespace

int launch_fill(double* p, double value, int64_t count, hipStream_t st) {
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, st, p, value,
                     count);
  return hip_ok() ? MIHS_OK : MIHS_ERR_HIP;
}

int launch_apply_rows(const mihs_handle* h, const void* A, int a_f32, int64_t n, int64_t d,
                      int64_t lda, const double* W, int64_t k, double* Y, int64_t ldy,
                      hipStream_t st) {
  (void)h;
  if (ldy != k) return MIHS_ERR_UNSUPPORTED;
  dim3 grid((unsigned)ceil_div(k, 64), (unsigned)ceil_div(n, 64), 1);
  if (a_f32)
    hipLaunchKernelGGL((gemm_f64_kernel<float, double>), grid, dim3(kBlock), 0, st,
                       (const float*)A, lda, n, d, W, k, k, d, Y);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<double, double>), grid, dim3(kBlock), 0, st,
                       (const double*)A, lda, n, d, W, k, k, d, Y);
  return hip_ok() ? MIHS_OK : MIHS_ERR_HIP;
}

int launch_neg_dot(const double* X, const double* W, int64_t count, double lam, double* out,
                   double* out_log, hipStream_t st) {
  hipLaunchKernelGGL(neg_dot_kernel, dim3(1), dim3(kBlock), 0, st, X, W, count, lam, out,
                     out_log);
  return hip_ok() ? MIHS_OK : MIHS_ERR_HIP;
}

size_t sketch_workspace_bytes(const mihs_handle* h, int64_t n, int64_t d, int64_t m, int64_t m2,
                              int kind, int a_f32, int mixed) {
  (void)a_f32;
  switch (kind) {
    case MIHS_GAUSSIAN: {
      const GaussPlan g = gauss_plan(h, m, n, d, mixed);
      return g.total();
    }
    case MIHS_SRHT: {
      const SrhtFusedPlan F = srht_fused_plan(h, n, d, m, mixed ? 4 : 8);
      if (F.ok) return F.total();
      const int64_t ldy = (d + 3) / 4 * 4;
      return align_up((size_t)m * 4, 256) + align_up((size_t)n * ldy * (mixed ? 4 : 8), 256);
    }
    case MIHS_COUNTSKETCH:
      return cs_plan(n, m).total;
    case MIHS_COUNT_GAUSS: {
      const int64_t ldc = (d + 3) / 4 * 4;
      const size_t ca = align_up((size_t)m * ldc * (mixed ? 4 : 8), 256);
      const GaussPlan g = gauss_plan(h, m2, m, d, mixed, kCountGaussTerms);
      const size_t a = cs_plan(n, m).total, b = g.total();
      return ca + (a > b ? a : b);
    }
    default:
      return 0;
  }
}

int launch_sketch(const mihs_handle* h, const void* A, int a_f32, int64_t n, int64_t d,
                  int64_t lda, int kind, int64_t m, int64_t m2, uint32_t seed, int mixed,
                  void* SA, int64_t ldsa, void* ws, size_t ws_bytes, hipStream_t st) {
  const size_t need = sketch_workspace_bytes(h, n, d, m, m2, kind, a_f32, mixed);
  if (!ws || ws_bytes < need) return MIHS_ERR_WORKSPACE;
  char* w = (char*)ws;
  switch (kind) {
    case MIHS_GAUSSIAN:
      if (a_f32)
        return run_gauss<float>(h, (const float*)A, n, d, lda, m, seed, 0, mixed, SA, ldsa, w, ws_bytes, st);
      return run_gauss<double>(h, (const double*)A, n, d, lda, m, seed, 0, mixed, SA, ldsa, w, ws_bytes, st);
    case MIHS_SRHT:
      if (mixed) {
        if (a_f32)
          return run_srht<float, float, float>(h, (const float*)A, n, d, lda, m, seed, (float*)SA, ldsa, w, ws_bytes, st);
        return run_srht<double, float, float>(h, (const double*)A, n, d, lda, m, seed, (float*)SA, ldsa, w, ws_bytes, st);
      }
      if (a_f32)
        return run_srht<float, double, double>(h, (const float*)A, n, d, lda, m, seed, (double*)SA, ldsa, w, ws_bytes, st);
      return run_srht<double, double, double>(h, (const double*)A, n, d, lda, m, seed, (double*)SA, ldsa, w, ws_bytes, st);
    case MIHS_COUNTSKETCH:
      if (mixed) {
        if (a_f32)
          return run_countsketch<float, float, float>((const float*)A, n, d, lda, m, seed, (float*)SA, ldsa, w, ws_bytes, st);
        return run_countsketch<double, float, float>((const double*)A, n, d, lda, m, seed, (float*)SA, ldsa, w, ws_bytes, st);
      }
      if (a_f32)
        return run_countsketch<float, double, double>((const float*)A, n, d, lda, m, seed, (double*)SA, ldsa, w, ws_bytes, st);
      return run_countsketch<double, double, double>((const double*)A, n, d, lda, m, seed, (double*)SA, ldsa, w, ws_bytes, st);
    case MIHS_COUNT_GAUSS: {
      const int64_t ldc = (d + 3) / 4 * 4;
      const size_t ca_bytes = align_up((size_t)m * ldc * (mixed ? 4 : 8), 256);
      char* rest = w + ca_bytes;
      const size_t rest_bytes = ws_bytes - ca_bytes;
      int rc;
      if (mixed) {
        float* CA = (float*)w;
        rc = a_f32 ? run_countsketch<float, float, float>((const float*)A, n, d, lda, m, seed, CA, ldc, rest, rest_bytes, st)
                   : run_countsketch<double, float, float>((const double*)A, n, d, lda, m, seed, CA, ldc, rest, rest_bytes, st);
        if (rc) return rc;
        return run_gauss<float>(h, CA, m, d, ldc, m2, seed, 1, 1, SA, ldsa, rest, rest_bytes, st,
                                kCountGaussTerms);
      }
      double* CA = (double*)w;
      rc = a_f32 ? run_countsketch<float, double, double>((const float*)A, n, d, lda, m, seed, CA, ldc, rest, rest_bytes, st)
                 : run_countsketch<double, double, double>((const double*)A, n, d, lda, m, seed, CA, ldc, rest, rest_bytes, st);
      if (rc) return rc;
      return run_gauss<double>(h, CA, m, d, ldc, m2, seed, 1, 0, SA, ldsa, rest, rest_bytes, st);
    }
    default:
      return MIHS_ERR_INVALID;
  }
}

}  // namespace mihs
