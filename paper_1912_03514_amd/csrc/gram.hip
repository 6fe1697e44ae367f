// Gram matrices H = M^T M of sketches (M = SA, m x d row-major) on the FP64
// matrix cores.  The inner CG applies the sub-problem operator (SA)^T SA as
// H p, one d x d product per step instead of two passes over SA.
#include <type_traits>

#include "device_util.hpp"
#include "internal.hpp"

namespace mihs {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kGramRows = 32;  // rows of M staged per step

// One 64 x 64 block (bi <= bj) of H: wave w owns rows 16 w.. of the block and
// all four 16-column blocks; 32-row chunks of M are staged in LDS (FP64).
// Entries with an index >= d come out zero; off-diagonal blocks are mirrored,
// so H is exactly symmetric.
template <typename TS, typename TH>
__device__ __forceinline__ void gram_block(const TS* __restrict__ M, int64_t m, int64_t ld, int d,
                                           TH* __restrict__ H, int64_t ldh, int bi, int bj) {
  __shared__ double ti[kGramRows][64 + 1];
  __shared__ double tj[kGramRows][64 + 1];
  const int lane = lane_id(), wave = wave_id();
  const int ci0 = bi * 64, cj0 = bj * 64;
  constexpr int PER = kGramRows * 64 / kBlock;
  f64x4 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = (f64x4){0.0, 0.0, 0.0, 0.0};
  for (int64_t r0 = 0; r0 < m; r0 += kGramRows) {
    double vi[PER], vj[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = i * kBlock + (int)threadIdx.x;
      const int r = e / 64, c = e % 64;
      const int64_t gr = r0 + r;
      const bool rok = gr < m;
      vi[i] = (rok && ci0 + c < d) ? (double)M[gr * ld + ci0 + c] : 0.0;
      vj[i] = (rok && cj0 + c < d) ? (double)M[gr * ld + cj0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = i * kBlock + (int)threadIdx.x;
      ti[e / 64][e % 64] = vi[i];
      tj[e / 64][e % 64] = vj[i];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kGramRows / 4; ++s) {
      const int r = 4 * s + (lane >> 4);
      const double av = ti[r][wave * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, tj[r][b * 16 + (lane & 15)], acc[b],
                                                      0, 0, 0);
    }
  }
  // result register r of lane l: row l/16 + 4 r, column l % 16
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = ci0 + wave * 16 + (lane >> 4) + 4 * r;
      const int64_t j = cj0 + b * 16 + (lane & 15);
      H[i * ldh + j] = (TH)acc[b][r];
      if (bi != bj) H[j * ldh + i] = (TH)acc[b][r];
    }
}

template <typename TS>
__global__ __launch_bounds__(kBlock) void gram_jobs_kernel(const GramJob* jobs) {
  const GramJob J = jobs[blockIdx.x];
  if (J.h_f32)
    gram_block<TS, float>((const TS*)J.M, J.m, J.ld, J.d, (float*)J.H, J.ldh, J.bi, J.bj);
  else
    gram_block<TS, double>((const TS*)J.M, J.m, J.ld, J.d, (double*)J.H, J.ldh, J.bi, J.bj);
}

// One matrix, grid (nb, nb); blocks below the diagonal return at once.
template <typename TS, typename TH>
__global__ __launch_bounds__(kBlock) void gram_one_kernel(const TS* M, int64_t m, int64_t ld,
                                                          int d, TH* H, int64_t ldh) {
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bi > bj) return;
  gram_block<TS, TH>(M, m, ld, d, H, ldh, bi, bj);
}

// One 128 x 128 tile (bi <= bj) of H per workgroup for the single-matrix case:
// the four waves form a 2 x 2 grid of 64 x 64 quarters (4 x 4 MFMA blocks of
// 16 x 16 each).  16-row chunks of M are loaded with 16-byte vector loads one
// chunk ahead into registers, converted to FP64 and stored to LDS (double-
// buffered, one barrier per chunk).  Entries of index >= d come out zero; only
// entries below hn (the padded size of H) are written; off-diagonal tiles are
// mirrored.
constexpr int kT = 128;       // tile edge
constexpr int kKC = 16;       // rows of M per chunk
constexpr int kLdt = kT + 4;  // LDS row stride (doubles)

template <typename TS, int W = 8>
struct ChunkLoad {
  // thread t: chunk row t / 16, columns c0 + W (t % 16) .. + W of one tile
  // (W = 8: a 128-column tile, W = 4: a 64-column tile)
  static constexpr int kVec = 16 / (int)sizeof(TS) < W ? 16 / (int)sizeof(TS) : W;
  static constexpr int kN = W / kVec;  // 16-byte (or 8-byte) loads per thread per tile
  typedef TS vec_t __attribute__((ext_vector_type(kVec)));
  static __device__ __forceinline__ void run(const TS* __restrict__ M, int64_t m, int64_t ld,
                                             int d, int64_t r0, int c0, double (&out)[W]) {
    const int t = threadIdx.x;
    const int64_t r = r0 + t / 16;
    const int c = c0 + W * (t % 16);
    if (r < m && c + W <= d) {
      const TS* p = M + r * ld + c;
#pragma unroll
      for (int i = 0; i < kN; ++i) {
        const vec_t v = *(const vec_t*)(p + i * kVec);
#pragma unroll
        for (int e = 0; e < kVec; ++e) out[i * kVec + e] = (double)v[e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < W; ++e) out[e] = (r < m && c + e < d) ? (double)M[r * ld + c + e] : 0.0;
    }
  }
};

// Tiles of 128 rows (i) by TN columns (j) of H.  TN = 128: the tiles on and
// above the diagonal, each written with its mirror (a diagonal tile computes
// both of its triangles).  TN = 64 (twice as many workgroups, for matrices
// with fewer 128-tiles than CUs): every tile that holds an entry with i <= j,
// and it writes those entries and their mirrors only.
template <typename TS, typename TH, int TN>
__global__ __launch_bounds__(kBlock) void gram_tile128_kernel(const TS* M, int64_t m, int64_t ld,
                                                              int d, TH* H, int64_t ldh, int hn) {
  static_assert(TN == 128 || TN == 64, "tile width");
  constexpr int NB = TN / 32;  // 16-column blocks per wave
  constexpr int WJ = TN / 16;  // columns of the j tile loaded per thread
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (TN == kT ? bi > bj : bi * kT > bj * TN + TN - 1) return;
  __shared__ double tl[2][2][kKC][kLdt];  // [buffer][i or j tile][row][col]
  const int lane = lane_id(), wave = wave_id();
  const int wr = wave >> 1, wc = wave & 1;
  const int ci0 = bi * kT, cj0 = bj * TN;
  f64x4 acc[4][NB];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = (f64x4){0.0, 0.0, 0.0, 0.0};
  const int srow = threadIdx.x / 16, scol = 8 * (threadIdx.x % 16), scolj = WJ * (threadIdx.x % 16);
  double gi[8], gj[WJ];
  ChunkLoad<TS>::run(M, m, ld, d, 0, ci0, gi);
  ChunkLoad<TS, WJ>::run(M, m, ld, d, 0, cj0, gj);
#pragma unroll
  for (int e = 0; e < 8; ++e) tl[0][0][srow][scol + e] = gi[e];
#pragma unroll
  for (int e = 0; e < WJ; ++e) tl[0][1][srow][scolj + e] = gj[e];
  __syncthreads();
  const int64_t nchunks = (m + kKC - 1) / kKC;
  for (int64_t ch = 0; ch < nchunks; ++ch) {
    const int cur = (int)(ch & 1);
    const bool more = ch + 1 < nchunks;
    if (more) {
      ChunkLoad<TS>::run(M, m, ld, d, (ch + 1) * kKC, ci0, gi);
      ChunkLoad<TS, WJ>::run(M, m, ld, d, (ch + 1) * kKC, cj0, gj);
    }
#pragma unroll
    for (int ks = 0; ks < kKC / 4; ++ks) {
      const int r = 4 * ks + (lane >> 4);
      double av[4], bv[NB];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = tl[cur][0][r][wr * 64 + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < NB; ++b) bv[b] = tl[cur][1][r][wc * (TN / 2) + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (more) {
#pragma unroll
      for (int e = 0; e < 8; ++e) tl[cur ^ 1][0][srow][scol + e] = gi[e];
#pragma unroll
      for (int e = 0; e < WJ; ++e) tl[cur ^ 1][1][srow][scolj + e] = gj[e];
    }
    __syncthreads();
  }
  // result register r of lane l: row l/16 + 4 r, column l % 16 of each 16 x 16 block
  if constexpr (sizeof(TH) == 4) {
    // FP32 output: keep the accumulators in the matrix-core registers up to
    // here (an empty statement with an AGPR operand at the loop exit) and round
    // them one block at a time.  Left to itself, the compiler moves all 64 of
    // them to VGPRs for the rounding and then carries them through the main
    // loop in VGPRs, copying them into the matrix-core registers and back at
    // every chunk.
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) asm volatile("" : "+a"(acc[a][b]));
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = ci0 + wr * 64 + a * 16 + (lane >> 4) + 4 * r;
          const int j = cj0 + wc * (TN / 2) + b * 16 + (lane & 15);
          if (i < hn && j < hn) {
            const TH v = (TH)acc[a][b][r];
            if (TN == kT) {
              H[(int64_t)i * ldh + j] = v;
              if (bi != bj) H[(int64_t)j * ldh + i] = v;
            } else if (i <= j) {
              H[(int64_t)i * ldh + j] = v;
              H[(int64_t)j * ldh + i] = v;
            }
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
  } else {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = ci0 + wr * 64 + a * 16 + (lane >> 4) + 4 * r;
          const int j = cj0 + wc * (TN / 2) + b * 16 + (lane & 15);
          if (i < hn && j < hn) {
            const TH v = (TH)acc[a][b][r];
            if (TN == kT) {
              H[(int64_t)i * ldh + j] = v;
              if (bi != bj) H[(int64_t)j * ldh + i] = v;
            } else if (i <= j) {
              H[(int64_t)i * ldh + j] = v;
              H[(int64_t)j * ldh + i] = v;
            }
          }
        }
  }
}

}  // namespace

int launch_gram_jobs(const GramJob* d_jobs, int64_t njobs, int m_f32, hipStream_t st) {
  if (njobs <= 0) return MIHS_OK;
  if (m_f32)
    gram_jobs_kernel<float><<<dim3((unsigned)njobs), dim3(kBlock), 0, st>>>(d_jobs);
  else
    gram_jobs_kernel<double><<<dim3((unsigned)njobs), dim3(kBlock), 0, st>>>(d_jobs);
  return hipGetLastError() == hipSuccess ? MIHS_OK : MIHS_ERR_HIP;
}

int launch_gram(const void* M, int m_f32, int64_t m, int64_t d, int64_t ld, void* H, int h_f32,
                int64_t ldh, hipStream_t st) {
  const unsigned nb = (unsigned)((d + 63) / 64);
  if (ldh < 64 * (int64_t)nb) return MIHS_ERR_INVALID;
  const int hn = 64 * (int)nb;
  if (d > 64) {
    // 128 x 128 tiles: a quarter of the 64 x 64 form's reloads of M; 128 x 64
    // tiles where the 128 x 128 ones on and above the diagonal would leave
    // CUs idle (d = 2048: 136 tiles, 272 of 128 x 64)
    const unsigned nt = (unsigned)((d + kT - 1) / kT);
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return MIHS_ERR_HIP;
    const bool narrow = (int64_t)nt * (nt + 1) / 2 < ncu;
    auto go = [&](auto tn) {
      constexpr int TN = decltype(tn)::value;
      const dim3 grid((unsigned)((d + TN - 1) / TN), nt);
      if (m_f32 && h_f32)
        gram_tile128_kernel<float, float, TN><<<grid, dim3(kBlock), 0, st>>>(
            (const float*)M, m, ld, (int)d, (float*)H, ldh, hn);
      else if (m_f32)
        gram_tile128_kernel<float, double, TN><<<grid, dim3(kBlock), 0, st>>>(
            (const float*)M, m, ld, (int)d, (double*)H, ldh, hn);
      else if (h_f32)
        gram_tile128_kernel<double, float, TN><<<grid, dim3(kBlock), 0, st>>>(
            (const double*)M, m, ld, (int)d, (float*)H, ldh, hn);
      else
        gram_tile128_kernel<double, double, TN><<<grid, dim3(kBlock), 0, st>>>(
            (const double*)M, m, ld, (int)d, (double*)H, ldh, hn);
    };
    if (narrow)
      go(std::integral_constant<int, 64>());
    else
      go(std::integral_constant<int, kT>());
    return hipGetLastError() == hipSuccess ? MIHS_OK : MIHS_ERR_HIP;
  }
  const dim3 grid(nb, nb);
  if (m_f32 && h_f32)
    gram_one_kernel<float, float><<<grid, dim3(kBlock), 0, st>>>((const float*)M, m, ld, (int)d,
                                                                 (float*)H, ldh);
  else if (m_f32)
    gram_one_kernel<float, double><<<grid, dim3(kBlock), 0, st>>>((const float*)M, m, ld, (int)d,
                                                                  (double*)H, ldh);
  else if (h_f32)
    gram_one_kernel<double, float><<<grid, dim3(kBlock), 0, st>>>((const double*)M, m, ld,
                                                                  (int)d, (float*)H, ldh);
  else
    gram_one_kernel<double, double><<<grid, dim3(kBlock), 0, st>>>((const double*)M, m, ld,
                                                                   (int)d, (double*)H, ldh);
  return hipGetLastError() == hipSuccess ? MIHS_OK : MIHS_ERR_HIP;
}

}  // namespace mihs
