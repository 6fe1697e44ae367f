// Gram matrices H = M^T M of sketches (M = SA, m x d row-major) on the FP64
// matrix cores.  The inner CG applies the sub-problem operator (SA)^T SA as
// H p, one d x d product per step instead of two passes over SA.
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
