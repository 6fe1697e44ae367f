// Statistical dimension estimate from a sketch (Section 3.4, Algorithm 5):
//   sd ~ d - (lambda / T) sum_l <v^l, z^l>,   ((SA)^T SA + lambda I) z^l = v^l,
// with T Rademacher probes v^l and each system solved to relative residual
// eps_tr.  The probes come from the counter-based rule the SRHT signs use
// (entry j of probe l is -1 iff bit 31 of murmur3(l d + j, seed) is set); each
// system is one step of the persistent solve kernel in right-hand-side mode
// (matrix SA, x = 0, alpha = 1, beta = 0) whose inner solver (AAb_Solver as in
// the paper, or CG) streams SA on every step: at eps_tr ~ 0.5 it takes a few
// steps, fewer reads of SA than forming the Gram matrix would cost.
#include "device_util.hpp"
#include "internal.hpp"
#include "rng.hpp"

namespace mihs {
namespace {

// Probe l occupies V[l * ldv .. l * ldv + d); the padding is zero.
__global__ __launch_bounds__(kBlock) void probe_kernel(double* V, double* Z, int64_t d,
                                                       int64_t ldv, int64_t T, uint32_t seed) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= T * ldv) return;
  const int64_t l = i / ldv, j = i - l * ldv;
  // the key is the unpadded flat index l * d + j taken modulo 2^32
  V[i] = j >= d ? 0.0 : ((murmur3_u32((uint32_t)(l * d + j), seed) >> 31) ? -1.0 : 1.0);
  Z[i] = 0.0;
}

// sd = d - (lambda / T) sum_i V[i] Z[i]; one workgroup, fixed summation order.
// The per-probe records keep the inner-solve counts; one outer step was asked
// for, so "maximum outer iterations" reads as converged.
__global__ __launch_bounds__(kBlock) void finish_kernel(const double* V, const double* Z,
                                                        int64_t d, int64_t ldv, int64_t T,
                                                        double lam, double* sd,
                                                        mihs_info_t* info) {
  __shared__ double s_red[kWavesPerBlock];
  double v = 0.0;
  const int64_t count = ldv * T;  // the padding of V is zero
  for (int64_t i = threadIdx.x; i < count; i += kBlock) v += V[i] * Z[i];
  v = block_sum(v, s_red);
  if (threadIdx.x == 0) *sd = (double)d - lam * v / (double)T;
  for (int64_t l = threadIdx.x; l < T; l += kBlock)
    if (info[l].status == MIHS_MAX_ITER) info[l].status = MIHS_CONVERGED;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// probe rows padded to 256 bytes so every right-hand side and iterate the
// solve kernel sees is aligned like a fresh allocation
inline int64_t probe_ld(int64_t d) { return (d + 31) / 32 * 32; }

struct EstLayout {
  size_t v, z, solve, total;
};

EstLayout est_layout(const mihs_handle* h, int64_t m, int64_t d, int64_t T, int mixed) {
  EstLayout L;
  const size_t vec = align_up((size_t)T * (size_t)probe_ld(d) * sizeof(double), 256);
  L.v = 0;
  L.z = vec;
  L.solve = 2 * vec;
  L.total = L.solve + solve_workspace_bytes(h, m, d, m, mixed, /*no_gram=*/1);
  return L;
}

}  // namespace

size_t estimate_workspace_bytes(const mihs_handle* h, int64_t m, int64_t d, int64_t T,
                                int mixed) {
  return est_layout(h, m, d, T, mixed).total;
}

int launch_estimate_sd(const mihs_handle* h, const void* SA, int64_t m, int64_t d, int64_t ldsa,
                       int mixed, int aab, double lam, int64_t T, uint32_t seed, double eps_tr,
                       int64_t max_inner, double* sd, double* Zout, mihs_info_t* info,
                       void* ws, size_t ws_bytes, hipStream_t stream) {
  const EstLayout L = est_layout(h, m, d, T, mixed);
  if (ws == nullptr || ws_bytes < L.total) return MIHS_ERR_WORKSPACE;
  char* base = (char*)ws;
  double* V = (double*)(base + L.v);
  double* Z = (double*)(base + L.z);
  const int64_t ldv = probe_ld(d);
  hipLaunchKernelGGL(probe_kernel, dim3((unsigned)ceil_div(T * ldv, kBlock)), dim3(kBlock), 0,
                     stream, V, Z, d, ldv, T, seed);
  if (hipGetLastError() != hipSuccess) return MIHS_ERR_HIP;
  for (int64_t l = 0; l < T; ++l) {
    SolveDesc s;
    s.A = SA;
    s.a_f32 = mixed;
    s.n = m;
    s.d = d;
    s.lda = ldsa;
    s.b = nullptr;
    s.rhs = V + l * ldv;
    s.SA = SA;
    s.mixed = mixed;
    s.m = m;
    s.ldsa = ldsa;
    s.lam = lam;
    s.alpha = 1.0;
    s.beta = 0.0;
    s.eps_sub = eps_tr;
    s.tol = 0.0;
    s.max_outer = 1;
    s.max_inner = max_inner;
    s.x = Z + l * ldv;
    s.x_prev = nullptr;
    s.info = info + l;
    s.no_gram = 1;
    s.aab = aab;
    const int rc = launch_solve(h, s, base + L.solve, L.total - L.solve, stream);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(kBlock), 0, stream, V, Z, d, ldv, T, lam, sd,
                     info);
  if (hipGetLastError() != hipSuccess) return MIHS_ERR_HIP;
  if (Zout &&
      hipMemcpy2DAsync(Zout, (size_t)d * sizeof(double), Z, (size_t)ldv * sizeof(double),
                       (size_t)d * sizeof(double), (size_t)T, hipMemcpyDeviceToDevice,
                       stream) != hipSuccess)
    return MIHS_ERR_HIP;
  return MIHS_OK;
}

}  // namespace mihs
