// Primal-Dual M-IHS (Section 2, two-stage sketching; Algorithms 3 and 4).
//
// The outer loop is M-IHS on the outer variable x (Algorithm 4: x in R^d for a
// tall A; Algorithm 3: nu in R^n, streaming A^T).  Its sub-problem
//   (Q Q^T + lambda I) dx = g,     Q = (S A)^T  (cols x m1),
// is solved through its dual: M M-IHS steps on
//   min_z 1/2 ||Q z - g||^2 + lambda/2 ||z||^2      (z in R^{m1}),
// whose Hessian Q^T Q + lambda I = (SA)(SA)^T + lambda I is sketched again by
// WQ = W Q (m2 x m1); then dx = (g - Q z) / lambda (eq. (dual_relation)).  The
// dual iterate and its momentum state carry over between outer steps.
//
// Per outer step the host enqueues, on one stream and without waiting:
//   gradient pass over the outer matrix     (two kernels)
//   the dual steps: one persistent solve on Q in ridge mode with b = g,
//     sketch WQ, M iterations, AAb_Solver or CG inner (CG through the Gram
//     matrix of WQ, formed once), warm-started from (z, z_prev)  (solve kernel)
//   t = Q z                                  (row dot products)
//   dx, heavy-ball update, relative-step test (one workgroup)
// The update kernel raises a device flag once the stop rule holds or the inner
// solve failed; every kernel of the later steps reads it first and returns, so
// the enqueued tail costs only launch latency.
#include <math.h>

#include "device_util.hpp"
#include "internal.hpp"

namespace mihs {
namespace {

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

__device__ __forceinline__ bool flag_set(const int* f) {
  return __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

__global__ __launch_bounds__(kBlock) void pd_init_kernel(const double* x, double* xp, int64_t cols,
                                                         double* z, double* zp, int64_t m1,
                                                         int* done, mihs_info_t* info) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < cols) xp[i] = x[i];  // x^0 = x^1
  if (i < m1) {
    z[i] = 0.0;
    zp[i] = 0.0;
  }
  if (i == 0) {
    *done = 0;
    info->outer_iters = 0;
    info->inner_iters_total = 0;
    info->inner_iters_max = 0;
    info->rel_step = 0.0;
    info->grad_norm = 0.0;
    info->status = MIHS_MAX_ITER;
    info->elapsed_us = 0;
  }
}

// t[r] = Q[r, :] . z, one wave per row (coalesced over the row).
template <typename TQ>
__global__ __launch_bounds__(kBlock) void pd_matvec_kernel(const TQ* Q, int64_t rows, int64_t ldq,
                                                           int64_t m1, const double* z, double* t,
                                                           const int* done) {
  if (flag_set(done)) return;
  const int64_t row = (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
  if (row >= rows) return;
  const TQ* q = Q + row * ldq;
  double s = 0.0;
  for (int64_t j = lane_id(); j < m1; j += kWave) s += (double)q[j] * z[j];
  s = wave_sum(s);
  if (lane_id() == 0) t[row] = s;
}

// dx = (g - t) / lambda; x+ = x + alpha1 dx + beta1 (x - x_prev); the relative
// step and the stop decision.  One workgroup.
__global__ __launch_bounds__(kBlock) void pd_update_kernel(const double* g, const double* t,
                                                           int64_t cols, double lam, double a1,
                                                           double b1, double thr, double* x,
                                                           double* xp, int* done,
                                                           const mihs_info_t* iinfo,
                                                           mihs_info_t* info) {
  __shared__ double s_red[kWavesPerBlock];
  if (flag_set(done)) return;
  const int inner_status = iinfo->status;
  if (inner_status < 0) {
    // the dual steps failed: keep x, report, stop
    if (threadIdx.x == 0) {
      info->status = inner_status;
      *done = 1;
    }
    return;
  }
  double s0 = 0.0, s1 = 0.0, gg = 0.0;
  for (int64_t k = threadIdx.x; k < cols; k += kBlock) {
    const double gk = g[k];
    const double dx = (gk - t[k]) / lam;
    const double xc = x[k];
    const double xn = xc + a1 * dx + b1 * (xc - xp[k]);
    xp[k] = xc;
    x[k] = xn;
    s0 += (xn - xc) * (xn - xc);
    s1 += xn * xn;
    gg += gk * gk;
  }
  s0 = block_sum(s0, s_red);
  s1 = block_sum(s1, s_red);
  gg = block_sum(gg, s_red);
  if (threadIdx.x == 0) {
    const int64_t kin = iinfo->inner_iters_total;
    info->outer_iters += 1;
    info->inner_iters_total += kin;
    if (kin > info->inner_iters_max) info->inner_iters_max = kin;
    const double step = s1 > 0.0 ? sqrt(s0 / s1) : 0.0;
    info->rel_step = step;
    info->grad_norm = sqrt(gg);
    int st = MIHS_MAX_ITER;
    if (!isfinite(step)) st = MIHS_BREAKDOWN;
    else if (thr > 0.0 && step <= thr) st = MIHS_CONVERGED;
    info->status = st;
    if (st != MIHS_MAX_ITER) *done = 1;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void transpose_kernel(const T* src, int64_t rows, int64_t cols,
                                                           int64_t lds, T* dst, int64_t ldd) {
  __shared__ T tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
  for (int k = ty; k < 32; k += kBlock / 32) {
    const int64_t r = r0 + k, c = c0 + tx;
    if (r < rows && c < cols) tile[k][tx] = src[r * lds + c];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += kBlock / 32) {
    const int64_t c = c0 + k, r = r0 + tx;
    if (c < cols && r < rows) dst[c * ldd + r] = tile[tx][k];
  }
}

struct PdLayout {
  size_t flag, iinfo, g, t, xp, z, zp, grad, solve, total;
};

PdLayout pd_layout(const mihs_handle* h, int64_t rows, int64_t cols, int64_t m1, int64_t m2,
                   int mixed) {
  PdLayout L;
  size_t off = 0;
  const size_t vc = align_up((size_t)cols * 8, 256), vm = align_up((size_t)m1 * 8, 256);
  L.flag = off;  off += 256;
  L.iinfo = off; off += align_up(sizeof(mihs_info_t), 256);
  L.g = off;     off += vc;
  L.t = off;     off += vc;
  L.xp = off;    off += vc;
  L.z = off;     off += vm;
  L.zp = off;    off += vm;
  L.grad = off;  off += grad_workspace_bytes(h, rows, cols);
  L.solve = off; off += solve_workspace_bytes(h, cols, m1, m2, mixed, /*no_gram=*/0);
  L.total = off;
  return L;
}

}  // namespace

size_t pd_workspace_bytes(const mihs_handle* h, int64_t rows, int64_t cols, int64_t m1,
                          int64_t m2, int mixed) {
  return pd_layout(h, rows, cols, m1, m2, mixed).total;
}

int launch_pd(const mihs_handle* h, const PdDesc& p, void* ws, size_t ws_bytes,
              hipStream_t stream) {
  const PdLayout L = pd_layout(h, p.rows, p.cols, p.m1, p.m2, p.mixed);
  if (ws == nullptr || ws_bytes < L.total) return MIHS_ERR_WORKSPACE;
  char* base = (char*)ws;
  int* done = (int*)(base + L.flag);
  mihs_info_t* iinfo = (mihs_info_t*)(base + L.iinfo);
  double* g = (double*)(base + L.g);
  double* t = (double*)(base + L.t);
  double* xp = (double*)(base + L.xp);
  double* z = (double*)(base + L.z);
  double* zp = (double*)(base + L.zp);
  const int64_t span = p.cols > p.m1 ? p.cols : p.m1;
  hipLaunchKernelGGL(pd_init_kernel, dim3((unsigned)ceil_div(span, kBlock)), dim3(kBlock), 0,
                     stream, p.x, xp, p.cols, z, zp, p.m1, done, p.info);
  if (hipGetLastError() != hipSuccess) return MIHS_ERR_HIP;
  const double thr = (p.tol > 0.0 && p.beta1 > 0.0 && p.beta1 < 1.0)
                         ? p.tol * (1.0 - sqrt(p.beta1)) / sqrt(p.beta1)
                         : (p.tol > 0.0 ? p.tol : 0.0);
  // the dual steps: Algorithm 1 on min 1/2 ||Q z - g||^2 + lambda/2 ||z||^2
  SolveDesc s;
  s.A = p.Q;
  s.a_f32 = p.mixed;
  s.n = p.cols;
  s.d = p.m1;
  s.lda = p.ldq;
  s.b = g;
  s.rhs = nullptr;
  s.SA = p.WQ;
  s.mixed = p.mixed;
  s.m = p.m2;
  s.ldsa = p.ldwq;
  s.lam = p.lam;
  s.alpha = p.alpha2;
  s.beta = p.beta2;
  s.eps_sub = p.eps_sub;
  s.tol = 0.0;
  s.max_outer = p.M;
  s.max_inner = p.max_inner;
  s.x = z;
  s.x_prev = zp;
  s.info = iinfo;
  // AAb_Solver streams WQ; CG goes through the Gram matrix of WQ when m2 >= m1,
  // formed by the first outer step and reused by the later ones
  s.no_gram = p.aab ? 1 : 0;
  s.aab = p.aab;
  s.skip = done;
  const unsigned mv_blocks = (unsigned)ceil_div(p.cols, kWavesPerBlock);
  for (int64_t i = 0; i < p.max_outer; ++i) {
    int rc = launch_grad(h, p.A, p.a_f32, p.rows, p.cols, p.lda, p.c, p.rhs, p.x, p.lam, g,
                         base + L.grad, L.solve - L.grad, done, stream);
    if (rc) return rc;
    s.gram_ready = i > 0 ? 1 : 0;
    rc = launch_solve(h, s, base + L.solve, L.total - L.solve, stream);
    if (rc) return rc;
    if (p.mixed)
      hipLaunchKernelGGL(pd_matvec_kernel<float>, dim3(mv_blocks), dim3(kBlock), 0, stream,
                         (const float*)p.Q, p.cols, p.ldq, p.m1, z, t, done);
    else
      hipLaunchKernelGGL(pd_matvec_kernel<double>, dim3(mv_blocks), dim3(kBlock), 0, stream,
                         (const double*)p.Q, p.cols, p.ldq, p.m1, z, t, done);
    hipLaunchKernelGGL(pd_update_kernel, dim3(1), dim3(kBlock), 0, stream, g, t, p.cols, p.lam,
                       p.alpha1, p.beta1, thr, p.x, xp, done, iinfo, p.info);
    if (hipGetLastError() != hipSuccess) return MIHS_ERR_HIP;
  }
  return MIHS_OK;
}

int launch_transpose(const void* src, int f32, int64_t rows, int64_t cols, int64_t lds,
                     void* dst, int64_t ldd, hipStream_t stream) {
  const int64_t gy = ceil_div(rows, 32);
  if (gy > 65535) return MIHS_ERR_UNSUPPORTED;
  dim3 grid((unsigned)ceil_div(cols, 32), (unsigned)gy);
  if (f32)
    hipLaunchKernelGGL(transpose_kernel<float>, grid, dim3(kBlock), 0, stream, (const float*)src,
                       rows, cols, lds, (float*)dst, ldd);
  else
    hipLaunchKernelGGL(transpose_kernel<double>, grid, dim3(kBlock), 0, stream,
                       (const double*)src, rows, cols, lds, (double*)dst, ldd);
  return hipGetLastError() == hipSuccess ? MIHS_OK : MIHS_ERR_HIP;
}

}  // namespace mihs
