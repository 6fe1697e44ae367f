// C ABI entry points of libmihs: handle management, argument validation and
// dispatch to the kernel launchers.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "internal.hpp"

using mihs::align_up;

namespace {

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

int elem_size(int f32) { return f32 ? 4 : 8; }

bool rows_aligned(const void* p, int64_t ld, int f32) {
  return aligned16(p) && ((ld * elem_size(f32)) % 16 == 0);
}

bool valid_matrix(const void* p, int64_t rows, int64_t cols, int64_t ld, int f32) {
  return p != nullptr && rows > 0 && cols > 0 && ld >= cols && rows_aligned(p, ld, f32);
}

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

}  // namespace

extern "C" {

int mihs_create(mihs_handle_t* handle, int device) {
  if (!handle) return MIHS_ERR_INVALID;
  *handle = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return MIHS_ERR_HIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return MIHS_ERR_HIP;
  if (!prop.cooperativeLaunch) return MIHS_ERR_UNSUPPORTED;
  int wall_khz = 0;
  if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess)
    wall_khz = 0;
  mihs_handle* h = new (std::nothrow) mihs_handle();
  if (!h) return MIHS_ERR_INVALID;
  h->device = device;
  h->num_cu = prop.multiProcessorCount;
  h->wall_khz = wall_khz;
  strncpy(h->arch, prop.gcnArchName, sizeof(h->arch) - 1);
  for (int k = 0; k < mihs::kXcds; ++k) h->row_weight[k] = mihs::kRowWeightMax;
  // this device's address of the static scratch of mihs_solve_noalloc, taken
  // once here with the device current (the caller's current device is kept)
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) {
    delete h;
    return MIHS_ERR_HIP;
  }
  const int rc = mihs::noalloc_scratch_address(&h->noalloc_scratch);
  if (hipSetDevice(prev) != hipSuccess || rc != MIHS_OK) {
    delete h;
    return MIHS_ERR_HIP;
  }
  *handle = h;
  return MIHS_OK;
}

int mihs_calibrate_rows(mihs_handle_t handle, int32_t* weights) {
  if (!handle) return MIHS_ERR_INVALID;
  const int rc = mihs::calibrate_rows(handle);
  if (rc == MIHS_OK && weights)
    for (int k = 0; k < mihs::kXcds; ++k) weights[k] = handle->row_weight[k];
  return rc;
}

int mihs_destroy(mihs_handle_t handle) {
  delete handle;
  return MIHS_OK;
}

const char* mihs_status_string(int code) {
  switch (code) {
    case MIHS_OK: return "ok / converged";
    case MIHS_MAX_ITER: return "maximum outer iterations reached";
    case MIHS_ERR_INVALID: return "invalid argument";
    case MIHS_ERR_WORKSPACE: return "workspace too small";
    case MIHS_ERR_HIP: return "HIP runtime error";
    case MIHS_ERR_UNSUPPORTED: return "unsupported combination";
    case MIHS_BREAKDOWN: return "inner solve breakdown (non-positive curvature or NaN)";
    case MIHS_BARRIER_TIMEOUT: return "device-wide barrier timed out";
    default: return "unknown status";
  }
}

int mihs_sketch_workspace_size(mihs_handle_t handle, int64_t n, int64_t d, int64_t m, int64_t m2,
                               mihs_sketch_kind_t kind, mihs_dtype_t a_dtype,
                               mihs_precision_t precision, size_t* bytes) {
  if (!handle || !bytes || n <= 0 || d <= 0 || m <= 0) return MIHS_ERR_INVALID;
  *bytes = mihs::sketch_workspace_bytes(handle, n, d, m, m2, (int)kind, a_dtype == MIHS_F32,
                                        precision == MIHS_MIXED);
  return MIHS_OK;
}

int mihs_sketch(mihs_handle_t handle, const void* A, mihs_dtype_t a_dtype, int64_t n, int64_t d,
                int64_t lda, mihs_sketch_kind_t kind, int64_t m, int64_t m2, uint32_t seed,
                mihs_precision_t precision, void* SA, int64_t ldsa, void* workspace,
                size_t ws_bytes, void* stream) {
  if (!handle) return MIHS_ERR_INVALID;
  const int a_f32 = a_dtype == MIHS_F32;
  const int mixed = precision == MIHS_MIXED;
  if (a_dtype != MIHS_F64 && a_dtype != MIHS_F32) return MIHS_ERR_INVALID;
  if (precision != MIHS_PLAIN_FP64 && precision != MIHS_MIXED) return MIHS_ERR_INVALID;
  if (!valid_matrix(A, n, d, lda, a_f32)) return MIHS_ERR_INVALID;
  if (m <= 0) return MIHS_ERR_INVALID;
  const int64_t rows_out = (kind == MIHS_COUNT_GAUSS) ? m2 : m;
  if (rows_out <= 0) return MIHS_ERR_INVALID;
  if (!valid_matrix(SA, rows_out, d, ldsa, mixed)) return MIHS_ERR_INVALID;
  switch (kind) {
    case MIHS_GAUSSIAN: break;
    case MIHS_SRHT:
      if ((n & (n - 1)) != 0) return MIHS_ERR_INVALID;
      break;
    case MIHS_COUNTSKETCH: break;
    case MIHS_COUNT_GAUSS:
      if (m2 <= 0) return MIHS_ERR_INVALID;
      break;
    default: return MIHS_ERR_INVALID;
  }
  if (hipSetDevice(handle->device) != hipSuccess) return MIHS_ERR_HIP;
  return mihs::launch_sketch(handle, A, a_f32, n, d, lda, (int)kind, m, m2, seed, mixed, SA, ldsa,
                             workspace, ws_bytes, as_stream(stream));
}

int mihs_solve_workspace_size(mihs_handle_t handle, int64_t n, int64_t d, int64_t m,
                              mihs_precision_t precision, size_t* bytes) {
  if (!handle || !bytes || n <= 0 || d <= 0 || m <= 0) return MIHS_ERR_INVALID;
  *bytes = mihs::solve_workspace_bytes(handle, n, d, m, precision == MIHS_MIXED);
  return MIHS_OK;
}

static int check_solve_common(const void* A, mihs_dtype_t a_dtype, int64_t n, int64_t d,
                              int64_t lda, double lambda, const void* SA, int64_t m, int64_t ldsa,
                              mihs_precision_t precision, double alpha, double beta,
                              double eps_sub, int64_t max_outer, int64_t max_inner) {
  if (a_dtype != MIHS_F64 && a_dtype != MIHS_F32) return MIHS_ERR_INVALID;
  if (precision != MIHS_PLAIN_FP64 && precision != MIHS_MIXED) return MIHS_ERR_INVALID;
  if (n < d) return MIHS_ERR_INVALID;
  if (!valid_matrix(A, n, d, lda, a_dtype == MIHS_F32)) return MIHS_ERR_INVALID;
  if (!valid_matrix(SA, m, d, ldsa, precision == MIHS_MIXED)) return MIHS_ERR_INVALID;
  if (!(lambda > 0.0) || !isfinite(lambda)) return MIHS_ERR_INVALID;
  if (!isfinite(alpha) || !isfinite(beta) || !(alpha > 0.0) || beta < 0.0 || beta >= 1.0)
    return MIHS_ERR_INVALID;
  if (!(eps_sub >= 0.0) || max_outer < 0 || max_inner < 1) return MIHS_ERR_INVALID;
  if (d > 4096) return MIHS_ERR_UNSUPPORTED;
  return MIHS_OK;
}

int mihs_solve(mihs_handle_t handle, const void* A, mihs_dtype_t a_dtype, int64_t n, int64_t d,
               int64_t lda, const double* b, double lambda, const void* SA, int64_t m,
               int64_t ldsa, mihs_precision_t precision, double alpha, double beta,
               double eps_sub, double tol, int64_t max_outer, int64_t max_inner, double* X,
               double* X_prev, mihs_info_t* d_info, void* workspace, size_t ws_bytes,
               void* stream) {
  return mihs_solve_inner(handle, A, a_dtype, n, d, lda, b, lambda, SA, m, ldsa, precision,
                          MIHS_INNER_CG, alpha, beta, eps_sub, tol, max_outer, max_inner, X,
                          X_prev, d_info, workspace, ws_bytes, stream);
}

int mihs_solve_noalloc(mihs_handle_t handle, const void* A, mihs_dtype_t a_dtype, int64_t n,
                       int64_t d, int64_t lda, const double* b, double lambda, const void* SA,
                       int64_t m, int64_t ldsa, mihs_precision_t precision, double alpha,
                       double beta, double eps_sub, double tol, int64_t max_outer,
                       int64_t max_inner, double* X, double* X_prev, mihs_info_t* d_info,
                       void* stream) {
  if (!handle || !handle->noalloc_scratch) return MIHS_ERR_INVALID;
  if (n <= 0 || d <= 0 || m <= 0) return MIHS_ERR_INVALID;
  if (precision != MIHS_PLAIN_FP64 && precision != MIHS_MIXED) return MIHS_ERR_INVALID;
  // the largest layout the solve could use at these sizes must fit the array
  if (mihs::solve_workspace_bytes(handle, n, d, m, precision == MIHS_MIXED) >
      mihs::kNoAllocScratchBytes)
    return MIHS_ERR_WORKSPACE;
  return mihs_solve_inner(handle, A, a_dtype, n, d, lda, b, lambda, SA, m, ldsa, precision,
                          MIHS_INNER_CG, alpha, beta, eps_sub, tol, max_outer, max_inner, X,
                          X_prev, d_info, handle->noalloc_scratch, mihs::kNoAllocScratchBytes,
                          stream);
}

int mihs_solve_inner(mihs_handle_t handle, const void* A, mihs_dtype_t a_dtype, int64_t n,
                     int64_t d, int64_t lda, const double* b, double lambda, const void* SA,
                     int64_t m, int64_t ldsa, mihs_precision_t precision, mihs_inner_t inner,
                     double alpha, double beta, double eps_sub, double tol, int64_t max_outer,
                     int64_t max_inner, double* X, double* X_prev, mihs_info_t* d_info,
                     void* workspace, size_t ws_bytes, void* stream) {
  if (!handle) return MIHS_ERR_INVALID;
  if (inner != MIHS_INNER_CG && inner != MIHS_INNER_AAB) return MIHS_ERR_INVALID;
  int rc = check_solve_common(A, a_dtype, n, d, lda, lambda, SA, m, ldsa, precision, alpha, beta,
                              eps_sub, max_outer, max_inner);
  if (rc) return rc;
  if (!b || !X || !d_info) return MIHS_ERR_INVALID;
  if (hipSetDevice(handle->device) != hipSuccess) return MIHS_ERR_HIP;
  mihs::SolveDesc s;
  s.A = A;
  s.a_f32 = a_dtype == MIHS_F32;
  s.n = n;
  s.d = d;
  s.lda = lda;
  s.b = b;
  s.rhs = nullptr;
  s.SA = SA;
  s.mixed = precision == MIHS_MIXED;
  s.m = m;
  s.ldsa = ldsa;
  s.lam = lambda;
  s.alpha = alpha;
  s.beta = beta;
  s.eps_sub = eps_sub;
  s.tol = tol;
  s.max_outer = max_outer;
  s.max_inner = max_inner;
  s.x = X;
  s.x_prev = X_prev;
  s.info = d_info;
  s.aab = inner == MIHS_INNER_AAB;
  return mihs::launch_solve(handle, s, workspace, ws_bytes, as_stream(stream));
}

int mihs_solve_dual_workspace_size(mihs_handle_t handle, int64_t n, int64_t d, int64_t m,
                                   mihs_precision_t precision, size_t* bytes) {
  if (!handle || !bytes || n <= 0 || d <= 0 || m <= 0) return MIHS_ERR_INVALID;
  // the iteration streams A^T (d x n): the tall solve with roles swapped
  *bytes = mihs::solve_workspace_bytes(handle, d, n, m, precision == MIHS_MIXED);
  return MIHS_OK;
}

int mihs_solve_dual(mihs_handle_t handle, const void* At, mihs_dtype_t a_dtype, int64_t n,
                    int64_t d, int64_t ldat, const double* b, double lambda, const void* SAt,
                    int64_t m, int64_t ldsa, mihs_precision_t precision, double alpha,
                    double beta, double eps_sub, double tol, int64_t max_outer,
                    int64_t max_inner, double* NU, double* X, mihs_info_t* d_info,
                    void* workspace, size_t ws_bytes, void* stream) {
  if (!handle) return MIHS_ERR_INVALID;
  // A^T is d x n with d >= n: the same checks as a tall solve on A^T
  int rc = check_solve_common(At, a_dtype, d, n, ldat, lambda, SAt, m, ldsa, precision, alpha,
                              beta, eps_sub, max_outer, max_inner);
  if (rc) return rc;
  if (!b || !NU || !X || !d_info) return MIHS_ERR_INVALID;
  if (hipSetDevice(handle->device) != hipSuccess) return MIHS_ERR_HIP;
  size_t need = 0;
  mihs_solve_dual_workspace_size(handle, n, d, m, precision, &need);
  if (!workspace || ws_bytes < need) return MIHS_ERR_WORKSPACE;
  hipStream_t st = as_stream(stream);
  // g = b - A A^T nu - lambda nu is the adjoint-form gradient of the tall
  // matrix A^T with right-hand side b and no data term
  mihs::SolveDesc s;
  s.A = At;
  s.a_f32 = a_dtype == MIHS_F32;
  s.n = d;
  s.d = n;
  s.lda = ldat;
  s.b = nullptr;
  s.rhs = b;
  s.SA = SAt;
  s.mixed = precision == MIHS_MIXED;
  s.m = m;
  s.ldsa = ldsa;
  s.lam = lambda;
  s.alpha = alpha;
  s.beta = beta;
  s.eps_sub = eps_sub;
  s.tol = tol;
  s.max_outer = max_outer;
  s.max_inner = max_inner;
  s.x = NU;
  s.x_prev = nullptr;
  s.info = d_info;
  rc = mihs::launch_solve(handle, s, workspace, ws_bytes, st);
  if (rc) return rc;
  // x = A^T nu (eq. (dual_relation)): rows of A^T times nu
  return mihs::launch_apply_rows(handle, At, a_dtype == MIHS_F32, d, n, ldat, NU, 1, X, 1, st);
}

static int check_pd(const void* A, mihs_dtype_t a_dtype, int64_t rows, int64_t cols,
                    int64_t lda, double lambda, const void* Q, int64_t m1, int64_t ldq,
                    const void* WQ, int64_t m2, int64_t ldwq, mihs_precision_t precision,
                    mihs_inner_t inner, double alpha1, double beta1, double alpha2, double beta2,
                    int64_t M, double eps_sub, int64_t max_outer, int64_t max_inner) {
  if (a_dtype != MIHS_F64 && a_dtype != MIHS_F32) return MIHS_ERR_INVALID;
  if (precision != MIHS_PLAIN_FP64 && precision != MIHS_MIXED) return MIHS_ERR_INVALID;
  if (inner != MIHS_INNER_CG && inner != MIHS_INNER_AAB) return MIHS_ERR_INVALID;
  const int mixed = precision == MIHS_MIXED;
  if (!valid_matrix(A, rows, cols, lda, a_dtype == MIHS_F32)) return MIHS_ERR_INVALID;
  if (!valid_matrix(Q, cols, m1, ldq, mixed)) return MIHS_ERR_INVALID;
  if (!valid_matrix(WQ, m2, m1, ldwq, mixed)) return MIHS_ERR_INVALID;
  if (!(lambda > 0.0) || !isfinite(lambda)) return MIHS_ERR_INVALID;
  for (double a : {alpha1, alpha2})
    if (!isfinite(a) || !(a > 0.0)) return MIHS_ERR_INVALID;
  for (double b : {beta1, beta2})
    if (!isfinite(b) || b < 0.0 || b >= 1.0) return MIHS_ERR_INVALID;
  if (M < 1 || !(eps_sub >= 0.0) || max_outer < 0 || max_inner < 1) return MIHS_ERR_INVALID;
  if (cols > 4096 || m1 > 4096) return MIHS_ERR_UNSUPPORTED;
  return MIHS_OK;
}

static mihs::PdDesc pd_desc(const void* A, mihs_dtype_t a_dtype, int64_t rows, int64_t cols,
                            int64_t lda, const double* c, const double* rhs, double lambda,
                            const void* Q, int64_t m1, int64_t ldq, const void* WQ, int64_t m2,
                            int64_t ldwq, mihs_precision_t precision, mihs_inner_t inner,
                            double alpha1, double beta1, double alpha2, double beta2, int64_t M,
                            double eps_sub, double tol, int64_t max_outer, int64_t max_inner,
                            double* x, mihs_info_t* info) {
  mihs::PdDesc p;
  p.A = A;
  p.a_f32 = a_dtype == MIHS_F32;
  p.rows = rows;
  p.cols = cols;
  p.lda = lda;
  p.c = c;
  p.rhs = rhs;
  p.Q = Q;
  p.m1 = m1;
  p.ldq = ldq;
  p.WQ = WQ;
  p.m2 = m2;
  p.ldwq = ldwq;
  p.mixed = precision == MIHS_MIXED;
  p.aab = inner == MIHS_INNER_AAB;
  p.lam = lambda;
  p.alpha1 = alpha1;
  p.beta1 = beta1;
  p.alpha2 = alpha2;
  p.beta2 = beta2;
  p.eps_sub = eps_sub;
  p.tol = tol;
  p.M = M;
  p.max_outer = max_outer;
  p.max_inner = max_inner;
  p.x = x;
  p.info = info;
  return p;
}

int mihs_solve_pd_workspace_size(mihs_handle_t handle, int64_t n, int64_t d, int64_t m1,
                                 int64_t m2, mihs_precision_t precision, size_t* bytes) {
  if (!handle || !bytes || n <= 0 || d <= 0 || m1 <= 0 || m2 <= 0) return MIHS_ERR_INVALID;
  *bytes = mihs::pd_workspace_bytes(handle, n, d, m1, m2, precision == MIHS_MIXED);
  return MIHS_OK;
}

int mihs_solve_pd(mihs_handle_t handle, const void* A, mihs_dtype_t a_dtype, int64_t n,
                  int64_t d, int64_t lda, const double* b, double lambda, const void* Q,
                  int64_t m1, int64_t ldq, const void* WQ, int64_t m2, int64_t ldwq,
                  mihs_precision_t precision, mihs_inner_t inner, double alpha1, double beta1,
                  double alpha2, double beta2, int64_t M, double eps_sub, double tol,
                  int64_t max_outer, int64_t max_inner, double* X, mihs_info_t* d_info,
                  void* workspace, size_t ws_bytes, void* stream) {
  if (!handle) return MIHS_ERR_INVALID;
  if (n < d) return MIHS_ERR_INVALID;
  const int rc = check_pd(A, a_dtype, n, d, lda, lambda, Q, m1, ldq, WQ, m2, ldwq, precision,
                          inner, alpha1, beta1, alpha2, beta2, M, eps_sub, max_outer, max_inner);
  if (rc) return rc;
  if (!b || !X || !d_info) return MIHS_ERR_INVALID;
  if (hipSetDevice(handle->device) != hipSuccess) return MIHS_ERR_HIP;
  // g = A^T (b - A x) - lambda x: the ridge form of the gradient pass
  const mihs::PdDesc p = pd_desc(A, a_dtype, n, d, lda, b, nullptr, lambda, Q, m1, ldq, WQ, m2,
                                 ldwq, precision, inner, alpha1, beta1, alpha2, beta2, M,
                                 eps_sub, tol, max_outer, max_inner, X, d_info);
  return mihs::launch_pd(handle, p, workspace, ws_bytes, as_stream(stream));
}

int mihs_solve_pd_dual_workspace_size(mihs_handle_t handle, int64_t n, int64_t d, int64_t m1,
                                      int64_t m2, mihs_precision_t precision, size_t* bytes) {
  if (!handle || !bytes || n <= 0 || d <= 0 || m1 <= 0 || m2 <= 0) return MIHS_ERR_INVALID;
  // the outer pass streams A^T (d x n) for the n-dimensional dual variable
  *bytes = mihs::pd_workspace_bytes(handle, d, n, m1, m2, precision == MIHS_MIXED);
  return MIHS_OK;
}

int mihs_solve_pd_dual(mihs_handle_t handle, const void* At, mihs_dtype_t a_dtype, int64_t n,
                       int64_t d, int64_t ldat, const double* b, double lambda, const void* Q,
                       int64_t m1, int64_t ldq, const void* WQ, int64_t m2, int64_t ldwq,
                       mihs_precision_t precision, mihs_inner_t inner, double alpha1,
                       double beta1, double alpha2, double beta2, int64_t M, double eps_sub,
                       double tol, int64_t max_outer, int64_t max_inner, double* NU, double* X,
                       mihs_info_t* d_info, void* workspace, size_t ws_bytes, void* stream) {
  if (!handle) return MIHS_ERR_INVALID;
  if (n > d) return MIHS_ERR_INVALID;
  int rc = check_pd(At, a_dtype, d, n, ldat, lambda, Q, m1, ldq, WQ, m2, ldwq, precision, inner,
                    alpha1, beta1, alpha2, beta2, M, eps_sub, max_outer, max_inner);
  if (rc) return rc;
  if (!b || !NU || !X || !d_info) return MIHS_ERR_INVALID;
  if (hipSetDevice(handle->device) != hipSuccess) return MIHS_ERR_HIP;
  hipStream_t st = as_stream(stream);
  // g = b - A A^T nu - lambda nu: the right-hand-side form of the pass over A^T
  const mihs::PdDesc p = pd_desc(At, a_dtype, d, n, ldat, nullptr, b, lambda, Q, m1, ldq, WQ, m2,
                                 ldwq, precision, inner, alpha1, beta1, alpha2, beta2, M,
                                 eps_sub, tol, max_outer, max_inner, NU, d_info);
  rc = mihs::launch_pd(handle, p, workspace, ws_bytes, st);
  if (rc) return rc;
  // x = A^T nu (eq. (dual_relation))
  return mihs::launch_apply_rows(handle, At, a_dtype == MIHS_F32, d, n, ldat, NU, 1, X, 1, st);
}

int mihs_transpose(mihs_handle_t handle, const void* src, mihs_dtype_t dtype, int64_t rows,
                   int64_t cols, int64_t lds, void* dst, int64_t ldd, void* stream) {
  if (!handle || !src || !dst || rows <= 0 || cols <= 0) return MIHS_ERR_INVALID;
  if (dtype != MIHS_F64 && dtype != MIHS_F32) return MIHS_ERR_INVALID;
  if (lds < cols || ldd < rows) return MIHS_ERR_INVALID;
  if (hipSetDevice(handle->device) != hipSuccess) return MIHS_ERR_HIP;
  return mihs::launch_transpose(src, dtype == MIHS_F32, rows, cols, lds, dst, ldd,
                                as_stream(stream));
}

int mihs_estimate_sd_workspace_size(mihs_handle_t handle, int64_t m, int64_t d, int64_t T,
                                    mihs_precision_t precision, size_t* bytes) {
  if (!handle || !bytes || m <= 0 || d <= 0 || T <= 0) return MIHS_ERR_INVALID;
  *bytes = mihs::estimate_workspace_bytes(handle, m, d, T, precision == MIHS_MIXED);
  return MIHS_OK;
}

int mihs_estimate_sd(mihs_handle_t handle, const void* SA, int64_t m, int64_t d, int64_t ldsa,
                     mihs_precision_t precision, mihs_inner_t inner, double lambda, int64_t T,
                     uint32_t seed, double eps_tr, int64_t max_inner, double* sd, double* Z,
                     mihs_info_t* d_info, void* workspace, size_t ws_bytes, void* stream) {
  if (!handle) return MIHS_ERR_INVALID;
  if (inner != MIHS_INNER_CG && inner != MIHS_INNER_AAB) return MIHS_ERR_INVALID;
  if (precision != MIHS_PLAIN_FP64 && precision != MIHS_MIXED) return MIHS_ERR_INVALID;
  const int mixed = precision == MIHS_MIXED;
  if (!valid_matrix(SA, m, d, ldsa, mixed)) return MIHS_ERR_INVALID;
  if (!(lambda > 0.0) || !isfinite(lambda)) return MIHS_ERR_INVALID;
  if (T < 1 || T > (int64_t)1 << 20 || !(eps_tr >= 0.0) || !isfinite(eps_tr) || max_inner < 1)
    return MIHS_ERR_INVALID;
  if (!sd || !d_info) return MIHS_ERR_INVALID;
  if (d > 4096) return MIHS_ERR_UNSUPPORTED;
  if (hipSetDevice(handle->device) != hipSuccess) return MIHS_ERR_HIP;
  return mihs::launch_estimate_sd(handle, SA, m, d, ldsa, mixed, inner == MIHS_INNER_AAB,
                                  lambda, T, seed, eps_tr, max_inner, sd, Z, d_info, workspace,
                                  ws_bytes, as_stream(stream));
}

static size_t backward_ws_bytes(mihs_handle_t handle, int64_t n, int64_t d, int64_t m,
                                int64_t k, int mixed) {
  const size_t params = align_up(3 * 16 * sizeof(double), 256);
  if (d <= mihs::block_max_d()) {
    std::vector<mihs::BlockEntryDesc> ents((size_t)((k + 15) / 16));
    for (auto& e : ents) {
      e.n = n;
      e.d = d;
      e.m = m;
      e.ncols = 16;
      e.sa_group = 0;
    }
    return params + mihs::block_workspace_bytes(handle, ents.data(), (int64_t)ents.size());
  }
  return params + mihs::solve_workspace_bytes(handle, n, d, m, mixed) +
         2 * align_up((size_t)d * sizeof(double), 256);
}

int mihs_solve_backward_workspace_size(mihs_handle_t handle, int64_t n, int64_t d, int64_t m,
                                       int64_t k, mihs_precision_t precision, size_t* bytes) {
  if (!handle || !bytes || n <= 0 || d <= 0 || m <= 0 || k < 1) return MIHS_ERR_INVALID;
  *bytes = backward_ws_bytes(handle, n, d, m, k, precision == MIHS_MIXED);
  return MIHS_OK;
}

int mihs_solve_backward(mihs_handle_t handle, const void* A, mihs_dtype_t a_dtype, int64_t n,
                        int64_t d, int64_t lda, const void* SA, int64_t m, int64_t ldsa,
                        double lambda, mihs_precision_t precision, const double* Xstar,
                        const double* Gbar, int64_t k, double alpha, double beta,
                        double eps_sub, double tol, int64_t max_outer, int64_t max_inner,
                        double* W, double* dB, double* dlambda, double* dloglambda,
                        mihs_info_t* d_info, void* workspace, size_t ws_bytes, void* stream) {
  if (!handle) return MIHS_ERR_INVALID;
  int rc = check_solve_common(A, a_dtype, n, d, lda, lambda, SA, m, ldsa, precision, alpha, beta,
                              eps_sub, max_outer, max_inner);
  if (rc) return rc;
  if (!Xstar || !Gbar || !W || !dlambda || !d_info || k < 1) return MIHS_ERR_INVALID;
  if (hipSetDevice(handle->device) != hipSuccess) return MIHS_ERR_HIP;
  const int mixed = precision == MIHS_MIXED;
  if (!workspace || ws_bytes < backward_ws_bytes(handle, n, d, m, k, mixed))
    return MIHS_ERR_WORKSPACE;
  hipStream_t st = as_stream(stream);
  char* base = (char*)workspace;
  const size_t params = align_up(3 * 16 * sizeof(double), 256);
  // The adjoint systems (A^T A + lambda I) w_j = gbar_j share A, SA and lambda:
  // M-IHS from w = 0 with gradient gbar_j - A^T A w_j - lambda w_j.
  rc = mihs::launch_fill(W, 0.0, d * k, st);
  if (rc) return rc;
  if (d <= mihs::block_max_d()) {
    double* pl = (double*)base;
    rc = mihs::launch_fill(pl, lambda, 16, st);
    if (!rc) rc = mihs::launch_fill(pl + 16, alpha, 16, st);
    if (!rc) rc = mihs::launch_fill(pl + 32, beta, 16, st);
    if (rc) return rc;
    std::vector<mihs::BlockEntryDesc> ents;
    for (int64_t g0 = 0; g0 < k; g0 += 16) {
      mihs::BlockEntryDesc e;
      e.A = A;
      e.n = n;
      e.d = d;
      e.lda = lda;
      e.B = nullptr;
      e.ldb = 0;
      e.ldbc = 0;
      e.RHS = Gbar + g0;
      e.ldr = k;
      e.SA = SA;
      e.m = m;
      e.ldsa = ldsa;
      e.X = W + g0;
      e.ldx = k;
      e.lam = pl;
      e.alpha = pl + 16;
      e.beta = pl + 32;
      e.info = d_info + g0;
      e.ncols = (int)((k - g0) < 16 ? (k - g0) : 16);
      e.sa_group = 0;
      ents.push_back(e);
    }
    rc = mihs::launch_block(handle, ents.data(), (int64_t)ents.size(), a_dtype == MIHS_F32, mixed,
                            eps_sub, tol, max_outer, max_inner, base + params, ws_bytes - params,
                            st);
    if (rc) return rc;
  } else {
    // wide problems: one single-column solve per right-hand side
    const size_t solve_ws = mihs::solve_workspace_bytes(handle, n, d, m, mixed);
    const size_t col_bytes = align_up((size_t)d * sizeof(double), 256);
    char* wsp = base + params;
    double* g_col = (double*)(wsp + solve_ws);
    double* w_col = (double*)(wsp + solve_ws + col_bytes);
    for (int64_t j = 0; j < k; ++j) {
      if (hipMemcpy2DAsync(g_col, sizeof(double), Gbar + j, (size_t)k * sizeof(double),
                           sizeof(double), (size_t)d, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return MIHS_ERR_HIP;
      rc = mihs::launch_fill(w_col, 0.0, d, st);
      if (rc) return rc;
      mihs::SolveDesc s;
      s.A = A;
      s.a_f32 = a_dtype == MIHS_F32;
      s.n = n;
      s.d = d;
      s.lda = lda;
      s.b = nullptr;
      s.rhs = g_col;
      s.SA = SA;
      s.mixed = mixed;
      s.m = m;
      s.ldsa = ldsa;
      s.lam = lambda;
      s.alpha = alpha;
      s.beta = beta;
      s.eps_sub = eps_sub;
      s.tol = tol;
      s.max_outer = max_outer;
      s.max_inner = max_inner;
      s.x = w_col;
      s.x_prev = nullptr;
      s.info = d_info + j;
      rc = mihs::launch_solve(handle, s, wsp, solve_ws, st);
      if (rc) return rc;
      if (hipMemcpy2DAsync(W + j, (size_t)k * sizeof(double), w_col, sizeof(double),
                           sizeof(double), (size_t)d, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return MIHS_ERR_HIP;
    }
  }
  if (dB) {
    rc = mihs::launch_apply_rows(handle, A, a_dtype == MIHS_F32, n, d, lda, W, k, dB, k, st);
    if (rc) return rc;
  }
  return mihs::launch_neg_dot(Xstar, W, d * k, lambda, dlambda, dloglambda, st);
}

int mihs_solve_multi_workspace_size(mihs_handle_t handle, int64_t n, int64_t d, int64_t m,
                                    int64_t k, mihs_precision_t precision, size_t* bytes) {
  if (!handle || !bytes || n <= 0 || d <= 0 || m <= 0 || k < 1) return MIHS_ERR_INVALID;
  (void)precision;
  std::vector<mihs::BlockEntryDesc> ents((size_t)((k + 15) / 16));
  for (auto& e : ents) {
    e.n = n;
    e.d = d;
    e.m = m;
    e.ncols = 16;
    e.sa_group = 0;
  }
  *bytes = align_up(3 * 16 * sizeof(double), 256) +
           mihs::block_workspace_bytes(handle, ents.data(), (int64_t)ents.size());
  return MIHS_OK;
}

int mihs_solve_multi(mihs_handle_t handle, const void* A, mihs_dtype_t a_dtype, int64_t n,
                     int64_t d, int64_t lda, const double* B, int64_t k, int64_t ldb,
                     double lambda, const void* SA, int64_t m, int64_t ldsa,
                     mihs_precision_t precision, double alpha, double beta, double eps_sub,
                     double tol, int64_t max_outer, int64_t max_inner, double* X,
                     mihs_info_t* d_info, void* workspace, size_t ws_bytes, void* stream) {
  if (!handle) return MIHS_ERR_INVALID;
  int rc = check_solve_common(A, a_dtype, n, d, lda, lambda, SA, m, ldsa, precision, alpha, beta,
                              eps_sub, max_outer, max_inner);
  if (rc) return rc;
  if (!B || !X || !d_info || k < 1 || ldb < k) return MIHS_ERR_INVALID;
  if (d > mihs::block_max_d()) return MIHS_ERR_UNSUPPORTED;
  size_t need = 0;
  mihs_solve_multi_workspace_size(handle, n, d, m, k, precision, &need);
  if (!workspace || ws_bytes < need) return MIHS_ERR_WORKSPACE;
  if (hipSetDevice(handle->device) != hipSuccess) return MIHS_ERR_HIP;
  hipStream_t st = as_stream(stream);
  char* base = (char*)workspace;
  const size_t params = align_up(3 * 16 * sizeof(double), 256);
  double* pl = (double*)base;
  rc = mihs::launch_fill(pl, lambda, 16, st);
  if (!rc) rc = mihs::launch_fill(pl + 16, alpha, 16, st);
  if (!rc) rc = mihs::launch_fill(pl + 32, beta, 16, st);
  if (rc) return rc;
  std::vector<mihs::BlockEntryDesc> ents;
  for (int64_t g0 = 0; g0 < k; g0 += 16) {
    mihs::BlockEntryDesc e;
    e.A = A;
    e.n = n;
    e.d = d;
    e.lda = lda;
    e.B = B + g0;
    e.ldb = ldb;
    e.ldbc = 1;
    e.RHS = nullptr;
    e.ldr = 0;
    e.SA = SA;
    e.m = m;
    e.ldsa = ldsa;
    e.X = X + g0;
    e.ldx = k;
    e.lam = pl;
    e.alpha = pl + 16;
    e.beta = pl + 32;
    e.info = d_info + g0;
    e.ncols = (int)((k - g0) < 16 ? (k - g0) : 16);
    e.sa_group = 0;
    ents.push_back(e);
  }
  return mihs::launch_block(handle, ents.data(), (int64_t)ents.size(), a_dtype == MIHS_F32,
                            precision == MIHS_MIXED, eps_sub, tol, max_outer, max_inner,
                            base + params, ws_bytes - params, st);
}

static void batched_entries(const mihs_problem_t* hp, int64_t nprob, const double* lambdas,
                            const double* alphas, const double* betas, int64_t nlam,
                            std::vector<mihs::BlockEntryDesc>* out) {
  out->clear();
  for (int64_t p = 0; p < nprob; ++p) {
    for (int64_t g0 = 0; g0 < nlam; g0 += 16) {
      mihs::BlockEntryDesc e;
      e.A = hp[p].A;
      e.n = hp[p].n;
      e.d = hp[p].d;
      e.lda = hp[p].lda;
      e.B = hp[p].b;  // one b shared by every lambda
      e.ldb = 1;
      e.ldbc = 0;
      e.RHS = nullptr;
      e.ldr = 0;
      e.SA = hp[p].SA;
      e.m = hp[p].m;
      e.ldsa = hp[p].ldsa;
      e.X = hp[p].X + g0;
      e.ldx = nlam;
      e.lam = lambdas ? lambdas + p * nlam + g0 : nullptr;
      e.alpha = alphas ? alphas + p * nlam + g0 : nullptr;
      e.beta = betas ? betas + p * nlam + g0 : nullptr;
      e.info = hp[p].info + g0;
      e.ncols = (int)((nlam - g0) < 16 ? (nlam - g0) : 16);
      e.sa_group = p;  // the lambda-path of one problem shares its sketch
      out->push_back(e);
    }
  }
}

int mihs_solve_batched_workspace_size(mihs_handle_t handle, const mihs_problem_t* h_problems,
                                      int64_t nprob, int64_t nlam, mihs_precision_t precision,
                                      size_t* bytes) {
  if (!handle || !h_problems || !bytes || nprob < 1 || nlam < 1) return MIHS_ERR_INVALID;
  (void)precision;
  std::vector<mihs::BlockEntryDesc> ents;
  batched_entries(h_problems, nprob, nullptr, nullptr, nullptr, nlam, &ents);
  *bytes = mihs::block_workspace_bytes(handle, ents.data(), (int64_t)ents.size());
  return MIHS_OK;
}

static int check_batched(mihs_handle_t handle, const mihs_problem_t* h_problems, int64_t nprob,
                         const double* lambdas, const double* alphas, const double* betas,
                         int64_t nlam, mihs_precision_t precision, double eps_sub,
                         int64_t max_outer, int64_t max_inner) {
  if (!handle || !h_problems || nprob < 1 || nlam < 1 || !lambdas || !alphas || !betas)
    return MIHS_ERR_INVALID;
  if (precision != MIHS_PLAIN_FP64 && precision != MIHS_MIXED) return MIHS_ERR_INVALID;
  if (!(eps_sub >= 0.0) || max_outer < 0 || max_inner < 1) return MIHS_ERR_INVALID;
  for (int64_t p = 0; p < nprob; ++p) {
    const mihs_problem_t& q = h_problems[p];
    if (q.n < q.d || !valid_matrix(q.A, q.n, q.d, q.lda, 0) || !q.b || !q.X || !q.info)
      return MIHS_ERR_INVALID;
    if (!valid_matrix(q.SA, q.m, q.d, q.ldsa, precision == MIHS_MIXED)) return MIHS_ERR_INVALID;
    if (q.d > mihs::block_max_d()) return MIHS_ERR_UNSUPPORTED;
  }
  if (hipSetDevice(handle->device) != hipSuccess) return MIHS_ERR_HIP;
  return MIHS_OK;
}

int mihs_solve_batched(mihs_handle_t handle, const mihs_problem_t* d_problems,
                       const mihs_problem_t* h_problems, int64_t nprob, const double* lambdas,
                       const double* alphas, const double* betas, int64_t nlam,
                       mihs_precision_t precision, double eps_sub, double tol,
                       int64_t max_outer, int64_t max_inner, void* workspace, size_t ws_bytes,
                       void* stream) {
  (void)d_problems;
  int rc = check_batched(handle, h_problems, nprob, lambdas, alphas, betas, nlam, precision,
                         eps_sub, max_outer, max_inner);
  if (rc) return rc;
  std::vector<mihs::BlockEntryDesc> ents;
  batched_entries(h_problems, nprob, lambdas, alphas, betas, nlam, &ents);
  return mihs::launch_block(handle, ents.data(), (int64_t)ents.size(), 0,
                            precision == MIHS_MIXED, eps_sub, tol, max_outer, max_inner, workspace,
                            ws_bytes, as_stream(stream));
}

}  // extern "C"

struct mihs_batched_plan {
  mihs::BlockPlan* plan;
  int device;
};

extern "C" {

int mihs_batched_plan_create(mihs_handle_t handle, const mihs_problem_t* h_problems,
                             int64_t nprob, const double* lambdas, const double* alphas,
                             const double* betas, int64_t nlam, mihs_precision_t precision,
                             double eps_sub, double tol, int64_t max_outer, int64_t max_inner,
                             const mihs_batched_tuning_t* tuning, void* workspace,
                             size_t ws_bytes, void* stream, mihs_batched_plan_t* plan) {
  if (!plan) return MIHS_ERR_INVALID;
  *plan = nullptr;
  int rc = check_batched(handle, h_problems, nprob, lambdas, alphas, betas, nlam, precision,
                         eps_sub, max_outer, max_inner);
  if (rc) return rc;
  if (tuning && !mihs::block_tuning_valid(*tuning)) return MIHS_ERR_INVALID;
  std::vector<mihs::BlockEntryDesc> ents;
  batched_entries(h_problems, nprob, lambdas, alphas, betas, nlam, &ents);
  const int64_t count = (int64_t)ents.size();
  std::vector<double> cost;
  mihs_batched_tuning_t tn = mihs::block_tuning_for(handle, ents.data(), count, &cost);
  if (tuning) tn = *tuning;  // (the measured costs still come from the handle)
  mihs::BlockPlan* P = nullptr;
  rc = mihs::plan_block(handle, ents.data(), count, 0, precision == MIHS_MIXED, eps_sub, tol,
                        max_outer, max_inner, tn, &cost, workspace, ws_bytes, as_stream(stream),
                        &P);
  if (rc) return rc;
  mihs_batched_plan* out = new (std::nothrow) mihs_batched_plan();
  if (!out) {
    mihs::free_block_plan(P);
    return MIHS_ERR_INVALID;
  }
  out->plan = P;
  out->device = handle->device;
  *plan = out;
  return MIHS_OK;
}

int mihs_batched_plan_run(mihs_batched_plan_t plan, void* stream) {
  if (!plan || !plan->plan) return MIHS_ERR_INVALID;
  if (hipSetDevice(plan->device) != hipSuccess) return MIHS_ERR_HIP;
  return mihs::run_block(plan->plan, as_stream(stream));
}

int mihs_batched_plan_destroy(mihs_batched_plan_t plan) {
  if (!plan) return MIHS_OK;
  mihs::free_block_plan(plan->plan);
  delete plan;
  return MIHS_OK;
}

int mihs_batched_cached_tuning(mihs_handle_t handle, const mihs_problem_t* h_problems,
                               int64_t nprob, int64_t nlam, mihs_batched_tuning_t* tuning) {
  if (!handle || !h_problems || !tuning || nprob < 1 || nlam < 1) return MIHS_ERR_INVALID;
  for (int64_t p = 0; p < nprob; ++p)
    if (h_problems[p].n < 1 || h_problems[p].d < 1 || h_problems[p].m < 1)
      return MIHS_ERR_INVALID;
  std::vector<mihs::BlockEntryDesc> ents;
  batched_entries(h_problems, nprob, nullptr, nullptr, nullptr, nlam, &ents);
  return mihs::block_tuning_lookup(handle, ents.data(), (int64_t)ents.size(), tuning)
             ? MIHS_OK
             : MIHS_ERR_UNSUPPORTED;
}

int mihs_tune_batched(mihs_handle_t handle, const mihs_problem_t* h_problems, int64_t nprob,
                      const double* lambdas, const double* alphas, const double* betas,
                      int64_t nlam, mihs_precision_t precision, double eps_sub, double tol,
                      int64_t trial_outer, int64_t measure_outer, int64_t max_inner,
                      int32_t allow_exact, void* workspace, size_t ws_bytes, void* stream,
                      mihs_batched_tuning_t* best, float* cand_ms, int32_t* ncand) {
  if (!best || trial_outer < 1 || measure_outer < 0) return MIHS_ERR_INVALID;
  if (allow_exact != 0 && allow_exact != 1) return MIHS_ERR_INVALID;
  int rc = check_batched(handle, h_problems, nprob, lambdas, alphas, betas, nlam, precision,
                         eps_sub, trial_outer, max_inner);
  if (rc) return rc;
  std::vector<mihs::BlockEntryDesc> ents;
  batched_entries(h_problems, nprob, lambdas, alphas, betas, nlam, &ents);
  const int64_t count = (int64_t)ents.size();
  hipStream_t st = as_stream(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return MIHS_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return MIHS_ERR_HIP;
  }
  int n_tried = 0;
  // one timed trial from X = 0
  auto trial = [&](const mihs_batched_tuning_t& tn, float* ms,
                   const std::vector<double>* cost = nullptr, int64_t outer = 0) -> int {
    for (int64_t p = 0; p < nprob; ++p) {
      const int r = mihs::launch_fill(h_problems[p].X, 0.0, h_problems[p].d * nlam, st);
      if (r) return r;
    }
    mihs::BlockPlan* P = nullptr;
    int r = mihs::plan_block(handle, ents.data(), count, 0, precision == MIHS_MIXED, eps_sub,
                             tol, outer > 0 ? outer : trial_outer, max_inner, tn, cost,
                             workspace, ws_bytes, st, &P);
    if (r) return r;
    if (hipEventRecord(e0, st) != hipSuccess) r = MIHS_ERR_HIP;
    if (!r) r = mihs::run_block(P, st);
    if (!r && hipEventRecord(e1, st) != hipSuccess) r = MIHS_ERR_HIP;
    if (!r && hipEventSynchronize(e1) != hipSuccess) r = MIHS_ERR_HIP;
    if (!r && hipEventElapsedTime(ms, e0, e1) != hipSuccess) r = MIHS_ERR_HIP;
    mihs::free_block_plan(P);
    if (!r && n_tried < MIHS_TUNE_MAX_CANDIDATES) {
      if (cand_ms) cand_ms[n_tried] = *ms;
      ++n_tried;
    }
    return r;
  };
  mihs_batched_tuning_t cur;
  mihs_batched_default_tuning(&cur);
  float cur_ms = 0.0f;
  rc = trial(cur, &cur_ms);
  // coordinate descent: inner_weight, then cg_cols, then a_dma
  const double weights[] = {6.25, 25.0, 400.0};
  for (double w : weights) {
    if (rc) break;
    mihs_batched_tuning_t t = cur;
    t.inner_weight = w;
    float ms = 0.0f;
    rc = trial(t, &ms);
    if (!rc && ms < cur_ms) {
      cur = t;
      cur_ms = ms;
    }
  }
  mihs_batched_tuning_t base = cur;
  const int cols[] = {16, 64, 512};
  for (int c : cols) {
    if (rc) break;
    mihs_batched_tuning_t t = base;
    t.cg_cols = c;
    float ms = 0.0f;
    rc = trial(t, &ms);
    if (!rc && ms < cur_ms) {
      cur = t;
      cur_ms = ms;
    }
  }
  if (!rc) {
    mihs_batched_tuning_t t = cur;
    t.a_dma = 0;
    float ms = 0.0f;
    rc = trial(t, &ms);
    if (!rc && ms < cur_ms) {
      cur = t;
      cur_ms = ms;
    }
  }
  // exact sub-solves (one Cholesky factor per column, formed in the launch),
  // teams sized for a sub-solve worth a few to a few tens of passes over H;
  // the short trials charge the factorizations to few outer iterations, so
  // the best exact shape is kept apart and compared over full runs below
  mihs_batched_tuning_t ex = cur;
  float ex_ms = 0.0f;
  const double exact_weights[] = {6.25, 25.0};
  for (int wi = 0; wi < 2 && !rc && allow_exact; ++wi) {
    mihs_batched_tuning_t t = cur;
    t.exact = 1;
    t.inner_weight = exact_weights[wi];
    float ms = 0.0f;
    rc = trial(t, &ms);
    if (!rc && (wi == 0 || ms < ex_ms)) {
      ex = t;
      ex_ms = ms;
    }
  }
  if (!rc && allow_exact && measure_outer == 0 && ex_ms < cur_ms) {
    cur = ex;
    cur_ms = ex_ms;
  }
  // measured costs: every entry's wall time in a full run times its team
  // size.  The best inexact and the best exact shape both run; the faster
  // one's costs then size a schedule, run for as long.
  std::vector<double> cost;
  if (!rc && measure_outer > 0) {
    auto full_run = [&](const mihs_batched_tuning_t& tn, float* ms,
                        std::vector<double>* c) -> int {
      std::vector<int> tsz;
      int r = mihs::block_team_sizes(handle, ents.data(), count, tn, nullptr, &tsz);
      if (!r) r = trial(tn, ms, nullptr, measure_outer);
      if (r) return r;
      c->resize(count);
      for (int64_t i = 0; i < count; ++i) {
        mihs_info_t rec;
        if (hipMemcpy(&rec, ents[i].info, sizeof(rec), hipMemcpyDeviceToHost) != hipSuccess)
          return MIHS_ERR_HIP;
        (*c)[i] = (double)rec.elapsed_us * tsz[i];
      }
      return MIHS_OK;
    };
    rc = full_run(cur, &cur_ms, &cost);
    if (!rc && allow_exact) {
      std::vector<double> ex_cost;
      float full_ex = 0.0f;
      rc = full_run(ex, &full_ex, &ex_cost);
      if (!rc && full_ex < cur_ms) {
        cur = ex;
        cur_ms = full_ex;
        cost.swap(ex_cost);
      }
    }
    // measured schedules: a run of each, keeping the fastest with the costs
    // it was sized from and the per-problem costs it measured in turn
    std::vector<double> used_cost, next_cost;
    auto run_measured = [&](const mihs_batched_tuning_t& t,
                            const std::vector<double>& c) -> int {
      float mms = 0.0f;
      int r = trial(t, &mms, &c, measure_outer);
      if (r || !(mms < cur_ms)) return r;
      std::vector<int> tsz;
      r = mihs::block_team_sizes(handle, ents.data(), count, t, &c, &tsz);
      if (r) return r;
      std::vector<double> nc(count);
      for (int64_t i = 0; i < count; ++i) {
        mihs_info_t rec;
        if (hipMemcpy(&rec, ents[i].info, sizeof(rec), hipMemcpyDeviceToHost) != hipSuccess)
          return MIHS_ERR_HIP;
        nc[i] = (double)rec.elapsed_us * tsz[i];
      }
      cur = t;
      cur_ms = mms;
      used_cost = c;
      next_cost.swap(nc);
      return MIHS_OK;
    };
    if (!rc) {
      mihs_batched_tuning_t t = cur;
      t.measured = 1;
      const mihs_batched_tuning_t base_measured = t;
      rc = run_measured(t, cost);
      // the measured schedule gives the costliest problems teams; with 64
      // columns per member their inner CG splits over the whole team too
      if (!rc && !base_measured.exact && base_measured.cg_cols != 64) {
        t = base_measured;
        t.cg_cols = 64;
        rc = run_measured(t, cost);
      }
      // the costs came from a run in which most problems ran alone; a team
      // does not run its problem tsize times faster, so size the schedule
      // again from the times measured under the best measured schedule, up to
      // three times while that still gains more than 2%
      for (int round = 0; round < 3 && !rc && cur.measured; ++round) {
        const float before = cur_ms;
        rc = run_measured(cur, std::vector<double>(next_cost));
        if (!(cur_ms < 0.98f * before)) break;
      }
      if (cur.measured) cost = used_cost;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (ncand) *ncand = n_tried;
  if (rc) return rc;
  *best = cur;
  mihs::block_tuning_store(handle, ents.data(), count, cur,
                           cur.measured ? cost : std::vector<double>());
  return MIHS_OK;
}

}  // extern "C"
