/*
 * mihs.h - C ABI of libmihs, an MI355X (gfx950) implementation of Momentum
 * Iterative Hessian Sketch (M-IHS) for tall ridge regression
 *
 *     x* = argmin_x  1/2 ||A x - b||^2 + lambda/2 ||x||^2,   A is n x d, n >= d
 *
 * (Ozaslan, Pilanci, Arikan, "M-IHS: Momentum Iterative Hessian Sketch",
 * arXiv:1912.03514; Section 1 eq. (intro), Section 3 eq. (mihs1), Algorithm 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All matrices are row-major.  `lda`/`ldsa`/`ldb` count elements between
 *   consecutive rows and must be >= the row length.  Matrix base pointers must
 *   be 16-byte aligned and the leading dimension a multiple of 16 bytes / the
 *   element size (2 for double, 4 for float); this keeps every row 16-byte
 *   aligned for vector loads.
 * - Pointers documented as "device" must point to device memory of the handle's
 *   GPU; "host" pointers to host memory.  The caller owns every buffer; the
 *   library allocates nothing inside mihs_sketch / mihs_solve /
 *   mihs_solve_batched / mihs_solve_backward (scratch comes from the
 *   caller's `workspace`, whose size the *_workspace_size queries return).
 * - Every call is asynchronous on `stream` (a hipStream_t; NULL = the default
 *   stream).  The return value reports argument and launch errors only:
 *       MIHS_OK (0), MIHS_ERR_INVALID (-1), MIHS_ERR_WORKSPACE (-2),
 *       MIHS_ERR_HIP (-3), MIHS_ERR_UNSUPPORTED (-4).
 *   Numerical outcomes are written to a device-side mihs_info_t, readable after
 *   the stream synchronises: status MIHS_CONVERGED (0), MIHS_MAX_ITER (1,
 *   result still usable), MIHS_BREAKDOWN (-5: non-positive curvature or NaN in
 *   the inner solve), MIHS_BARRIER_TIMEOUT (-6: the solver's device-wide
 *   barrier gave up waiting; the result is invalid).
 * - Calls that overlap on one workspace race; use one workspace per stream.
 */
#ifndef MIHS_H_
#define MIHS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mihs_handle* mihs_handle_t;

typedef enum { MIHS_F64 = 0, MIHS_F32 = 1 } mihs_dtype_t;

/* Sketch families of Lemma 3: (iv) Gaussian, (iii) SRHT, (i) CountSketch, and
 * CountSketch followed by a Gaussian second stage. */
typedef enum {
  MIHS_GAUSSIAN = 0,
  MIHS_SRHT = 1,
  MIHS_COUNTSKETCH = 2,
  MIHS_COUNT_GAUSS = 3
} mihs_sketch_kind_t;

/* PLAIN_FP64: sketch and inner solve in double.
 * MIXED: Gaussian stages use BF16 inputs with FP32 accumulation, SRHT and
 * CountSketch use FP32 arithmetic; SA is stored as float and the inner CG runs
 * in float.  The outer gradient A^T (b - A x) - lambda x is always FP64, so the
 * outer loop refines the inexact inner steps to full FP64 accuracy. */
typedef enum { MIHS_PLAIN_FP64 = 0, MIHS_MIXED = 1 } mihs_precision_t;

/* Inner solver of ((SA)^T SA + lambda I) z = g.
 * CG:  conjugate gradients from z = 0, stopped when ||r|| <= eps ||g||; applied
 *      through the Gram matrix (SA)^T SA when m >= d, else by streaming SA.
 * AAB: AAb_Solver (Algorithm 6, Section 3.5): Golub-Kahan bidiagonalisation of
 *      SA started from g, with the sqrt(lambda) I block folded in by Givens
 *      rotations; stopped when its residual estimate |phi rhobar| / ||g|| falls
 *      below eps (the paper's stable alternative to CG on the explicit
 *      (SA)^T SA, Section 3.1).  Always streams SA (one pass per step). */
typedef enum { MIHS_INNER_CG = 0, MIHS_INNER_AAB = 1 } mihs_inner_t;

enum {
  MIHS_OK = 0,
  MIHS_ERR_INVALID = -1,
  MIHS_ERR_WORKSPACE = -2,
  MIHS_ERR_HIP = -3,
  MIHS_ERR_UNSUPPORTED = -4
};

enum {
  MIHS_CONVERGED = 0,
  MIHS_MAX_ITER = 1,
  MIHS_BREAKDOWN = -5,
  MIHS_BARRIER_TIMEOUT = -6
};

/* Device-side result record of one solve (one per right-hand side / lambda). */
typedef struct {
  int64_t outer_iters;        /* outer M-IHS iterations performed */
  int64_t inner_iters_total;  /* inner CG iterations summed over the solve */
  int64_t inner_iters_max;    /* largest inner CG count of one outer iteration */
  double rel_step;            /* last ||x^{i+1} - x^i|| / ||x^{i+1}|| */
  double grad_norm;           /* ||g|| at the last outer iteration */
  int32_t status;             /* MIHS_CONVERGED, MIHS_MAX_ITER, ... */
  int32_t elapsed_us;         /* batched and multi-RHS solves: wall time of the
                                 record's entry (its group of up to 16 columns)
                                 on its workgroups, in microseconds; 0 elsewhere */
} mihs_info_t;

/* Create a handle bound to HIP device `device` (it queries the CU count and
 * the cooperative-launch occupancy once).  Returns MIHS_ERR_HIP if the device
 * cannot be used. */
int mihs_create(mihs_handle_t* handle, int device);
int mihs_destroy(mihs_handle_t handle);

/* ------------------------------------------------------------------------
 * Row shares of the gradient pass (Algorithm 1: g = A^T (b - A x) - lambda x,
 * one pass over A per outer iteration).
 *
 * The calls that run the persistent solve kernel (mihs_solve,
 * mihs_solve_noalloc, mihs_solve_inner, mihs_solve_dual, mihs_solve_pd,
 * mihs_solve_pd_dual, mihs_estimate_sd, the per-column solves of
 * mihs_solve_backward) split the rows of A over their workgroups, which the device dispatches to its 8 XCDs in turn
 * (workgroup v on XCD v mod 8).  Workgroup v of G takes rows in proportion to
 * the weight w[v mod 8] of its XCD: rows [bound(v), bound(v + 1)) with
 * bound(v) = floor(n P(v) / P(G)), P(v) = sum of w[u mod 8] over u < v.  Equal
 * weights give the even split floor(n v / G).  XCDs need not stream from HBM
 * at the same rate; with equal shares the pass lasts as long as the slowest.
 * The weights belong to the handle (equal after mihs_create): every solve on
 * the handle uses them, so results repeat bit for bit on one handle; other
 * weights change the grouping of the partial sums, hence the rounding.
 *
 * mihs_calibrate_rows   times the gradient pass's row loop on every XCD, with
 *   one workgroup per CU and equal shares of a 2 GiB zero matrix (2048 FP64
 *   columns) that the call allocates and frees (6 warm-up and 15 timed
 *   passes, ~8 ms; synchronous), then sets
 *   w_k = 4 round(16 (t_min / t_k)^(3/4)) clamped to [32, 64] (t_k: the XCD's
 *   median over the passes of its workgroups' mean time; the power damps the correction, since slow XCDs speed up once
 *   fast ones finish; steps of 4 keep the 1-2% drift of the means between
 *   calibrations from moving the split).  weights (8 entries, may be NULL) receives the result.
 *   MIHS_ERR_HIP (weights unchanged) when the buffer cannot be allocated or a
 *   HIP call fails.  The Python binding calls it once per handle.
 * mihs_set_row_weights  sets the 8 weights, each in [1, 64]; NULL restores
 *   equal weights.  MIHS_ERR_INVALID for a weight out of range.  Solves read the
 *   weights when they are enqueued; changing them while another thread enqueues
 *   a solve on the same handle is not synchronised (any mix of old and new
 *   weights still gives a valid split).
 * mihs_get_row_weights  copies the handle's 8 weights to weights.
 * mihs_row_split        host only: bounds[0..G] of the split above for n rows
 *   over G workgroups (bounds[0] = 0, bounds[G] = n); MIHS_ERR_INVALID for
 *   n < 0, G < 1 or a weight out of [1, 64].
 * ------------------------------------------------------------------------ */
int mihs_calibrate_rows(mihs_handle_t handle, int32_t* weights);
int mihs_set_row_weights(mihs_handle_t handle, const int32_t* weights);
int mihs_get_row_weights(mihs_handle_t handle, int32_t* weights);
int mihs_row_split(int64_t n, int32_t G, const int32_t* weights, int64_t* bounds);

/* Human-readable text for a return code or an info status. */
const char* mihs_status_string(int code);

/* ------------------------------------------------------------------------
 * Momentum parameters of the heavy-ball iteration (host computations).
 *
 * mihs_momentum_cor4  Corollary 4: a sketch with m rows of a problem whose
 *   statistical dimension is sd (0 < sd < m) gives beta = sd / m and
 *   alpha = (1 - beta)^2, for which the iteration contracts at rate sqrt(beta).
 *   An over-estimate of sd keeps the rate bound (remark after Corollary 4).
 *   m is the number of rows of the sketch the solver sees (m2 for
 *   MIHS_COUNT_GAUSS).  Returns MIHS_ERR_INVALID unless 0 < sd < m, both
 *   finite, and alpha, beta are non-null.
 * mihs_momentum_thm1  Theorem 1: when the sketched Hessian satisfies the
 *   subspace-embedding bound with distortion eps (0 < eps < 1), the optimal
 *   momentum is beta* = (eps / (1 + sqrt(1 - eps^2)))^2 and step
 *   alpha* = (1 - beta*) sqrt(1 - eps^2), with rate sqrt(beta*).  Returns
 *   MIHS_ERR_INVALID unless 0 < eps < 1.
 * ------------------------------------------------------------------------ */
int mihs_momentum_cor4(double sd, int64_t m, double* alpha, double* beta);
int mihs_momentum_thm1(double eps, double* alpha, double* beta);

/* The regularisation parameter of the differentiable ridge layer, which is
 * parametrised by log(lambda) so that lambda stays positive:
 * *lambda = exp(log_lambda).  MIHS_ERR_INVALID if the result is not a finite
 * positive number or lambda is null. */
int mihs_lambda_from_log(double log_lambda, double* lambda);

/* ------------------------------------------------------------------------
 * Sketch:  SA = S A  (Algorithm 1's RP_fun; E[S^T S] = I, Section 3.1)
 *
 * A      device, n x d, dtype `a_dtype`, row stride lda.
 * kind   MIHS_GAUSSIAN:  S_ij = N(0,1)/sqrt(m) (Lemma 3(iv)); the N(0,1) draw of
 *          element (i, j) is Box-Muller on Philox-4x32-10 block (i*n+j)/4 with
 *          key (seed, 0) and stream 0.
 *        MIHS_SRHT:  S = (1/sqrt(m)) P H D (Lemma 3(iii)); n must be a power of
 *          two; D_ii = -1 iff bit 31 of murmur3_x86_32(i, seed); row k of P
 *          samples H's row murmur3_x86_32(k, seed + 0x9E3779B9) & (n-1), with
 *          replacement; H is the unnormalised Sylvester Walsh-Hadamard matrix.
 *        MIHS_COUNTSKETCH: row i of A is added with sign s(i) to row h(i) mod m
 *          of SA, h = murmur3_x86_32(i, seed), s(i) = -1 iff bit 31 of h
 *          (Lemma 3(i)); no scaling.
 *        MIHS_COUNT_GAUSS: CountSketch to m rows, then a Gaussian m2 x m stage
 *          (Philox stream 1, scale 1/sqrt(m2)).  The output has m2 rows.
 * precision  PLAIN_FP64: SA is double.  MIXED: SA is float (Gaussian stages:
 *          BF16 S and BF16 A, FP32 accumulation on the matrix cores).
 * SA     device, output rows (m, or m2 for COUNT_GAUSS) x d, row stride ldsa,
 *        double (PLAIN_FP64) or float (MIXED).
 * workspace  device scratch of at least mihs_sketch_workspace_size() bytes.
 * ------------------------------------------------------------------------ */
int mihs_sketch_workspace_size(mihs_handle_t handle, int64_t n, int64_t d, int64_t m,
                               int64_t m2, mihs_sketch_kind_t kind, mihs_dtype_t a_dtype,
                               mihs_precision_t precision, size_t* bytes);

int mihs_sketch(mihs_handle_t handle, const void* A, mihs_dtype_t a_dtype, int64_t n,
                int64_t d, int64_t lda, mihs_sketch_kind_t kind, int64_t m, int64_t m2,
                uint32_t seed, mihs_precision_t precision, void* SA, int64_t ldsa,
                void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Solve (Algorithm 1 with a conjugate-gradient inner solver):
 *   g^i     = A^T (b - A x^i) - lambda x^i                 (FP64, one pass over A)
 *   dx^i    : ((SA)^T SA + lambda I) dx = g^i by CG from 0,
 *             stopped when ||residual|| <= eps_sub ||g^i|| or after max_inner
 *   x^{i+1} = x^i + alpha dx^i + beta (x^i - x^{i-1})
 * The whole loop runs in one cooperative device launch (no host round trips).
 * It stops when ||x^{i+1} - x^i|| / ||x^{i+1}|| <= tol (1 - sqrt(beta)) / sqrt(beta)
 * (an estimate of ||x - x*|| / ||x*|| <= tol for contraction rate sqrt(beta),
 * Corollary 4), or after max_outer iterations.  tol <= 0 runs exactly
 * max_outer iterations.
 *
 * A       device, n x d (a_dtype), row stride lda.
 * b       device, n doubles.
 * lambda  > 0.
 * SA      device, m x d sketch from mihs_sketch with the same `precision`.
 * alpha, beta  momentum (Corollary 4: beta = sd/m, alpha = (1-beta)^2).
 * X       device, d doubles: in = x^1 (warm start), out = last iterate.
 * X_prev  device, d doubles or NULL: in = x^0 (the momentum term's previous
 *         iterate; NULL means x^0 = x^1), out = the iterate before X.
 * d_info  device, one mihs_info_t.
 * ------------------------------------------------------------------------ */
int mihs_solve_workspace_size(mihs_handle_t handle, int64_t n, int64_t d, int64_t m,
                              mihs_precision_t precision, size_t* bytes);

int mihs_solve(mihs_handle_t handle, const void* A, mihs_dtype_t a_dtype, int64_t n, int64_t d,
               int64_t lda, const double* b, double lambda, const void* SA, int64_t m,
               int64_t ldsa, mihs_precision_t precision, double alpha, double beta,
               double eps_sub, double tol, int64_t max_outer, int64_t max_inner, double* X,
               double* X_prev, mihs_info_t* d_info, void* workspace, size_t ws_bytes,
               void* stream);

/* ------------------------------------------------------------------------
 * mihs_solve without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, algorithm, kernels and results as
 * mihs_solve; the scratch is a static device array inside the library of
 * MIHS_NOALLOC_SCRATCH_BYTES bytes, one per GPU, held from the first
 * mihs_create on that GPU until the process ends (the library takes its
 * address in mihs_create).  The call allocates nothing (no hipMalloc, no
 * hipFree, no allocating library routine) and clears the parts of the array
 * that must start at zero itself, with a kernel.
 * Limit: returns MIHS_ERR_WORKSPACE, before any GPU work, when the solve at
 * these sizes could need more scratch than the array holds
 * (mihs_solve_workspace_size() > MIHS_NOALLOC_SCRATCH_BYTES; e.g. d <= 2048
 * with m >= d fits in both precisions).
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (two streams, two threads) race and
 * must be serialised by the caller.
 * ------------------------------------------------------------------------ */
#define MIHS_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)

int mihs_solve_noalloc(mihs_handle_t handle, const void* A, mihs_dtype_t a_dtype, int64_t n,
                       int64_t d, int64_t lda, const double* b, double lambda, const void* SA,
                       int64_t m, int64_t ldsa, mihs_precision_t precision, double alpha,
                       double beta, double eps_sub, double tol, int64_t max_outer,
                       int64_t max_inner, double* X, double* X_prev, mihs_info_t* d_info,
                       void* stream);

/* mihs_solve with a choice of inner solver (mihs_inner_t); MIHS_INNER_CG is
 * mihs_solve itself.  With MIHS_INNER_AAB, eps_sub bounds AAb_Solver's residual
 * estimate and d_info's inner counts are AAb steps.  Same workspace size. */
int mihs_solve_inner(mihs_handle_t handle, const void* A, mihs_dtype_t a_dtype, int64_t n,
                     int64_t d, int64_t lda, const double* b, double lambda, const void* SA,
                     int64_t m, int64_t ldsa, mihs_precision_t precision, mihs_inner_t inner,
                     double alpha, double beta, double eps_sub, double tol, int64_t max_outer,
                     int64_t max_inner, double* X, double* X_prev, mihs_info_t* d_info,
                     void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Dual M-IHS (Algorithm 2; Section 2, eqs. (intro_dual), (dual_mihs1)) for an
 * under-determined problem, n <= d.  The dual variable nu lives in R^n; the
 * caller passes At = A^T (d x n, row-major) -- the tall matrix each iteration
 * streams -- and SAt = S A^T (m x n) from mihs_sketch on At.  Per iteration:
 *   g^i      = b - A A^T nu^i - lambda nu^i                (FP64, one pass over At)
 *   dnu^i    : ((S A^T)^T S A^T + lambda I) dnu = g^i by CG (as in mihs_solve)
 *   nu^{i+1} = nu^i + alpha dnu^i + beta (nu^i - nu^{i-1})
 * and finally X = A^T nu (eq. (dual_relation)).  The stop rule is mihs_solve's,
 * applied to nu; momentum from Corollary 4 with sd(A) and m.
 *
 * At      device, d x n (a_dtype), row stride ldat (16-byte aligned rows); n <= d.
 * b       device, n doubles.
 * SAt     device, m x n sketch of At with the same `precision`.
 * NU      device, n doubles: in = nu^1 (zeros for Algorithm 2), out = last iterate.
 * X       device, d doubles: out = A^T nu.
 * d_info  device, one mihs_info_t (iteration counts refer to nu).
 * Errors as mihs_solve (n > d is MIHS_ERR_INVALID).  Workspace from
 * mihs_solve_dual_workspace_size().
 * ------------------------------------------------------------------------ */
int mihs_solve_dual_workspace_size(mihs_handle_t handle, int64_t n, int64_t d, int64_t m,
                                   mihs_precision_t precision, size_t* bytes);

int mihs_solve_dual(mihs_handle_t handle, const void* At, mihs_dtype_t a_dtype, int64_t n,
                    int64_t d, int64_t ldat, const double* b, double lambda, const void* SAt,
                    int64_t m, int64_t ldsa, mihs_precision_t precision, double alpha,
                    double beta, double eps_sub, double tol, int64_t max_outer,
                    int64_t max_inner, double* NU, double* X, mihs_info_t* d_info,
                    void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Primal-Dual M-IHS (Section 2, two-stage sketching, eq. (pd_mihs1);
 * Algorithm 4 for n >= d, Algorithm 3 for n <= d).  The outer iteration is
 * M-IHS; its sub-problem ((SA)^T SA + lambda I) dx = g is solved through its
 * dual by M M-IHS steps on
 *     min_z 1/2 ||Q z - g||^2 + lambda/2 ||z||^2,   Q = (S A)^T  (z in R^{m1}),
 * with the second sketch WQ = W Q, then dx = (g - Q z) / lambda.  The dual
 * steps use `inner` (AAb_Solver in the paper; CG goes through the Gram matrix
 * of WQ, formed once per call, when m2 >= m1) with forcing term eps_sub, and
 * z with its momentum state carries over between outer steps
 * (z^{i+1,1} = z^{i,M+1}, z^{i+1,0} = z^{i,M}).  Momentum (Corollary 4):
 * beta_l = sd / m_l, alpha_l = (1 - beta_l)^2 for l = 1 (outer), 2 (dual).
 * The stop rule is mihs_solve's on the outer iterate with beta1.
 *
 * mihs_solve_pd (Algorithm 4, n >= d):
 *   A    device n x d (a_dtype), row stride lda;  b  device, n doubles.
 *   Q    device d x m1, (S A)^T: mihs_transpose of an m1 x d sketch of A.
 *   X    device, d doubles: in = x^1, out = last iterate.
 * mihs_solve_pd_dual (Algorithm 3, n <= d):
 *   At   device d x n, A^T (a_dtype), row stride ldat;  b  device, n doubles.
 *   Q    device n x m1, (S A^T)^T: mihs_transpose of an m1 x n sketch of A^T.
 *   NU   device, n doubles: in = nu^1 (zeros in Algorithm 3), out = last iterate.
 *   X    device, d doubles: out = A^T nu.
 * Both:
 *   WQ   device m2 x m1: a sketch of Q (mihs_sketch on Q with m2 rows).
 *   Q and WQ are double for PLAIN_FP64 and float for MIXED.
 *   M >= 1 dual steps per outer step; the outer dimension (d, resp. n) and m1
 *   are at most 4096 (MIHS_ERR_UNSUPPORTED otherwise).
 *   d_info  one record: outer_iters, inner_iters_total (inner-solver steps over
 *           all dual steps), inner_iters_max (per outer step), rel_step,
 *           grad_norm (||g|| of the last outer step), status.
 * The host enqueues max_outer outer steps without waiting; once the stop rule
 * holds, the remaining enqueued kernels return at once.
 * ------------------------------------------------------------------------ */
int mihs_solve_pd_workspace_size(mihs_handle_t handle, int64_t n, int64_t d, int64_t m1,
                                 int64_t m2, mihs_precision_t precision, size_t* bytes);

int mihs_solve_pd(mihs_handle_t handle, const void* A, mihs_dtype_t a_dtype, int64_t n,
                  int64_t d, int64_t lda, const double* b, double lambda, const void* Q,
                  int64_t m1, int64_t ldq, const void* WQ, int64_t m2, int64_t ldwq,
                  mihs_precision_t precision, mihs_inner_t inner, double alpha1, double beta1,
                  double alpha2, double beta2, int64_t M, double eps_sub, double tol,
                  int64_t max_outer, int64_t max_inner, double* X, mihs_info_t* d_info,
                  void* workspace, size_t ws_bytes, void* stream);

int mihs_solve_pd_dual_workspace_size(mihs_handle_t handle, int64_t n, int64_t d, int64_t m1,
                                      int64_t m2, mihs_precision_t precision, size_t* bytes);

int mihs_solve_pd_dual(mihs_handle_t handle, const void* At, mihs_dtype_t a_dtype, int64_t n,
                       int64_t d, int64_t ldat, const double* b, double lambda, const void* Q,
                       int64_t m1, int64_t ldq, const void* WQ, int64_t m2, int64_t ldwq,
                       mihs_precision_t precision, mihs_inner_t inner, double alpha1,
                       double beta1, double alpha2, double beta2, int64_t M, double eps_sub,
                       double tol, int64_t max_outer, int64_t max_inner, double* NU, double* X,
                       mihs_info_t* d_info, void* workspace, size_t ws_bytes, void* stream);

/* Transpose: dst (cols x rows, row stride ldd) = src^T, src rows x cols with row
 * stride lds; dtype for both.  Forms Q = (S A)^T for the Primal-Dual solves. */
int mihs_transpose(mihs_handle_t handle, const void* src, mihs_dtype_t dtype, int64_t rows,
                   int64_t cols, int64_t lds, void* dst, int64_t ldd, void* stream);

/* ------------------------------------------------------------------------
 * Statistical dimension estimate from a sketch: the inexact Hutchinson trace
 * estimator of Section 3.4 (Algorithm 5),
 *   sd ~ d - (lambda / T) sum_{l<T} <v^l, z^l>,
 *   ((SA)^T SA + lambda I) z^l = v^l solved to ||r|| <= eps_tr ||v^l||,
 * which estimates d - lambda tr(((SA)^T SA + lambda I)^{-1}), the statistical
 * dimension sum sigma_i^2 / (sigma_i^2 + lambda) seen through the sketch; its
 * value sets beta = sd / m in Corollary 4.  The paper uses T = 2 or 3 and
 * eps_tr = 0.5.
 *
 * SA        m x d, row stride ldsa (device; double for PLAIN_FP64, float for
 *           MIXED, whose inner CG then runs in float).  Any m >= 1.
 * T, seed   the probes: entry j of probe l (0 <= j < d, 0 <= l < T) is -1 if
 *           bit 31 of MurmurHash3_x86_32(l * d + j mod 2^32, seed) is set,
 *           else +1.  T <= 2^20.
 * inner     the inner solver: MIHS_INNER_AAB is the paper's AAb_Solver (stops
 *           when its residual estimate falls below eps_tr), MIHS_INNER_CG is
 *           CG from z = 0 stopped at ||r|| <= eps_tr ||v^l||.
 * sd        one device double, the estimate.
 * Z         optional (NULL to skip): T x d row-major doubles, z^l in row l.
 * d_info    T device records: inner_iters_total = inner steps of probe l,
 *           status MIHS_CONVERGED or MIHS_BREAKDOWN.
 * Needs d <= 4096 (MIHS_ERR_UNSUPPORTED otherwise); the workspace size comes
 * from mihs_estimate_sd_workspace_size().
 * ------------------------------------------------------------------------ */
int mihs_estimate_sd_workspace_size(mihs_handle_t handle, int64_t m, int64_t d, int64_t T,
                                    mihs_precision_t precision, size_t* bytes);

int mihs_estimate_sd(mihs_handle_t handle, const void* SA, int64_t m, int64_t d, int64_t ldsa,
                     mihs_precision_t precision, mihs_inner_t inner, double lambda, int64_t T,
                     uint32_t seed, double eps_tr, int64_t max_inner, double* sd, double* Z,
                     mihs_info_t* d_info, void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Multi-RHS solve: k right-hand sides B (n x k, row stride ldb) with one
 * lambda, all sharing A and SA.  Algorithm 1 per column, the columns run in
 * blocks of 16 that share each pass over A and SA (FP64 matrix cores); needs
 * d <= 1024.  X is d x k row-major (in: warm start, out: solution); d_info
 * holds k records.  Workspace size from mihs_solve_multi_workspace_size().
 * ------------------------------------------------------------------------ */
int mihs_solve_multi_workspace_size(mihs_handle_t handle, int64_t n, int64_t d, int64_t m,
                                    int64_t k, mihs_precision_t precision, size_t* bytes);

int mihs_solve_multi(mihs_handle_t handle, const void* A, mihs_dtype_t a_dtype, int64_t n,
                     int64_t d, int64_t lda, const double* B, int64_t k, int64_t ldb,
                     double lambda, const void* SA, int64_t m, int64_t ldsa,
                     mihs_precision_t precision, double alpha, double beta, double eps_sub,
                     double tol, int64_t max_outer, int64_t max_inner, double* X,
                     mihs_info_t* d_info, void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Batched lambda-path solve: nprob independent problems, each solved for nlam
 * regularisation values that share the problem's one sketch SA_k.  One
 * persistent launch runs every (problem, lambda) pair; problems are split in
 * row blocks over the GPU and each pass over A_k serves all nlam iterates.
 *
 * problems  device array of nprob mihs_problem_t records (see below).
 * lambdas, alphas, betas  device, nprob x nlam doubles each (row k = problem k).
 * Each problem's X is d_k x nlam row-major doubles (column j = lambda j; in:
 * warm start, out: solution) and info points at nlam mihs_info_t records.
 * A_k is FP64 with d_k <= 1024; SA_k has the precision's type (double / float).
 * Every pass and the inner CG run in FP64 on the matrix cores (16 lambdas
 * per pass).  h_problems is the host copy of the table the call schedules
 * from (large problems get teams of workgroups, small ones share one);
 * d_problems may be NULL.  The call copies its schedule to the workspace and
 * waits for that copy before it returns (mihs_batched_plan_create and
 * mihs_batched_plan_run below split the two halves).
 * ------------------------------------------------------------------------ */
typedef struct {
  const void* A;    /* n x d, row stride lda (double) */
  const double* b;  /* n */
  const void* SA;   /* m x d, row stride ldsa */
  double* X;        /* d x nlam */
  mihs_info_t* info;/* nlam records */
  int64_t n, d, lda, m, ldsa;
} mihs_problem_t;

int mihs_solve_batched_workspace_size(mihs_handle_t handle, const mihs_problem_t* h_problems,
                                      int64_t nprob, int64_t nlam, mihs_precision_t precision,
                                      size_t* bytes);

int mihs_solve_batched(mihs_handle_t handle, const mihs_problem_t* d_problems,
                       const mihs_problem_t* h_problems, int64_t nprob, const double* lambdas,
                       const double* alphas, const double* betas, int64_t nlam,
                       mihs_precision_t precision, double eps_sub, double tol,
                       int64_t max_outer, int64_t max_inner, void* workspace, size_t ws_bytes,
                       void* stream);

/* ------------------------------------------------------------------------
 * Tunable shape of the batched launch (not in the paper; the schedule and the
 * tiling of the one persistent launch above).
 *   cg_cols       columns of the Gram matrix owned by one workgroup of a
 *                 problem's inner-CG sub-team (16, 32, 64, 128 or 512): the
 *                 sub-team has ceil(d / cg_cols) members, at most the problem's
 *                 team (512: for d <= 512 the inner CG runs inside one
 *                 workgroup);
 *   a_dma         1: each pass over A moves 64 KiB groups of rows straight
 *                 into LDS (rows of 1-4 KiB); 0: 16-row tiles staged through
 *                 registers;
 *   inner_weight  the expected inner-CG cost per outer iteration, in passes
 *                 over H per column group, used to size the teams (team size
 *                 proportional to n d + inner_weight d^2; 1 to 10000).
 * mihs_batched_default_tuning() fills the defaults (32, 1, 100, measured 0,
 * exact 0).
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t cg_cols;
  int32_t a_dma;
  double inner_weight;
  int32_t measured;  /* 1: size the teams from the per-problem costs that
                        mihs_tune_batched measured on an equal problem set
                        (inner_weight unused); without such a measurement the
                        model above is used */
  int32_t exact;     /* 1: solve the sub-problem of every outer step exactly
                        (Exact M-IHS, Table 2 and Section 4.2: the variant
                        that factorizes the sketched system): one
                        FP64 Cholesky factor of (SA)^T SA + lambda_j I per
                        column, formed in the launch before the solve, then a
                        forward and a backward substitution per outer step
                        (inner_iters counts 1 per outer step; cg_cols unused).
                        A column whose factorization meets a non-positive
                        pivot makes its problem use the inexact CG instead.
                        0: the inexact inner CG to eps_sub */
} mihs_batched_tuning_t;

void mihs_batched_default_tuning(mihs_batched_tuning_t* tuning);

/* ------------------------------------------------------------------------
 * The batched solve split into a plan and a launch, for callers that capture
 * the launch in a HIP graph or repeat it (same problems, new data in b, SA or
 * X at the same addresses).
 *
 * mihs_batched_plan_create  validates the problems as mihs_solve_batched does,
 *   schedules them, writes the schedule tables into `workspace` (which must
 *   stay allocated and untouched for the plan's lifetime; its size comes from
 *   mihs_solve_batched_workspace_size) and waits for that copy.  `tuning`
 *   NULL takes the handle's tuned choice for this problem set (see
 *   mihs_tune_batched) or the defaults.  The host pointers in h_problems,
 *   lambdas, alphas and betas are device addresses recorded in the plan.
 * mihs_batched_plan_run  enqueues the solve on `stream`: a fill kernel that
 *   clears the barrier words, the Gram matrices of the sketches, then the
 *   persistent kernel.  It does not synchronise, allocate, copy from the host
 *   or issue a memset, so it may be captured in a HIP graph; under capture the
 *   persistent kernel goes in as an ordinary launch of one workgroup per
 *   compute unit (the plan checked that one fits per unit; every wait is
 *   bounded and ends in MIHS_BARRIER_TIMEOUT).  X is read as the start x^1
 *   and overwritten; reset it between runs to restart from zero.  Runs of one
 *   plan, or of plans sharing a workspace, must not overlap.
 * mihs_batched_plan_destroy  frees the plan (not the workspace).
 * ------------------------------------------------------------------------ */
typedef struct mihs_batched_plan* mihs_batched_plan_t;

int mihs_batched_plan_create(mihs_handle_t handle, const mihs_problem_t* h_problems,
                             int64_t nprob, const double* lambdas, const double* alphas,
                             const double* betas, int64_t nlam, mihs_precision_t precision,
                             double eps_sub, double tol, int64_t max_outer, int64_t max_inner,
                             const mihs_batched_tuning_t* tuning, void* workspace,
                             size_t ws_bytes, void* stream, mihs_batched_plan_t* plan);
int mihs_batched_plan_run(mihs_batched_plan_t plan, void* stream);
int mihs_batched_plan_destroy(mihs_batched_plan_t plan);

/* ------------------------------------------------------------------------
 * Autotuner of the batched launch shape.  Times trial solves of the given
 * problems (each from X = 0, at most trial_outer outer iterations, HIP events
 * on `stream`) over candidate shapes by coordinate descent: inner_weight in
 * {6.25, 25, 100, 400}, then cg_cols in {16, 32, 64, 512}, then a_dma in {1, 0}.
 * These shapes all use the inexact inner CG (Algorithm 1's decomposition-free
 * sub-solver).  Only with allow_exact = 1 does it also try exact = 1 (Exact
 * M-IHS: one Cholesky factor per column) with inner_weight in {6.25, 25} (the
 * best exact shape is kept apart: short trials charge its factorizations to
 * few outer iterations); allow_exact = 0 never chooses exact sub-solves.
 * If measure_outer > 0 it then runs the best inexact shape (and, with
 * allow_exact, the best exact shape) for up to measure_outer outer iterations
 * each (normally the solve's own limit, so that every problem runs to its
 * stop), keeps the faster, reads the
 * wall time of every problem in that run (mihs_info_t.elapsed_us), takes time
 * x team size as the problem's cost on one workgroup, and runs a schedule
 * sized from those costs (teams of
 * ceil(cost / L) workgroups for problems above a makespan L, first-fit bins
 * of capacity L for the rest, a team member's remaining capacity after its
 * team problem included; the smallest L that fits) for as long, with the
 * shape's cg_cols and (inexact shapes) with cg_cols = 64, so that a team's
 * inner CG splits over all its members; if one of them beat the plain runs,
 * up to three times more with costs re-measured under the best of them (a
 * team does not run its problem team-size times faster), while a round gains
 * more than 2%; measured = 1 in *best if a measured schedule was the fastest.  The best
 * shape is returned in *best and kept in the handle, keyed by the problem set's
 * shapes (n, d, m of every problem and nlam); later mihs_solve_batched and
 * mihs_batched_plan_create calls on an equal set use it.  cand_ms (nullable,
 * room for MIHS_TUNE_MAX_CANDIDATES floats) receives each trial's time in
 * candidate order and *ncand their count (nullable).  The trials overwrite X
 * and info: initialise X after tuning.  Blocks until the trials end.
 * ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------
 * The batched launch's schedule without a device (host computation only; for
 * inspection and tests).  Problem k of nprob has n[k] x d[k] and nlam columns
 * (one entry per group of up to 16); num_cu workgroups.  With tuning->measured
 * = 1 and cost non-NULL (one value per entry: its time on one workgroup) the
 * teams come from the makespan rule of mihs_tune_batched, else from the model
 * n d + inner_weight d^2.  Per entry (problem-major, groups of 16 columns in
 * order): team0[e] first workgroup, tsize[e] team size (1: the entry shares a
 * single-workgroup bin), tcg[e] inner-solve sub-team size (exact
 * sub-solves: min(tsize, 16), one member per column at most).  Arrays hold
 * nprob * ceil(nlam / 16) values.  Returns MIHS_ERR_UNSUPPORTED if the entries
 * do not fit.
 * ------------------------------------------------------------------------ */
int mihs_batched_schedule(int32_t num_cu, const int64_t* n, const int64_t* d, int64_t nprob,
                          int64_t nlam, const mihs_batched_tuning_t* tuning, const double* cost,
                          int32_t* team0, int32_t* tsize, int32_t* tcg);

#define MIHS_TUNE_MAX_CANDIDATES 16

int mihs_tune_batched(mihs_handle_t handle, const mihs_problem_t* h_problems, int64_t nprob,
                      const double* lambdas, const double* alphas, const double* betas,
                      int64_t nlam, mihs_precision_t precision, double eps_sub, double tol,
                      int64_t trial_outer, int64_t measure_outer, int64_t max_inner,
                      int32_t allow_exact, void* workspace, size_t ws_bytes, void* stream,
                      mihs_batched_tuning_t* best, float* cand_ms, int32_t* ncand);

/* ------------------------------------------------------------------------
 * Tuning cache (host only).  The shapes mihs_tune_batched keeps in a handle,
 * with their measured per-entry costs, written to / read from one JSON file
 *   {"format": "libmihs-batched-tuning", "version": 1, "arch": ..., "num_cu": ...,
 *    "entries": [{"key": "<16 hex digits>", "cg_cols", "a_dma", "inner_weight",
 *                 "measured", "exact", "cost": [...]}, ...]}
 * so that a later process skips the tuning of a problem set it has seen.
 * mihs_tuning_cache_save writes every kept shape (replacing the file through a
 *   temporary and a rename).  MIHS_ERR_INVALID if the file cannot be written.
 * mihs_tuning_cache_load adds the file's shapes to the handle (replacing equal
 *   keys) when its arch and num_cu equal the handle's device; a file for
 *   another device is read and ignored (*loaded = 0).  *loaded (nullable) is
 *   the number of shapes taken.  MIHS_ERR_INVALID if the file is missing or
 *   not in this format (the handle is then unchanged).
 * mihs_batched_cached_tuning returns MIHS_OK and the kept shape in *tuning if
 *   the handle holds one for this problem set (shapes n, d, m of every problem
 *   and nlam), else MIHS_ERR_UNSUPPORTED.
 * ------------------------------------------------------------------------ */
int mihs_tuning_cache_save(mihs_handle_t handle, const char* path);
int mihs_tuning_cache_load(mihs_handle_t handle, const char* path, int32_t* loaded);
int mihs_batched_cached_tuning(mihs_handle_t handle, const mihs_problem_t* h_problems,
                               int64_t nprob, int64_t nlam, mihs_batched_tuning_t* tuning);

/* ------------------------------------------------------------------------
 * Backward of x*_j = (A^T A + lambda I)^{-1} A^T b_j for k right-hand sides.
 * Given Gbar = dL/dX* (d x k), solves the adjoint systems
 *   (A^T A + lambda I) w_j = gbar_j
 * by M-IHS on the same sketch (gradient gbar_j - A^T A w_j - lambda w_j), then
 *   dL/dB = A W  (n x k)    and    dL/dlambda = - sum_j x*_j^T w_j.
 * Xstar, Gbar, W are d x k row-major doubles (device); dB is n x k (device,
 * NULL to skip); dlambda is one device double; dloglambda (device, NULL to
 * skip) receives dL/dlog(lambda) = lambda dL/dlambda, the derivative for the
 * log(lambda) parametrisation of mihs_lambda_from_log.  d_info holds k records.
 * For d <= 1024 the k systems run as blocks of 16 right-hand sides that share
 * each pass over A and SA (FP64 matrix cores); wider problems solve the
 * columns one after another.  The workspace size comes from
 * mihs_solve_backward_workspace_size().
 * ------------------------------------------------------------------------ */
int mihs_solve_backward_workspace_size(mihs_handle_t handle, int64_t n, int64_t d, int64_t m,
                                       int64_t k, mihs_precision_t precision, size_t* bytes);

int mihs_solve_backward(mihs_handle_t handle, const void* A, mihs_dtype_t a_dtype, int64_t n,
                        int64_t d, int64_t lda, const void* SA, int64_t m, int64_t ldsa,
                        double lambda, mihs_precision_t precision, const double* Xstar,
                        const double* Gbar, int64_t k, double alpha, double beta,
                        double eps_sub, double tol, int64_t max_outer, int64_t max_inner,
                        double* W, double* dB, double* dlambda, double* dloglambda,
                        mihs_info_t* d_info, void* workspace, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MIHS_H_ */
