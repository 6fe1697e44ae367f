// Internal host-side interfaces between the C ABI layer and the kernel files.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/mihs.h"

#include <mutex>
#include <utility>
#include <vector>

// A batched launch shape chosen by mihs_tune_batched for one problem set, with
// the per-entry costs (one workgroup, microseconds) it measured.
struct mihs_tuned_set {
  uint64_t key;
  mihs_batched_tuning_t tuning;
  std::vector<double> cost;
};

struct mihs_handle {
  int device;
  int num_cu;
  int wall_khz;  // rate of the device's constant wall clock
  char arch[64];
  int32_t row_weight[8];  // gradient-pass row shares per XCD (mihs_set_row_weights)
  void* noalloc_scratch;  // this device's address of the library's static scratch
  std::mutex tune_mu;
  std::vector<mihs_tuned_set> tuned;
};

namespace mihs {

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Static device scratch of mihs_solve_noalloc (bytes; MIHS_NOALLOC_SCRATCH_BYTES).
constexpr size_t kNoAllocScratchBytes = (size_t)MIHS_NOALLOC_SCRATCH_BYTES;
// This device's address of that scratch (hipGetSymbolAddress; the handle's
// device must be current).
int noalloc_scratch_address(void** ptr);

#if defined(__HIPCC__)
#define MIHS_HOST_DEVICE __host__ __device__
#else
#define MIHS_HOST_DEVICE
#endif

// Rows of the solve kernel's gradient pass: workgroups are dispatched to the
// XCDs in turn (workgroup v on XCD v mod 8), and workgroup v takes rows in
// proportion to its XCD's weight w[v mod 8] (1..kRowWeightMax).  Returns the
// first row of workgroup v of G (v = G gives n).  Equal weights give
// floor(n v / G), the even split.
constexpr int kXcds = 8;
constexpr int32_t kRowWeightMax = 64;
MIHS_HOST_DEVICE inline int64_t row_split_bound(int64_t n, int G, const int32_t* w, int v) {
  if (v >= G) return n;
  int64_t sum = 0;
  for (int k = 0; k < kXcds; ++k) sum += w[k];
  int64_t pre = (int64_t)(v / kXcds) * sum, tot = (int64_t)(G / kXcds) * sum;
  for (int k = 0; k < v % kXcds; ++k) pre += w[k];
  for (int k = 0; k < G % kXcds; ++k) tot += w[k];
  return n * pre / tot;
}

// Measures each XCD's streaming time and sets h->row_weight from it
// (mihs_calibrate_rows).
int calibrate_rows(mihs_handle* h);

// Padded vector length used by the row kernels: 64 lanes x elements-per-lane.
int ept_for(int64_t d);
inline int64_t dpad_for(int64_t d) { return 64 * (int64_t)ept_for(d); }

// ---- solve ----------------------------------------------------------------
struct SolveDesc {
  const void* A;
  int a_f32;
  int64_t n, d, lda;
  const double* b;    // ridge mode (n)   -- exactly one of b / rhs is set
  const double* rhs;  // adjoint mode (d)
  const void* SA;
  int mixed;
  int64_t m, ldsa;
  double lam, alpha, beta, eps_sub, tol;
  int64_t max_outer, max_inner;
  double* x;
  double* x_prev;  // may be null
  mihs_info_t* info;
  // 1: the inner CG streams SA on every step even where m >= d (no Gram
  // matrix); pays off when the inner solve takes only a few steps.
  int no_gram = 0;
  // 1: AAb_Solver (Algorithm 6) as the inner solver (streams SA; no Gram matrix)
  int aab = 0;
  // device flag: when nonzero at launch time the solve returns at once
  const int* skip = nullptr;
  // 1: the Gram matrix of SA is already in this workspace (an earlier call with
  // the same SA and workspace formed it)
  int gram_ready = 0;
  // launch shape; 0 = chosen from the sizes: workgroups of the inner-solve
  // group, and the fewest rows of A per workgroup
  int cg_groups = 0;
  int64_t rows_per_wg = 0;
};

// g = A^T (c - A x) + rhs - lambda x (c and rhs may be null) for A n x d, d <= 4096;
// returns at once when *skip is nonzero.  Workspace: grad_workspace_bytes().
size_t grad_workspace_bytes(const mihs_handle* h, int64_t n, int64_t d);
int launch_grad(const mihs_handle* h, const void* A, int a_f32, int64_t n, int64_t d,
                int64_t lda, const double* c, const double* rhs, const double* x, double lam,
                double* g, void* ws, size_t ws_bytes, const int* skip, hipStream_t stream);

size_t solve_workspace_bytes(const mihs_handle* h, int64_t n, int64_t d, int64_t m, int mixed,
                             int no_gram = 0);
int launch_solve(const mihs_handle* h, const SolveDesc& s, void* ws, size_t ws_bytes,
                 hipStream_t stream);

// ---- statistical dimension estimate ------------------------------------------
size_t estimate_workspace_bytes(const mihs_handle* h, int64_t m, int64_t d, int64_t T, int mixed);
int launch_estimate_sd(const mihs_handle* h, const void* SA, int64_t m, int64_t d, int64_t ldsa,
                       int mixed, int aab, double lam, int64_t T, uint32_t seed, double eps_tr,
                       int64_t max_inner, double* sd, double* Zout, mihs_info_t* info,
                       void* ws, size_t ws_bytes, hipStream_t stream);

// ---- Primal-Dual M-IHS (Algorithms 3, 4) ------------------------------------
struct PdDesc {
  const void* A;      // outer matrix streamed by the gradient: A (n x d) or A^T (d x n)
  int a_f32;
  int64_t rows, cols, lda;  // its shape; the outer variable has `cols` entries
  const double* c;    // Algorithm 4: b (rows); Algorithm 3: null
  const double* rhs;  // Algorithm 3: b (cols); Algorithm 4: null
  const void* Q;      // transposed first-stage sketch, cols x m1
  int64_t m1, ldq;
  const void* WQ;     // second-stage sketch W Q, m2 x m1
  int64_t m2, ldwq;
  int mixed, aab;
  double lam, alpha1, beta1, alpha2, beta2, eps_sub, tol;
  int64_t M, max_outer, max_inner;
  double* x;          // outer iterate (cols): in x^1, out the last iterate
  mihs_info_t* info;
};
size_t pd_workspace_bytes(const mihs_handle* h, int64_t rows, int64_t cols, int64_t m1,
                          int64_t m2, int mixed);
int launch_pd(const mihs_handle* h, const PdDesc& p, void* ws, size_t ws_bytes,
              hipStream_t stream);
// dst (cols x rows, row stride ldd) = src^T for src rows x cols (row stride lds)
int launch_transpose(const void* src, int f32, int64_t rows, int64_t cols, int64_t lds,
                     void* dst, int64_t ldd, hipStream_t stream);

// ---- sketches -------------------------------------------------------------
size_t sketch_workspace_bytes(const mihs_handle* h, int64_t n, int64_t d, int64_t m, int64_t m2,
                              int kind, int a_f32, int mixed);
int launch_sketch(const mihs_handle* h, const void* A, int a_f32, int64_t n, int64_t d,
                  int64_t lda, int kind, int64_t m, int64_t m2, uint32_t seed, int mixed,
                  void* SA, int64_t ldsa, void* ws, size_t ws_bytes, hipStream_t stream);

// ---- block M-IHS (many problems x up to 16 right-hand sides each) ------------
struct BlockEntryDesc {
  const void* A;
  int64_t n, d, lda;
  const double* B;    // ridge mode: C[i][j] = B[i * ldb + j * ldbc], or null
  int64_t ldb, ldbc;
  const double* RHS;  // adjoint mode: RHS[c * ldr + j], or null
  int64_t ldr;
  const void* SA;
  int64_t m, ldsa;
  double* X;          // d x ncols, X[c * ldx + j]
  int64_t ldx;
  const double* lam;  // device, ncols values each
  const double* alpha;
  const double* beta;
  mihs_info_t* info;  // device, ncols records
  int ncols;          // 1..16
  int64_t sa_group;   // entries with equal sa_group share SA (and its Gram matrix)
};
int block_max_d();
// Largest workspace over every tuning candidate (any shape fits).
size_t block_workspace_bytes(const mihs_handle* h, const BlockEntryDesc* ents, int64_t count);
// Key of a problem set for the tuning cache: (n, d, m, ncols, sketch group) of each entry.
uint64_t block_signature(const BlockEntryDesc* ents, int64_t count);
bool block_tuning_valid(const mihs_batched_tuning_t& t);
// Right-hand sides per block entry (one matrix-core column block).
constexpr int kBlockRhs = 16;
// Deterministic schedule of the entries over G workgroups (also used to size
// the workspace): dedicated teams for heavy entries, single-workgroup bins for
// the rest; items[g] lists workgroup g's entries in order.
struct Schedule {
  std::vector<int> team0, tsize, tcg;
  std::vector<std::vector<int>> items;
  size_t stride = 1;
};
int make_schedule(const BlockEntryDesc* ents, int64_t count, int G,
                  const mihs_batched_tuning_t& tn, const std::vector<double>* cost,
                  Schedule* S);
// The tuned shape for this set if the handle has one, else the defaults; the
// measured per-entry costs go to *cost (empty if none).
mihs_batched_tuning_t block_tuning_for(mihs_handle* h, const BlockEntryDesc* ents, int64_t count,
                                       std::vector<double>* cost);
// The tuned shape kept for this set, if any.
bool block_tuning_lookup(mihs_handle* h, const BlockEntryDesc* ents, int64_t count,
                         mihs_batched_tuning_t* tuning);
// Keep a tuned shape (and its measured costs) for this set.
void block_tuning_store(mihs_handle* h, const BlockEntryDesc* ents, int64_t count,
                        const mihs_batched_tuning_t& tuning, const std::vector<double>& cost);
// Team size of every entry under a shape (cost: measured costs or null).
int block_team_sizes(const mihs_handle* h, const BlockEntryDesc* ents, int64_t count,
                     const mihs_batched_tuning_t& tuning, const std::vector<double>* cost,
                     std::vector<int>* tsize);
struct BlockPlan;  // opaque: kernel, launch shape, argument block, device tables
// cost: per-entry costs for tuning.measured (null or empty: the n d + w d^2 model)
int plan_block(const mihs_handle* h, const BlockEntryDesc* ents, int64_t count, int a_f32,
               int sa_f32, double eps_sub, double tol, int64_t max_outer, int64_t max_inner,
               const mihs_batched_tuning_t& tuning, const std::vector<double>* cost, void* ws,
               size_t ws_bytes, hipStream_t stream, BlockPlan** plan);
int run_block(const BlockPlan* plan, hipStream_t stream);
void free_block_plan(BlockPlan* plan);
// plan + run + free with the handle's tuning (one call, as before).
int launch_block(mihs_handle* h, const BlockEntryDesc* ents, int64_t count, int a_f32,
                 int sa_f32, double eps_sub, double tol, int64_t max_outer, int64_t max_inner,
                 void* ws, size_t ws_bytes, hipStream_t stream);

// ---- Gram matrices H = M^T M (FP64 accumulation on the matrix cores) --------
// One 64 x 64 block (bi <= bj) of one matrix per job; H is dp x dp with the
// entries of index >= d set to zero; accumulation is FP64 either way.
struct GramJob {
  const void* M;
  int64_t m, ld;
  void* H;     // FP64, or FP32 when h_f32
  int64_t ldh;
  int d, bi, bj, h_f32;
};
int launch_gram_jobs(const GramJob* d_jobs, int64_t njobs, int m_f32, hipStream_t stream);
// H (ldh >= 64 * ceil(d / 64), FP64 or FP32) = M^T M for M m x d (FP64 or FP32).
int launch_gram(const void* M, int m_f32, int64_t m, int64_t d, int64_t ld, void* H, int h_f32,
                int64_t ldh, hipStream_t stream);

// ---- dense helper kernels --------------------------------------------------
// Y (n x k, row stride ldy) = A (n x d) W (d x k row-major); FP64 accumulation.
int launch_apply_rows(const mihs_handle* h, const void* A, int a_f32, int64_t n, int64_t d,
                      int64_t lda, const double* W, int64_t k, double* Y, int64_t ldy,
                      hipStream_t stream);
// p[0..count) = value
int launch_fill(double* p, double value, int64_t count, hipStream_t stream);
// out = -sum over all entries of X .* W (d x k), one device double; out_log
// (nullable) = lam * out.
int launch_neg_dot(const double* X, const double* W, int64_t count, double lam, double* out,
                   double* out_log, hipStream_t stream);

}  // namespace mihs
