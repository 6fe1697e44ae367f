// Block M-IHS: many problems, each with up to 16 right-hand sides that share
// one pass over A per outer iteration (a lambda-path shares A, b and SA; the
// backward's adjoint systems share A, SA and lambda).
//
// One persistent cooperative launch.  The host scheduler gives each large
// problem a dedicated team of workgroups (synchronised by a team barrier) and
// packs small problems into single-workgroup bins that run them one after the
// other.  Per entry (problem x group of 16 columns) and outer iteration:
//
//   pass  for each 16-row tile of M (A, then SA in every CG iteration):
//         stage the tile in LDS (FP64), U = C - M_tile X on the matrix cores
//         (v_mfma_f64_16x16x4, the four waves split the d-range and add their
//         partial U in LDS), then G += M_tile^T U for each wave's d-slice.
//   A     G = A^T (B - A X) (+ RHS) - X diag(lambda), reduced over the team.
//   CG    16 CGs in lockstep on ((SA)^T SA + lambda_j I), per-column step
//         lengths, per-column convergence masks; two team barriers each.
//   U     per-column heavy-ball step and relative-step stop test.
//
// Everything is FP64; all reductions run in a fixed order.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "device_util.hpp"
#include "internal.hpp"

namespace mihs {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int KR = 16;       // right-hand sides per entry (one MFMA column block)
constexpr int TROWS = 16;    // rows per tile
constexpr int kNScal = 4 * KR;

struct BatchEntry {
  const void* A;
  int64_t n, lda;
  const double* B;    // ridge: C[i][j] = B[i * ldb + j * ldbc] (ldbc = 0: one shared b)
  int64_t ldb, ldbc;
  const double* RHS;  // adjoint: extra d-space term RHS[c * ldr + j] (or null)
  int64_t ldr;
  const void* SA;
  int64_t m, ldsa;
  double* X;          // X[c * ldx + j], in: start, out: result
  int64_t ldx;
  const double* lam;
  const double* alpha;
  const double* beta;
  mihs_info_t* info;  // ncols records
  double* work;       // per-entry scratch (see entry_layout)
  unsigned* bar;      // team barrier counter (own 128-byte line)
  int d, dp, ncols;
  int team0, tsize;
};

struct BatchArgs {
  const BatchEntry* entries;
  const int* wg_items;  // per workgroup: entry indices, -1 terminated
  int items_stride;
  int* err;
  int a_f32, sa_f32;
  double eps_sub, tol;
  int64_t max_outer, max_inner;
  BarrierSpin spin;
};

// Scratch of one entry, in doubles: partial block vectors of every team member,
// then R, Z, P0, P1, XP (dp x KR each), then scalar partial slots.
struct EntryLayout {
  size_t part, R, Z, P0, P1, XP, scal, total;
};
__host__ __device__ inline EntryLayout entry_layout(int dp, int tsize) {
  EntryLayout L;
  const size_t blk = (size_t)dp * KR;
  size_t o = 0;
  L.part = o; o += (size_t)tsize * blk;
  L.R = o; o += blk;
  L.Z = o; o += blk;
  L.P0 = o; o += blk;
  L.P1 = o; o += blk;
  L.XP = o; o += blk;
  L.scal = o; o += (size_t)tsize * kNScal;
  L.total = (o + 31) / 32 * 32;
  return L;
}

struct Shared {
  double ured[kWavesPerBlock][TROWS * KR];
  double ufin[TROWS * KR];
  double red[kBlock];
  double lam[KR], alpha[KR], beta[KR], thr[KR];
  double rr[KR], rr0[KR], bcg[KR], acg[KR];
  int active[KR], done[KR];
  int64_t outer[KR], inner[KR], inner_max[KR], kin[KR];
  double step[KR], gnorm[KR];
  int flag;
};

__device__ __forceinline__ bool team_sync(const BatchEntry& e, unsigned& epoch, int* err,
                                          int* s_flag, BarrierSpin spin) {
  if (e.tsize <= 1) {
    __threadfence_block();
    __syncthreads();
    return true;
  }
  return barrier_flat(e.bar, epoch, (unsigned)e.tsize, err, s_flag, spin);
}

// Sum over the team's slots: out[j] = sum_t scal[t * kNScal + s0 + j], j < KR.
__device__ __forceinline__ void team_slot_sums(const double* scal, int T, int s0, double* out,
                                               double* red) {
  // thread (j, q) with j = tid % 16 sums t = q, q + 16, ... ; fixed tree over q
  const int j = threadIdx.x % KR, q = threadIdx.x / KR;
  double v = 0.0;
  for (int t = q; t < T; t += kBlock / KR) v += scal[(int64_t)t * kNScal + s0 + j];
  __syncthreads();
  red[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x < KR) {
    double a = red[threadIdx.x];
    for (int i = 1; i < kBlock / KR; ++i) a += red[i * KR + threadIdx.x];
    out[threadIdx.x] = a;
  }
  __syncthreads();
}

// Per-column sums of values held by all threads (thread tid owns column tid % 16).
__device__ __forceinline__ void column_partials(double v, double* out, double* red) {
  __syncthreads();
  red[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x < KR) {
    double a = red[threadIdx.x];
    for (int i = 1; i < kBlock / KR; ++i) a += red[i * KR + threadIdx.x];
    out[threadIdx.x] = a;
  }
  __syncthreads();
}

// One pass over rows [0, rows) of M (tiles t = rank, rank + T, ...):
//   U = C - M_tile V (C from B in ridge mode, 0 otherwise), uu[j] += sum U^2,
//   Gacc (this wave's d-slice) += M_tile^T U.
// V is the B operand in registers: Vreg[s] = V[kbase + 4 s + lane/16][lane % 16].
template <typename TM, int DP>
__device__ __forceinline__ void block_pass(const TM* __restrict__ M, int64_t ld, int64_t rows,
                                           int d, int rank, int T, const double* __restrict__ B,
                                           int64_t ldb, int64_t ldbc, int ncols,
                                           const double (&Vreg)[DP / 16],
                                           f64x4 (&Gacc)[DP / 64], double* tile, Shared& sh,
                                           double& uu_lane) {
  constexpr int DQ = DP / 4;   // columns per wave
  constexpr int KS = DQ / 4;   // k-steps per wave
  constexpr int NB = DQ / 16;  // 16-column output blocks per wave
  constexpr int LDT = DP + 1;  // LDS tile row stride (odd: spreads the 16 rows over banks)
  const int lane = lane_id(), wave = wave_id();
  const int kbase = wave * DQ;
  const int64_t ntiles = (rows + TROWS - 1) / TROWS;
  for (int64_t t = rank; t < ntiles; t += T) {
    const int64_t row0 = t * TROWS;
    __syncthreads();  // previous tile fully consumed
    for (int e = threadIdx.x; e < TROWS * DP; e += kBlock) {
      const int r = e / DP, c = e % DP;
      const int64_t gr = row0 + r;
      tile[r * LDT + c] = (gr < rows && c < d) ? (double)M[gr * ld + c] : 0.0;
    }
    __syncthreads();
    // partial U over this wave's k-range
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const double a = tile[(lane & 15) * LDT + kbase + 4 * s + (lane >> 4)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Vreg[s], acc, 0, 0, 0);
    }
    // result register r of lane l: row l/16 + 4 r, column l % 16
#pragma unroll
    for (int r = 0; r < 4; ++r) sh.ured[wave][((lane >> 4) + 4 * r) * KR + (lane & 15)] = acc[r];
    __syncthreads();
    {
      const int rr = threadIdx.x / KR, j = threadIdx.x % KR;  // one (row, column) per thread
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < kWavesPerBlock; ++w) s += sh.ured[w][rr * KR + j];
      const int64_t gr = row0 + rr;
      double u = 0.0;
      if (gr < rows && j < ncols) u = (B ? B[gr * ldb + j * ldbc] : 0.0) - s;
      sh.ufin[rr * KR + j] = u;
      uu_lane += u * u;
    }
    __syncthreads();
    // Gacc[b] += M_tile[:, slice block b]^T U
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int rr = 4 * s + (lane >> 4);
        const double a = tile[rr * LDT + kbase + 16 * b + (lane & 15)];
        const double bv = sh.ufin[rr * KR + (lane & 15)];
        Gacc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, Gacc[b], 0, 0, 0);
      }
    }
  }
}

// Store this wave's Gacc (d-slice x 16) to out[c * KR + j].
template <int DP>
__device__ __forceinline__ void store_block(const f64x4 (&Gacc)[DP / 64], double* out) {
  constexpr int DQ = DP / 4;
  const int lane = lane_id(), kbase = wave_id() * DQ;
#pragma unroll
  for (int b = 0; b < DQ / 16; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = kbase + 16 * b + (lane >> 4) + 4 * r;
      out[(int64_t)c * KR + (lane & 15)] = Gacc[b][r];
    }
}

template <int DP>
__device__ void run_entry(const BatchArgs& a, const BatchEntry& e, int rank, double* tile,
                          Shared& sh) {
  constexpr int DQ = DP / 4;
  constexpr int KS = DQ / 4;
  constexpr int NB = DQ / 16;
  const int T = e.tsize;
  const int d = e.d;
  const int lane = lane_id(), wave = wave_id();
  const int kbase = wave * DQ;
  const EntryLayout L = entry_layout(DP, T);
  double* W = e.work;
  double* part = W + L.part;
  double* R = W + L.R;
  double* Z = W + L.Z;
  double* P[2] = {W + L.P0, W + L.P1};
  double* XP = W + L.XP;
  double* scal = W + L.scal;
  double* myscal = scal + (int64_t)rank * kNScal;
  const int cpw = (d + T - 1) / T;
  const int c_lo = min(d, rank * cpw), c_hi = min(d, c_lo + cpw);
  const int nown = c_hi - c_lo;
  unsigned epoch = 0;
  int* s_flag = &sh.flag;
  bool alive = true;

  if (threadIdx.x < KR) {
    const int j = threadIdx.x;
    const bool on = j < e.ncols;
    sh.lam[j] = on ? e.lam[j] : 1.0;
    sh.alpha[j] = on ? e.alpha[j] : 0.0;
    sh.beta[j] = on ? e.beta[j] : 0.0;
    const double b = sh.beta[j];
    sh.thr[j] = (a.tol > 0.0 && b > 0.0 && b < 1.0) ? a.tol * (1.0 - sqrt(b)) / sqrt(b)
                                                    : (a.tol > 0.0 ? a.tol : 0.0);
    sh.done[j] = on ? 0 : 1;
    sh.outer[j] = 0;
    sh.inner[j] = 0;
    sh.inner_max[j] = 0;
    sh.step[j] = 0.0;
    sh.gnorm[j] = 0.0;
  }
  // x_prev = x on the owned columns
  for (int idx = threadIdx.x; idx < nown * KR; idx += kBlock) {
    const int c = c_lo + idx / KR, j = idx % KR;
    XP[(int64_t)c * KR + j] = (j < e.ncols) ? e.X[(int64_t)c * e.ldx + j] : 0.0;
  }
  __syncthreads();

  int status_all = MIHS_MAX_ITER;
  int64_t outer = 0;
  for (; outer < a.max_outer; ++outer) {
    // ---- A pass: G partial = A^T (C - A X) over this member's tiles
    double Vreg[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int c = kbase + 4 * s + (lane >> 4), j = lane & 15;
      Vreg[s] = (c < d && j < e.ncols) ? e.X[(int64_t)c * e.ldx + j] : 0.0;
    }
    f64x4 Gacc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) Gacc[b] = (f64x4){0.0, 0.0, 0.0, 0.0};
    double uu_lane = 0.0;
    if (a.a_f32)
      block_pass<float, DP>((const float*)e.A, e.lda, e.n, d, rank, T, e.B, e.ldb, e.ldbc,
                            e.ncols, Vreg, Gacc, tile, sh, uu_lane);
    else
      block_pass<double, DP>((const double*)e.A, e.lda, e.n, d, rank, T, e.B, e.ldb, e.ldbc,
                             e.ncols, Vreg, Gacc, tile, sh, uu_lane);
    store_block<DP>(Gacc, part + (int64_t)rank * DP * KR);
    if (!(alive = team_sync(e, epoch, a.err, s_flag, a.spin))) break;

    // ---- owners: g = sum of partials + rhs - lambda x; CG start (r = p = g, z = 0)
    double rr_lane = 0.0;
    for (int idx = threadIdx.x; idx < nown * KR; idx += kBlock) {
      const int c = c_lo + idx / KR, j = idx % KR;
      double g = 0.0;
      for (int t = 0; t < T; ++t) g += part[((int64_t)t * DP + c) * KR + j];
      if (j < e.ncols) {
        if (e.RHS) g += e.RHS[(int64_t)c * e.ldr + j];
        g -= sh.lam[j] * e.X[(int64_t)c * e.ldx + j];
      }
      if (sh.done[j]) g = 0.0;
      const int64_t o = (int64_t)c * KR + j;
      R[o] = g;
      Z[o] = 0.0;
      P[0][o] = g;
      rr_lane += g * g;
    }
    column_partials(rr_lane, myscal + 0, sh.red);
    if (!(alive = team_sync(e, epoch, a.err, s_flag, a.spin))) break;
    team_slot_sums(scal, T, 0, sh.rr0, sh.red);
    if (threadIdx.x < KR) {
      const int j = threadIdx.x;
      sh.rr[j] = sh.rr0[j];
      sh.gnorm[j] = sh.done[j] ? sh.gnorm[j] : sqrt(sh.rr0[j]);
      sh.active[j] = (!sh.done[j] && sh.rr0[j] > 0.0) ? 1 : 0;
      sh.bcg[j] = 0.0;
      sh.kin[j] = 0;
      // a column whose gradient is exactly zero sits at its solution
      if (!sh.done[j] && !(sh.rr0[j] > 0.0)) sh.done[j] = 1;
    }
    __syncthreads();

    // ---- lockstep CG
    int64_t k = 0;
    while (true) {
      int any = 0;
      for (int j = 0; j < KR; ++j) any |= sh.active[j];
      if (!any || k >= a.max_inner) break;
      double* pcur = P[k & 1];
      const double* pprev = P[(k + 1) & 1];
      // p = r + beta_cg p_prev for this wave's slice (B operand layout); owners store theirs
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int c = kbase + 4 * s + (lane >> 4), j = lane & 15;
        double v = 0.0;
        if (c < d) {
          const int64_t o = (int64_t)c * KR + j;
          v = (k == 0) ? pcur[o] : (sh.active[j] ? R[o] + sh.bcg[j] * pprev[o] : 0.0);
          if (k > 0 && c >= c_lo && c < c_hi) pcur[o] = v;
        }
        Vreg[s] = v;
      }
      // ||p_j||^2 over all d (all four waves' slices)
      double pp_lane = 0.0;
#pragma unroll
      for (int s = 0; s < KS; ++s) pp_lane += Vreg[s] * Vreg[s];
      // lanes with equal lane % 16 hold column j; combine within the wave, then waves
      pp_lane += __shfl_xor(pp_lane, 16, kWave);
      pp_lane += __shfl_xor(pp_lane, 32, kWave);
      __syncthreads();
      if (lane < KR) sh.ured[wave][lane] = pp_lane;
      __syncthreads();
      if (threadIdx.x < KR) {
        double t = 0.0;
        for (int w = 0; w < kWavesPerBlock; ++w) t += sh.ured[w][threadIdx.x];
        sh.acg[threadIdx.x] = t;  // holds ||p_j||^2 until the step length is formed
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < NB; ++b) Gacc[b] = (f64x4){0.0, 0.0, 0.0, 0.0};
      double uu = 0.0;
      if (a.sa_f32)
        block_pass<float, DP>((const float*)e.SA, e.ldsa, e.m, d, rank, T, nullptr, 0, 0,
                              e.ncols, Vreg, Gacc, tile, sh, uu);
      else
        block_pass<double, DP>((const double*)e.SA, e.ldsa, e.m, d, rank, T, nullptr, 0, 0,
                               e.ncols, Vreg, Gacc, tile, sh, uu);
      store_block<DP>(Gacc, part + (int64_t)rank * DP * KR);
      column_partials(uu, myscal + KR, sh.red);
      if (!(alive = team_sync(e, epoch, a.err, s_flag, a.spin))) break;

      // step lengths: p^T q = ||SA p||^2 + lambda ||p||^2
      team_slot_sums(scal, T, KR, sh.ufin, sh.red);  // ufin[0..15] <- sum ||u_j||^2
      if (threadIdx.x < KR) {
        const int j = threadIdx.x;
        const double pq = sh.ufin[j] + sh.lam[j] * sh.acg[j];
        double al = 0.0;
        if (sh.active[j]) {
          al = sh.rr[j] / pq;
          if (!(pq > 0.0) || !isfinite(al)) {
            al = 0.0;
            sh.active[j] = 0;  // breakdown in this column: keep the current step
          }
        }
        sh.acg[j] = al;
      }
      __syncthreads();
      double rr_lane2 = 0.0;
      for (int idx = threadIdx.x; idx < nown * KR; idx += kBlock) {
        const int c = c_lo + idx / KR, j = idx % KR;
        const int64_t o = (int64_t)c * KR + j;
        double q = 0.0;
        for (int t = 0; t < T; ++t) q += part[((int64_t)t * DP + c) * KR + j];
        q = -q + sh.lam[j] * pcur[o];
        const double al = sh.acg[j];
        if (sh.active[j]) {
          Z[o] += al * pcur[o];
          R[o] -= al * q;
        }
        rr_lane2 += R[o] * R[o];
      }
      column_partials(rr_lane2, myscal + 0, sh.red);
      if (!(alive = team_sync(e, epoch, a.err, s_flag, a.spin))) break;
      team_slot_sums(scal, T, 0, sh.ufin, sh.red);  // ufin[0..15] <- new ||r_j||^2
      ++k;
      if (threadIdx.x < KR) {
        const int j = threadIdx.x;
        if (sh.active[j]) {
          const double rn = sh.ufin[j];
          sh.bcg[j] = rn / sh.rr[j];
          sh.rr[j] = rn;
          sh.kin[j] = k;
          if (rn <= a.eps_sub * a.eps_sub * sh.rr0[j]) sh.active[j] = 0;
        }
      }
      __syncthreads();
    }
    if (!alive) break;
    if (threadIdx.x < KR) {
      const int j = threadIdx.x;
      if (!sh.done[j]) {
        sh.inner[j] += sh.kin[j];
        if (sh.kin[j] > sh.inner_max[j]) sh.inner_max[j] = sh.kin[j];
      }
    }

    // ---- heavy-ball update per column (owners) and relative-step partials
    double s0 = 0.0, s1 = 0.0;
    for (int idx = threadIdx.x; idx < nown * KR; idx += kBlock) {
      const int c = c_lo + idx / KR, j = idx % KR;
      if (j >= e.ncols || sh.done[j]) continue;
      const int64_t o = (int64_t)c * KR + j;
      double* xp = e.X + (int64_t)c * e.ldx + j;
      const double xc = *xp;
      const double xn = xc + sh.alpha[j] * Z[o] + sh.beta[j] * (xc - XP[o]);
      XP[o] = xc;
      *xp = xn;
      s0 += (xn - xc) * (xn - xc);
      s1 += xn * xn;
    }
    column_partials(s0, myscal + 2 * KR, sh.red);
    column_partials(s1, myscal + 3 * KR, sh.red);
    if (!(alive = team_sync(e, epoch, a.err, s_flag, a.spin))) break;
    team_slot_sums(scal, T, 2 * KR, sh.ufin, sh.red);
    team_slot_sums(scal, T, 3 * KR, sh.acg, sh.red);
    int all_done = 1;
    if (threadIdx.x < KR) {
      const int j = threadIdx.x;
      if (!sh.done[j]) {
        sh.outer[j] += 1;
        const double st = sh.acg[j] > 0.0 ? sqrt(sh.ufin[j] / sh.acg[j]) : 0.0;
        sh.step[j] = st;
        if (sh.thr[j] > 0.0 && st <= sh.thr[j]) sh.done[j] = 1;
      }
    }
    __syncthreads();
    for (int j = 0; j < KR; ++j) all_done &= sh.done[j];
    if (all_done) {
      status_all = MIHS_CONVERGED;
      ++outer;
      break;
    }
  }
  if (rank == 0 && threadIdx.x < KR && threadIdx.x < e.ncols) {
    const int j = threadIdx.x;
    mihs_info_t* inf = e.info + j;
    inf->outer_iters = sh.outer[j];
    inf->inner_iters_total = sh.inner[j];
    inf->inner_iters_max = sh.inner_max[j];
    inf->rel_step = sh.step[j];
    inf->grad_norm = sh.gnorm[j];
    inf->status = !alive ? MIHS_BARRIER_TIMEOUT
                         : ((sh.thr[j] > 0.0 && sh.done[j]) ? MIHS_CONVERGED : MIHS_MAX_ITER);
    inf->reserved = 0;
  }
  (void)status_all;
  __syncthreads();
}

template <int DPMAX>
__global__ __launch_bounds__(kBlock) void batched_kernel(BatchArgs a) {
  extern __shared__ double tile[];
  __shared__ Shared sh;
  const int* items = a.wg_items + (int64_t)blockIdx.x * a.items_stride;
  for (int i = 0; i < a.items_stride; ++i) {
    const int ei = items[i];
    if (ei < 0) break;
    const BatchEntry e = a.entries[ei];
    const int rank = (int)blockIdx.x - e.team0;
    // each entry runs at its own padded width (<= DPMAX)
    if (e.dp <= 64) run_entry<64>(a, e, rank, tile, sh);
    else if (DPMAX >= 128 && e.dp <= 128) run_entry<(DPMAX >= 128 ? 128 : 64)>(a, e, rank, tile, sh);
    else if (DPMAX >= 256 && e.dp <= 256) run_entry<(DPMAX >= 256 ? 256 : 64)>(a, e, rank, tile, sh);
    else if (DPMAX >= 512 && e.dp <= 512) run_entry<(DPMAX >= 512 ? 512 : 64)>(a, e, rank, tile, sh);
    else if (DPMAX >= 1024) run_entry<(DPMAX >= 1024 ? 1024 : 64)>(a, e, rank, tile, sh);
  }
}

typedef void (*BatchKernel)(BatchArgs);

BatchKernel pick(int dp) {
  switch (dp) {
    case 64: return batched_kernel<64>;
    case 128: return batched_kernel<128>;
    case 256: return batched_kernel<256>;
    case 512: return batched_kernel<512>;
    case 1024: return batched_kernel<1024>;
    default: return nullptr;
  }
}

int dp_for(int64_t d) {
  int dp = 64;
  while (dp < d) dp *= 2;
  return dp;
}

size_t tile_bytes(int dp) { return (size_t)TROWS * (dp + 1) * sizeof(double); }

}  // namespace

int block_max_d() { return 1024; }

size_t block_workspace_bytes(const BlockEntryDesc* ents, int64_t count, int num_cu) {
  // entries + items + per-entry scratch (assume the largest possible team) + barriers
  size_t total = align_up((size_t)count * sizeof(BatchEntry), 256);
  total += align_up((size_t)num_cu * (size_t)(count + 1) * sizeof(int), 256);
  for (int64_t i = 0; i < count; ++i) {
    const int dp = dp_for(ents[i].d);
    total += align_up(entry_layout(dp, num_cu).total * sizeof(double), 256);
  }
  total += align_up((size_t)(count + 2) * 128, 256);
  return total;
}

int launch_block(const mihs_handle* h, const BlockEntryDesc* ents, int64_t count, int a_f32,
                 int sa_f32, double eps_sub, double tol, int64_t max_outer, int64_t max_inner,
                 void* ws, size_t ws_bytes, hipStream_t st) {
  if (count <= 0) return MIHS_OK;
  int dpmax = 64;
  for (int64_t i = 0; i < count; ++i) {
    if (ents[i].d < 1 || ents[i].d > block_max_d() || ents[i].ncols < 1 || ents[i].ncols > KR)
      return MIHS_ERR_INVALID;
    dpmax = std::max(dpmax, dp_for(ents[i].d));
  }
  BatchKernel kern = pick(dpmax);
  if (!kern) return MIHS_ERR_UNSUPPORTED;
  const size_t shmem = tile_bytes(dpmax);
  if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)shmem) != hipSuccess)
    return MIHS_ERR_HIP;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kBlock, shmem) != hipSuccess)
    return MIHS_ERR_HIP;
  if (occ < 1) return MIHS_ERR_UNSUPPORTED;
  const int G = h->num_cu * std::min(occ, 1);

  // ---- schedule: large entries get dedicated teams, small ones share bins
  std::vector<double> wgt(count);
  double total = 0.0;
  for (int64_t i = 0; i < count; ++i) {
    const double inner_est = 12.0;  // typical inner iterations per outer iteration
    wgt[i] = (double)ents[i].n * ents[i].d + inner_est * (double)ents[i].m * ents[i].d;
    total += wgt[i];
  }
  std::vector<int64_t> order(count);
  for (int64_t i = 0; i < count; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return wgt[x] > wgt[y]; });
  std::vector<int> team0(count, 0), tsize(count, 1);
  std::vector<std::vector<int>> items(G);
  const double per_wg = total / G;
  int next = 0;  // next free workgroup for dedicated teams
  int64_t first_small = count;
  for (int64_t oi = 0; oi < count; ++oi) {
    const int64_t i = order[oi];
    const int want = (int)std::floor(wgt[i] / per_wg);
    if (want >= 2 && next + want <= G - 1) {
      team0[i] = next;
      tsize[i] = want;
      for (int t = 0; t < want; ++t) items[next + t].push_back((int)i);
      next += want;
    } else {
      first_small = oi;
      break;
    }
  }
  // remaining entries: greedy bin packing over the free workgroups
  std::vector<double> load(G, 0.0);
  for (int64_t oi = first_small; oi < count; ++oi) {
    const int64_t i = order[oi];
    int best = next;
    for (int g = next; g < G; ++g)
      if (load[g] < load[best]) best = g;
    if (next >= G) return MIHS_ERR_UNSUPPORTED;
    team0[i] = best;
    tsize[i] = 1;
    items[best].push_back((int)i);
    load[best] += wgt[i];
  }
  size_t stride = 1;
  for (int g = 0; g < G; ++g) stride = std::max(stride, items[g].size() + 1);

  // ---- workspace: entries, items, per-entry scratch, barrier lines, error flag
  char* base = (char*)ws;
  size_t off = 0;
  const size_t ent_off = off;
  off = align_up(off + (size_t)count * sizeof(BatchEntry), 256);
  const size_t item_off = off;
  off = align_up(off + (size_t)G * stride * sizeof(int), 256);
  std::vector<size_t> work_off(count);
  for (int64_t i = 0; i < count; ++i) {
    work_off[i] = off;
    off = align_up(off + entry_layout(dp_for(ents[i].d), tsize[i]).total * sizeof(double), 256);
  }
  const size_t bar_off = off;
  off = align_up(off + (size_t)(count + 2) * 128, 256);
  if (!ws || off > ws_bytes) return MIHS_ERR_WORKSPACE;

  std::vector<BatchEntry> host(count);
  for (int64_t i = 0; i < count; ++i) {
    const BlockEntryDesc& s = ents[i];
    BatchEntry& e = host[i];
    e.A = s.A;
    e.n = s.n;
    e.lda = s.lda;
    e.B = s.B;
    e.ldb = s.ldb;
    e.ldbc = s.ldbc;
    e.RHS = s.RHS;
    e.ldr = s.ldr;
    e.SA = s.SA;
    e.m = s.m;
    e.ldsa = s.ldsa;
    e.X = s.X;
    e.ldx = s.ldx;
    e.lam = s.lam;
    e.alpha = s.alpha;
    e.beta = s.beta;
    e.info = s.info;
    e.work = (double*)(base + work_off[i]);
    e.bar = (unsigned*)(base + bar_off + (size_t)(i + 1) * 128);
    e.d = (int)s.d;
    e.dp = dp_for(s.d);
    e.ncols = s.ncols;
    e.team0 = team0[i];
    e.tsize = tsize[i];
  }
  std::vector<int> hitems((size_t)G * stride, -1);
  for (int g = 0; g < G; ++g)
    for (size_t k = 0; k < items[g].size(); ++k) hitems[(size_t)g * stride + k] = items[g][k];

  if (hipMemcpyAsync(base + ent_off, host.data(), (size_t)count * sizeof(BatchEntry),
                     hipMemcpyHostToDevice, st) != hipSuccess)
    return MIHS_ERR_HIP;
  if (hipMemcpyAsync(base + item_off, hitems.data(), hitems.size() * sizeof(int),
                     hipMemcpyHostToDevice, st) != hipSuccess)
    return MIHS_ERR_HIP;
  if (hipMemsetAsync(base + bar_off, 0, (size_t)(count + 2) * 128, st) != hipSuccess)
    return MIHS_ERR_HIP;
  // the host tables above are freed when this function returns
  if (hipStreamSynchronize(st) != hipSuccess) return MIHS_ERR_HIP;

  BatchArgs a;
  a.entries = (const BatchEntry*)(base + ent_off);
  a.wg_items = (const int*)(base + item_off);
  a.items_stride = (int)stride;
  a.err = (int*)(base + bar_off);
  a.a_f32 = a_f32;
  a.sa_f32 = sa_f32;
  a.eps_sub = eps_sub;
  a.tol = tol;
  a.max_outer = max_outer;
  a.max_inner = max_inner;
  a.spin.limit = 1L << 26;
  a.spin.sleep = 1;
  void* args[] = {&a};
  if (hipLaunchCooperativeKernel((const void*)kern, dim3(G), dim3(kBlock), args, shmem, st) !=
      hipSuccess)
    return MIHS_ERR_HIP;
  return MIHS_OK;
}

}  // namespace mihs
