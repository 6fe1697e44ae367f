// Persistent M-IHS solve kernel (Algorithm 1 with a CG inner solver).
//
// One cooperative launch runs the whole outer loop.  All G workgroups stream
// A; a subgroup of the first Gc workgroups runs the inner solve, so the inner
// loop only pays for a small, fast barrier.  Phases:
//
//   A1  (all G)  stage x in LDS; stream this workgroup's contiguous row block
//       of A once: each wave holds whole rows in registers, forms
//       r_i = b_i - A_i x by a wave reduction and accumulates A_i^T r_i into
//       per-lane partial gradients; the four waves combine in LDS and write one
//       partial d-vector.                                   -> barrier (all)
//   A2  (Gc)     column owners add the G partials (fixed order), form
//       g = sum + rhs - lambda x and start CG (z = 0, r = p = g).  -> barrier (Gc)
//   CG  (Gc)     per iteration two barriers:
//       C1  every CG workgroup forms p = r + beta_cg p_prev in LDS (owners
//           also store their slice) and streams its rows of SA:
//           u_j = SA_j p, partial -SA^T u, sum u_j^2.        -> barrier (Gc)
//       C2  p^T q = ||u||^2 + lambda ||p||^2 (scalar partials, fixed order);
//           owners form q = -sum + lambda p and update z, r. -> barrier (Gc)
//       The stop test ||r|| <= eps_sub ||g|| uses sums every CG workgroup
//       computes identically, so they all leave the loop together.
//   U   (Gc)     owners apply x+ = x + alpha z + beta (x - x_prev) and write
//       the relative-step partials.                          -> barrier (all)
//       Every workgroup then evaluates the same stop test.
//
// Every reduction runs in a fixed order, so a solve is bit-reproducible.
#include <math.h>
#include <stdlib.h>

#include <algorithm>

#include "device_util.hpp"
#include "internal.hpp"

namespace mihs {

namespace {

constexpr int kScal = 8;           // scalar partial slots per workgroup
constexpr double kCg1MaxCond = 1e5;  // single-reduction CG up to this trace(H)/lambda
constexpr int kMaxBlocksPerCU = 2;
constexpr int kQuarterRows = 4;    // rows per group in rowpass_quarters

struct SolveArgs {
  const void* A;
  int64_t n;
  int64_t lda;
  const double* b;
  const double* rhs;
  const void* SA;
  int64_t m;
  int64_t ldsa;
  double lam, alpha, beta, eps_sub, step_thr;
  int64_t max_outer, max_inner;
  double* x;
  double* xp;
  int xp_from_x;
  mihs_info_t* info;
  double* partA;   // G x dpad
  void* partS;     // Gc x dpad (TV)
  double* scal;    // G x kScal
  void* r;
  void* z;
  void* p0;
  void* p1;
  unsigned* bar_all;  // 9 lines (hierarchical barrier)
  unsigned* bar_cg;   // 1 line (flat inner-solve barrier)
  unsigned* bar_cgh;  // 9 lines (hierarchical inner-solve barrier)
  int* err;
  int* status;        // decision published by the CG group
  const void* H;      // Gram matrix (SA)^T SA (TS), dpad x dpad, when the CG uses it
  int64_t ldh;
  int cg1;            // Gram path: single-reduction CG (one barrier per step)
  int aab;            // streaming path: AAb_Solver (Algorithm 6) instead of CG
  double* yrow;       // AAb: m doubles, -(M v - theta p) of each row of SA
  const int* skip;    // when set and nonzero the launch returns at once
  int d, dpad, G, Gc, cpw;
  int cg_hier;        // inner-solve group large enough for the two-level barrier
  int32_t xw[kXcds];  // gradient-pass row weight of each XCD (row_split_bound)
  BarrierSpin spin_fast, spin_idle;
};

// Rows loaded per wave step: enough bytes in flight for short rows, one row
// when the row buffer and the EPT accumulators already fill the registers.
template <typename TM, int EPT>
struct RowsInFlight {
  static constexpr int kBytes = EPT * (int)sizeof(TM);   // bytes per lane per row
  static constexpr int value =
      (kBytes >= 512 || (EPT >= 32 && sizeof(TM) < 8)) ? 1 : (kBytes >= 256 ? 2 : 4);
};

// One pass over rows [r0, r1) of M: for each row, u = cs c_row - M_row . v and
// acc += u * M_row (acc in this lane's columns), ssq += u^2; u is also stored
// to uout[row] when uout is set (uout may alias c: each row is read before it
// is written, by the same wave).
template <typename TM, typename TV, int EPT, bool NT, int R>
__device__ __forceinline__ void rowpass(const TM* __restrict__ M, int64_t ld, int64_t r0,
                                        int64_t r1, int d, const TV* __restrict__ v,
                                        const double* c, TV (&acc)[EPT], TV& ssq,
                                        double cs = 1.0, double* uout = nullptr) {
  using L = RowLayout<TM, EPT>;
  const int lane = lane_id();
  for (int64_t row = r0 + (int64_t)wave_id() * R; row < r1; row += (int64_t)kWavesPerBlock * R) {
    TM rv[R][EPT];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      if (row + t < r1) {
        load_row<TM, EPT, NT>(M + (row + t) * ld, d, lane, rv[t]);
      } else {
#pragma unroll
        for (int e = 0; e < EPT; ++e) rv[t][e] = TM(0);
      }
    }
    TV dot[R];
#pragma unroll
    for (int t = 0; t < R; ++t) dot[t] = TV(0);
#pragma unroll
    for (int j = 0; j < L::J; ++j) {
#pragma unroll
      for (int vv = 0; vv < L::V; ++vv) {
        const TV xv = v[L::col(j, lane, vv)];
#pragma unroll
        for (int t = 0; t < R; ++t) dot[t] += (TV)rv[t][j * L::V + vv] * xv;
      }
    }
#pragma unroll
    for (int t = 0; t < R; ++t) dot[t] = wave_sum(dot[t]);
#pragma unroll
    for (int t = 0; t < R; ++t) {
      TV u = TV(0);
      if (row + t < r1) {
        u = (c ? (TV)(cs * c[row + t]) : TV(0)) - dot[t];
        if (uout && lane == 0) uout[row + t] = (double)u;
      }
      ssq += u * u;
#pragma unroll
      for (int e = 0; e < EPT; ++e) acc[e] += u * (TV)rv[t][e];
    }
  }
}

// Workgroup barrier without the memory fence of __syncthreads, whose release
// would wait for every load in flight (here: the next rows, fetched ahead).
// The caller waits for its own LDS writes first (lgkmcnt(0)); the empty asm
// statements keep the compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// The gradient pass for rows too long for one wave's registers (d > 2048): the
// four waves split every row into quarters of 64 * EQ columns, each lane holding
// EQ entries of its wave's quarter.  Per group of R rows every wave forms its
// partial dot products, they meet in LDS (double-buffered, one barrier per
// group), and each wave accumulates u_i * A_i on its own quarter, so no
// cross-wave reduction is needed at the end.  The next group's rows are loaded
// before the current group is processed.  u_i = c_i - A_i . v (c may be null).
template <typename TM, int EQ, bool NT, int R>
__device__ __forceinline__ void rowpass_quarters(const TM* __restrict__ M, int64_t ld, int64_t r0,
                                                 int64_t r1, int d, const double* __restrict__ v,
                                                 const double* __restrict__ c, double (&acc)[EQ],
                                                 double* s_part) {
  using L = RowLayout<TM, EQ>;
  // fetch the next group during this one only while both fit in registers
  constexpr bool PF = R * EQ * (int)sizeof(TM) <= 256;
  const int lane = lane_id(), w = wave_id();
  const int q0 = w * kWave * EQ;  // first column of this wave's quarter
  const int dq = d - q0;          // valid columns from q0 (may be <= 0)
  double vr[EQ];
#pragma unroll
  for (int j = 0; j < L::J; ++j)
#pragma unroll
    for (int vv = 0; vv < L::V; ++vv) vr[j * L::V + vv] = v[q0 + L::col(j, lane, vv)];
  auto load_group = [&](int64_t row0, TM (&buf)[R][EQ]) {
#pragma unroll
    for (int t = 0; t < R; ++t) {
      if (row0 + t < r1) {
        load_row<TM, EQ, NT>(M + (row0 + t) * ld + q0, dq, lane, buf[t]);
      } else {
#pragma unroll
        for (int e = 0; e < EQ; ++e) buf[t][e] = TM(0);
      }
    }
  };
  TM cur[R][EQ];
  if constexpr (PF) load_group(r0, cur);
  int buf = 0;
  for (int64_t row = r0; row < r1; row += R) {
    TM nxt[R][EQ];
    if constexpr (PF) load_group(row + R, nxt);
    else load_group(row, cur);
    double dot[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      dot[t] = 0.0;
#pragma unroll
      for (int e = 0; e < EQ; ++e) dot[t] += (double)cur[t][e] * vr[e];
      dot[t] = wave_sum(dot[t]);
    }
    if (lane == 0) {
#pragma unroll
      for (int t = 0; t < R; ++t) s_part[(buf * R + t) * kWavesPerBlock + w] = dot[t];
    }
    lds_barrier();
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const double* sp = s_part + (buf * R + t) * kWavesPerBlock;
      const double total = ((sp[0] + sp[1]) + sp[2]) + sp[3];
      const double u = (row + t < r1) ? ((c ? c[row + t] : 0.0) - total) : 0.0;
#pragma unroll
      for (int e = 0; e < EQ; ++e) acc[e] += u * (double)cur[t][e];
    }
    buf ^= 1;
    if constexpr (PF) {
#pragma unroll
      for (int t = 0; t < R; ++t)
#pragma unroll
        for (int e = 0; e < EQ; ++e) cur[t][e] = nxt[t][e];
    }
  }
}

// Store a wave's quarter of the partial vector (rowpass_quarters layout).
template <typename TM, int EQ>
__device__ __forceinline__ void store_quarters(const double (&acc)[EQ], double* out, int d) {
  using L = RowLayout<TM, EQ>;
  const int lane = lane_id();
  const int q0 = wave_id() * kWave * EQ;
#pragma unroll
  for (int j = 0; j < L::J; ++j)
#pragma unroll
    for (int vv = 0; vv < L::V; ++vv) {
      const int col = q0 + L::col(j, lane, vv);
      if (col < d) co_store(out + col, acc[j * L::V + vv]);
    }
}

// Combine the four waves' per-lane partial vectors (fixed wave order) and
// store them to `out[0..d)`.
template <typename TM, typename TV, int EPT>
__device__ __forceinline__ void wg_store_partial(const TV (&acc)[EPT], TV* red, TV* out, int d) {
  using L = RowLayout<TM, EPT>;
  const int lane = lane_id();
#pragma unroll
  for (int w = 0; w < kWavesPerBlock; ++w) {
    if (wave_id() == w) {
#pragma unroll
      for (int j = 0; j < L::J; ++j)
#pragma unroll
        for (int vv = 0; vv < L::V; ++vv) {
          const int col = L::col(j, lane, vv);
          red[col] = (w == 0 ? TV(0) : red[col]) + acc[j * L::V + vv];
        }
    }
    __syncthreads();
  }
  for (int col = threadIdx.x; col < d; col += kBlock) co_store(out + col, red[col]);
}

template <typename TV>
__device__ __forceinline__ TV wg_sum_ssq(TV ssq, double* s_red) {
  // every lane of a wave holds the same ssq; combine the four waves in order
  __syncthreads();
  if (lane_id() == 0) s_red[wave_id()] = (double)ssq;
  __syncthreads();
  double t = s_red[0];
  for (int w = 1; w < kWavesPerBlock; ++w) t += s_red[w];
  return (TV)t;
}

// Two workgroup sums at once (fixed wave order, the same result as two
// block_sum calls, with one pair of barriers).
__device__ __forceinline__ void block_sum2(double& a, double& b, double* s_red2) {
  a = wave_sum(a);
  b = wave_sum(b);
  __syncthreads();
  if (lane_id() == 0) {
    s_red2[2 * wave_id()] = a;
    s_red2[2 * wave_id() + 1] = b;
  }
  __syncthreads();
  a = s_red2[0];
  b = s_red2[1];
  for (int w = 1; w < kWavesPerBlock; ++w) {
    a += s_red2[2 * w];
    b += s_red2[2 * w + 1];
  }
}

// Two scalar sums over K workgroups' slots (fixed order), returned to every thread.
__device__ __forceinline__ void sum2_slots(const double* scal, int K, int s0, int s1,
                                           double* s_red2, double& o0, double& o1) {
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < K; k += kBlock) {
    a += co_load(scal + (int64_t)k * kScal + s0);
    b += co_load(scal + (int64_t)k * kScal + s1);
  }
  a = wave_sum(a);
  b = wave_sum(b);
  __syncthreads();
  if (lane_id() == 0) {
    s_red2[2 * wave_id()] = a;
    s_red2[2 * wave_id() + 1] = b;
  }
  __syncthreads();
  o0 = s_red2[0];
  o1 = s_red2[1];
  for (int w = 1; w < kWavesPerBlock; ++w) {
    o0 += s_red2[2 * w];
    o1 += s_red2[2 * w + 1];
  }
}

// Column sums over K partial vectors for this workgroup's owned columns,
// out[i] = sum_k P[k * ldp + c0 + i], with every load of a thread issued before
// any is used (one memory round trip for K <= 16 * threads-per-column).
template <typename T>
__device__ __forceinline__ void owned_column_sums(const T* __restrict__ P, int K, int64_t ldp,
                                                  int c0, int ncols, double* out,
                                                  double* scratch) {
  constexpr int NB = 16;
  for (int cc0 = 0; cc0 < ncols; cc0 += kBlock) {
    const int CC = min(kBlock, ncols - cc0);
    int TPC = 1;
    while (TPC * 2 * CC <= kBlock) TPC *= 2;
    const int t = threadIdx.x;
    const int col = t % CC, ks = t / CC;
    double s = 0.0;
    if (ks < TPC) {
      const T* base = P + c0 + cc0 + col;
      for (int k0 = ks; k0 < K; k0 += NB * TPC) {
        T v[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const int k = k0 + i * TPC;
          v[i] = (k < K) ? co_load(base + (int64_t)k * ldp) : T(0);
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) s += (double)v[i];
      }
    }
    __syncthreads();
    scratch[t] = s;
    __syncthreads();
    if (t < CC) {
      double acc = scratch[t];
      for (int i = 1; i < TPC; ++i) acc += scratch[i * CC + t];
      out[cc0 + t] = acc;
    }
    __syncthreads();
  }
}

// out[c - r0] = H[c, :] . v for rows c in [r0, r1), in a fixed order.  Each
// wave loads R rows before using any: a CG workgroup owns few rows, so this is
// usually one round trip.
template <typename TH, typename TV, int EPT, int R>
__device__ __forceinline__ void rowdots_r(const TH* __restrict__ H, int64_t ldh, int r0, int r1,
                                          int d, const TV* __restrict__ v, double* out) {
  using L = RowLayout<TH, EPT>;
  const int lane = lane_id();
  for (int c = r0 + wave_id() * R; c < r1; c += kWavesPerBlock * R) {
    TH rv[R][EPT];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      if (c + t < r1) {
        load_row<TH, EPT, false>(H + (int64_t)(c + t) * ldh, d, lane, rv[t]);
      } else {
#pragma unroll
        for (int e = 0; e < EPT; ++e) rv[t][e] = TH(0);
      }
    }
    TV dot[R];
#pragma unroll
    for (int t = 0; t < R; ++t) dot[t] = TV(0);
#pragma unroll
    for (int j = 0; j < L::J; ++j) {
#pragma unroll
      for (int vv = 0; vv < L::V; ++vv) {
        const TV xv = v[L::col(j, lane, vv)];
#pragma unroll
        for (int t = 0; t < R; ++t) dot[t] += (TV)rv[t][j * L::V + vv] * xv;
      }
    }
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const TV sdot = wave_sum(dot[t]);
      if (lane == 0 && c + t < r1) out[c + t - r0] = (double)sdot;
    }
  }
}

// Rows per wave: up to 512 bytes per lane in flight (at most 4 rows), halved
// when the workgroup owns too few rows to give every wave a full set.  Rows of
// 4096 entries keep one row in flight: a second FP32 row spilled the solve
// kernel's registers to scratch (89 VGPRs), which cost more than the extra
// round trip saves.
template <typename TH, typename TV, int EPT>
__device__ __forceinline__ void rowdots(const TH* __restrict__ H, int64_t ldh, int r0, int r1,
                                        int d, const TV* __restrict__ v, double* out) {
  constexpr int RB = (EPT >= 64 ? 256 : 512) / (EPT * (int)sizeof(TH));
  constexpr int R = RB < 1 ? 1 : (RB > 4 ? 4 : RB);
  if constexpr (R > 1) {
    if (r1 - r0 <= kWavesPerBlock * (R / 2)) {
      rowdots_r<TH, TV, EPT, R / 2>(H, ldh, r0, r1, d, v, out);
      return;
    }
  }
  rowdots_r<TH, TV, EPT, R>(H, ldh, r0, r1, d, v, out);
}

// Barrier of the inner-solve group: one counter for small groups, the two-level
// form (per-XCD counters, then one top counter) from 256 workgroups on, where
// one counter's arrivals queue up (128 workgroups: 2.1 us either way; 256:
// 3.8 us flat against 2.2 us two-level).
__device__ __forceinline__ bool cg_sync(const SolveArgs& a, unsigned& epoch, int* s_flag) {
  return a.cg_hier ? barrier_hier(a.bar_cgh, epoch, a.Gc, a.err, s_flag, a.spin_fast)
                   : barrier_flat(a.bar_cg, epoch, a.Gc, a.err, s_flag, a.spin_fast);
}

// GRAM: the inner CG applies (SA)^T SA through the precomputed H (owners form
// their entries of q directly); otherwise through two passes over SA rows.
template <typename TA, typename TS, typename TV, int EPT, bool GRAM>
__global__ __launch_bounds__(kBlock) void solve_kernel(SolveArgs a) {
  // a driver that enqueues several solves ahead stops them once it is done
  if (a.skip && __hip_atomic_load(a.skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  extern __shared__ double smem[];
  const int cpw = a.cpw;
  double* vbuf = smem;                 // x (A pass) or p (CG, as TV)
  double* rbuf = vbuf + a.dpad;        // workgroup reduction buffer
  double* colbuf = rbuf + a.dpad;      // owned-column sums
  double* scratch = colbuf + cpw;      // kBlock doubles
  double* own_x = scratch + kBlock;    // owner-private state of the owned columns
  double* own_xp = own_x + cpw;
  double* own_rhs = own_xp + cpw;
  TV* own_r = (TV*)(own_rhs + cpw);
  TV* own_z = (TV*)(own_rhs + 2 * cpw);
  __shared__ double s_red[2 * kWavesPerBlock];
  __shared__ double s_part[2 * kQuarterRows * kWavesPerBlock];  // rowpass_quarters exchange
  __shared__ int s_flag;

  const int w = blockIdx.x;
  const int G = a.G, Gc = a.Gc;
  const int d = a.d;
  const bool in_cg = w < Gc;
  unsigned ep_all = 0, ep_cg = 0;
  const int c_lo = in_cg ? min(d, w * cpw) : d;
  const int c_hi = in_cg ? min(d, c_lo + cpw) : d;
  const int nown = c_hi - c_lo;
  double* scal_w = a.scal + (int64_t)w * kScal;
  // CG vectors exchanged between the CG workgroups: every access goes through
  // co_store / co_load (agent-scope, global address space)
  TV* r = (TV*)a.r;
  TV* P[2] = {(TV*)a.p0, (TV*)a.p1};
  TV* partS = (TV*)a.partS;
  const TA* A = (const TA*)a.A;
  const TS* SA = (const TS*)a.SA;
  constexpr int RA = RowsInFlight<TA, EPT>::value;
  constexpr int RS = RowsInFlight<TS, EPT>::value;
  constexpr int NPT = EPT >= 4 ? EPT / 4 : 1;  // vector entries per thread (dpad / kBlock)

  for (int i = threadIdx.x; i < nown; i += kBlock) {
    const int c = c_lo + i;
    own_x[i] = a.x[c];
    own_xp[i] = a.xp_from_x ? a.x[c] : a.xp[c];
    own_rhs[i] = a.rhs ? a.rhs[c] : 0.0;
  }
  // this workgroup's rows of the CG operator H (read from L2 / Infinity Cache
  // on every step; keeping them in LDS measured slower: the step is bound by
  // its barrier and round trips, not by these reads)
  const TS* Hrows = (GRAM && in_cg) ? (const TS*)a.H + (int64_t)c_lo * a.ldh : nullptr;
  const int64_t ldhr = a.ldh;
  __syncthreads();

  // Single-reduction CG only where the sub-problem is well conditioned for its
  // precision: trace(H) / lambda bounds kappa(H + lambda I) from above.  Every CG
  // workgroup sums the same diagonal in the same order, so all decide alike.
  bool cg1 = false;
  if (GRAM && a.cg1 && in_cg) {
    const TS* Hm = (const TS*)a.H;
    double tr = 0.0;
    for (int c = threadIdx.x; c < d; c += kBlock) tr += (double)Hm[(int64_t)c * a.ldh + c];
    tr = block_sum(tr, s_red);
    cg1 = tr <= kCg1MaxCond * a.lam;
  }

  const int64_t a_r0 = row_split_bound(a.n, G, a.xw, w);
  const int64_t a_r1 = row_split_bound(a.n, G, a.xw, w + 1);
  const int64_t s_r0 = in_cg ? a.m * w / Gc : 0;
  const int64_t s_r1 = in_cg ? a.m * (w + 1) / Gc : 0;

  int64_t outer = 0, inner_total = 0, inner_max = 0;
  double last_step = 0.0, last_gnorm = 0.0;
  int status = MIHS_MAX_ITER;
  bool alive = true;

  // x in LDS for the first gradient pass; later passes get it at the end of
  // the previous iteration, fetched together with the stop test's sums
  for (int c = threadIdx.x; c < a.dpad; c += kBlock) vbuf[c] = (c < d) ? co_load(a.x + c) : 0.0;
  __syncthreads();
  while (outer < a.max_outer) {
    // ---- A1 (all): partial A^T (b - A x) over this workgroup's rows
    if constexpr (EPT == 64) {
      double acc[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[e] = 0.0;
      rowpass_quarters<TA, 16, true, kQuarterRows>(A, a.lda, a_r0, a_r1, d, vbuf, a.b, acc, s_part);
      store_quarters<TA, 16>(acc, a.partA + (int64_t)w * a.dpad, d);
      __syncthreads();
    } else {
      double acc[EPT];
#pragma unroll
      for (int e = 0; e < EPT; ++e) acc[e] = 0.0;
      double ssq = 0.0;
      rowpass<TA, double, EPT, true, RA>(A, a.lda, a_r0, a_r1, d, vbuf, a.b, acc, ssq);
      wg_store_partial<TA, double, EPT>(acc, rbuf, a.partA + (int64_t)w * a.dpad, d);
    }
    if (!(alive = barrier_hier(a.bar_all, ep_all, G, a.err, &s_flag, a.spin_fast))) break;

    int decision = 0;  // 0 continue, 1 converged, 2 breakdown
    if (in_cg) {
      // ---- A2: owners form g and start CG (z = 0, r = p = g)
      owned_column_sums(a.partA, G, a.dpad, c_lo, nown, colbuf, scratch);
      double rr_part = 0.0;
      for (int i = threadIdx.x; i < nown; i += kBlock) {
        const TV gt = (TV)(colbuf[i] + own_rhs[i] - a.lam * own_x[i]);
        own_r[i] = gt;
        own_z[i] = TV(0);
        co_store(r + c_lo + i, gt);
        co_store(P[0] + c_lo + i, gt);
        rr_part += (double)gt * (double)gt;
      }
      rr_part = block_sum(rr_part, s_red);
      if (threadIdx.x == 0) co_store(scal_w + 0, rr_part);
      if (!(alive = cg_sync(a, ep_cg, &s_flag))) break;

      // the single-reduction CG starts from the whole of r = g: its loads are
      // issued before the slot sum
      TV rpre[NPT];
      if (GRAM && cg1) {
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
          const int c = threadIdx.x + i * kBlock;
          rpre[i] = (c < d) ? co_load(r + c) : TV(0);
        }
      }
      double rr0, unused;
      sum2_slots(a.scal, Gc, 0, 0, s_red, rr0, unused);
      last_gnorm = sqrt(rr0);
      int64_t k = 0;
      if (!(rr0 > 0.0)) {
        decision = (rr0 == 0.0) ? 1 : 2;  // stationary point, or NaN
      } else {
        const double stop = a.eps_sub * a.eps_sub * rr0;
        if (!GRAM && a.aab) {
          // AAb_Solver (Algorithm 6) on ((SA)^T SA + lambda I) z = g: Golub-Kahan
          // bidiagonalisation of M = SA started from v = g / ||g||, the
          // sqrt(lambda) I block folded in by Givens rotations.  One pass over
          // the owned rows of M per step gives y = M v - theta p and M^T y
          // together (p = y_prev / rho_prev is never normalised in memory, the
          // scale rides on the next pass), then two barriers: one for rho = ||y||
          // and M^T y, one for theta = ||w||, w = M^T p - rho v.  Every CG
          // workgroup keeps v in LDS and the same scalars; owners keep the
          // direction vector (in own_r) and the iterate z on their columns.
          TV* vp = (TV*)vbuf;
          TV* wv = r;  // w, exchanged through the residual buffer
          TV* dv = own_r;
          const double theta1 = sqrt(rr0);
          for (int c = threadIdx.x; c < a.dpad; c += kBlock)
            vp[c] = (c < d) ? (TV)((double)co_load(r + c) / theta1) : TV(0);
          __syncthreads();
          double theta = 0.0, rho_prev = 1.0, rhobar = 0.0, cs = 0.0, sn = 0.0, phi = 0.0;
          bool first = true;
          while (true) {
            TV ssq = TV(0);
            {
              TV acc[EPT];
#pragma unroll
              for (int e = 0; e < EPT; ++e) acc[e] = TV(0);
              // u = -(M v - theta p) = (-theta / rho_prev) y_prev - M v
              rowpass<TS, TV, EPT, false, RS>(SA, a.ldsa, s_r0, s_r1, d, vp,
                                              first ? nullptr : a.yrow, acc, ssq,
                                              -theta / rho_prev, a.yrow);
              wg_store_partial<TS, TV, EPT>(acc, (TV*)rbuf, partS + (int64_t)w * a.dpad, d);
              ssq = wg_sum_ssq(ssq, s_red);
            }
            if (threadIdx.x == 0) co_store(scal_w + 1, (double)ssq);
            if (!(alive = cg_sync(a, ep_cg, &s_flag))) break;
            // colbuf = -M^T y on the owned columns; rho = ||y||
            owned_column_sums(partS, Gc, a.dpad, c_lo, nown, colbuf, scratch);
            double rho2, unused2;
            sum2_slots(a.scal, Gc, 1, 1, s_red, rho2, unused2);
            const double rho = sqrt(rho2);
            double t;
            if (first) {
              rhobar = sqrt(rho * rho + a.lam);
              cs = rho / rhobar;
              sn = sqrt(a.lam) / rhobar;
              phi = theta1 / rhobar;
              for (int i = threadIdx.x; i < nown; i += kBlock) {
                const TV dn = (TV)((double)vp[c_lo + i] / rhobar);
                dv[i] = dn;
                own_z[i] = (TV)(phi * (double)dn);
              }
              t = INFINITY;
              first = false;
            } else {
              const double lbar = sqrt(a.lam + (sn * theta) * (sn * theta));
              const double thetabar = cs * theta;
              rhobar = sqrt(rho * rho + lbar * lbar);
              cs = rho / rhobar;
              sn = lbar / rhobar;
              phi = -phi * thetabar / rhobar;
              for (int i = threadIdx.x; i < nown; i += kBlock) {
                const TV dn =
                    (TV)(((double)vp[c_lo + i] - thetabar * (double)dv[i]) / rhobar);
                dv[i] = dn;
                own_z[i] = own_z[i] + (TV)(phi * (double)dn);
              }
              t = fabs(phi * rhobar) / theta1;
              ++k;
            }
            if (!isfinite(phi) || !isfinite(rhobar)) {
              decision = 2;
              break;
            }
            // stop on the relative residual of the current iterate; rho = 0
            // ends the Krylov space (the iterate is then exact)
            if (!(t >= a.eps_sub) || k >= a.max_inner || !(rho > 0.0)) break;
            // w = M^T p - rho v = (M^T y) / rho - rho v on the owned columns
            double th_part = 0.0;
            for (int i = threadIdx.x; i < nown; i += kBlock) {
              const TV wc = (TV)(-colbuf[i] / rho - rho * (double)vp[c_lo + i]);
              co_store(wv + c_lo + i, wc);
              th_part += (double)wc * (double)wc;
            }
            th_part = block_sum(th_part, s_red);
            if (threadIdx.x == 0) co_store(scal_w + 2, th_part);
            if (!(alive = cg_sync(a, ep_cg, &s_flag))) break;
            double th2;
            sum2_slots(a.scal, Gc, 2, 2, s_red, th2, unused2);
            theta = sqrt(th2);
            if (!(theta > 0.0)) break;  // w = 0: the iterate is exact
            rho_prev = rho;
            for (int c = threadIdx.x; c < a.dpad; c += kBlock)
              vp[c] = (c < d) ? (TV)((double)co_load(wv + c) / theta) : TV(0);
            __syncthreads();
          }
          if (!alive) break;
        } else if (GRAM && cg1) {
          // Single-reduction CG (Chronopoulos-Gear): with s = M p kept by its own
          // recurrence, one matrix product (w = M r on the owned rows) and one
          // fused reduction (r^T r, w^T r) per step, so one barrier per step.
          // Every CG workgroup keeps full copies of r and s in LDS (identical
          // arithmetic everywhere), gathers w from global memory (two buffers,
          // alternating) and owns p and z on its columns.
          TV* rv = (TV*)vbuf;
          TV* sv = (TV*)rbuf;
          const TV lt = (TV)a.lam;
#pragma unroll
          for (int i = 0; i < NPT; ++i) {
            const int c = threadIdx.x + i * kBlock;
            if (c < a.dpad) rv[c] = rpre[i];
          }
          __syncthreads();
          int wb = 0;
          double mu = rr0, alpha = 0.0, unused2;
          {
            rowdots<TS, TV, EPT>(Hrows, ldhr, 0, nown, d, rv, colbuf);
            __syncthreads();
            double nu_part = 0.0;
            for (int i = threadIdx.x; i < nown; i += kBlock) {
              const TV rc = rv[c_lo + i];
              const TV wc = (TV)colbuf[i] + lt * rc;
              co_store(P[wb] + c_lo + i, wc);
              nu_part += (double)wc * (double)rc;
            }
            nu_part = block_sum(nu_part, s_red);
            if (threadIdx.x == 0) co_store(scal_w + 1, nu_part);
            if (!(alive = cg_sync(a, ep_cg, &s_flag))) break;
#pragma unroll
            for (int i = 0; i < NPT; ++i) {
              const int c = threadIdx.x + i * kBlock;
              rpre[i] = (c < d) ? co_load(P[wb] + c) : TV(0);  // w, for s below
            }
            double nu;
            sum2_slots(a.scal, Gc, 1, 1, s_red, nu, unused2);
            alpha = mu / nu;
            if (!(nu > 0.0) || !isfinite(alpha)) decision = 2;
          }
          if (decision == 0) {
            // s = w, p = r
#pragma unroll
            for (int i = 0; i < NPT; ++i) {
              const int c = threadIdx.x + i * kBlock;
              if (c < a.dpad) sv[c] = rpre[i];
            }
            for (int i = threadIdx.x; i < nown; i += kBlock) own_r[i] = rv[c_lo + i];
            __syncthreads();
            while (true) {
              const TV at = (TV)alpha;
              for (int i = threadIdx.x; i < nown; i += kBlock) own_z[i] = own_z[i] + at * own_r[i];
              for (int c = threadIdx.x; c < a.dpad; c += kBlock) rv[c] = rv[c] - at * sv[c];
              __syncthreads();
              ++k;
              wb ^= 1;
              rowdots<TS, TV, EPT>(Hrows, ldhr, 0, nown, d, rv, colbuf);
              __syncthreads();
              double mu_p = 0.0, nu_p = 0.0;
              for (int i = threadIdx.x; i < nown; i += kBlock) {
                const TV rc = rv[c_lo + i];
                const TV wc = (TV)colbuf[i] + lt * rc;
                co_store(P[wb] + c_lo + i, wc);
                mu_p += (double)rc * (double)rc;
                nu_p += (double)wc * (double)rc;
              }
              block_sum2(mu_p, nu_p, s_red);
              // the step's scalar slots alternate like w: one barrier separates
              // a step's reads of a slot pair from its next write (two steps on)
              const int sp = 2 + 4 * wb;
              if (threadIdx.x == 0) {
                co_store(scal_w + sp, mu_p);
                co_store(scal_w + sp + 1, nu_p);
              }
              if (!(alive = cg_sync(a, ep_cg, &s_flag))) break;
              // fetch w (written by every CG workgroup before the barrier) while
              // the scalar partials are summed
              TV wpre[NPT];
#pragma unroll
              for (int i = 0; i < NPT; ++i) {
                const int c = threadIdx.x + i * kBlock;
                wpre[i] = (c < d) ? co_load(P[wb] + c) : TV(0);
              }
              double mu_n, nu_n;
              sum2_slots(a.scal, Gc, sp, sp + 1, s_red, mu_n, nu_n);
              if (mu_n <= stop || k >= a.max_inner) break;
              const double bt = mu_n / mu;
              const double den = nu_n - bt * mu_n / alpha;
              const double an = mu_n / den;
              if (!(den > 0.0) || !isfinite(an)) {
                decision = 2;
                break;
              }
              mu = mu_n;
              alpha = an;
              // s = w + beta s (full), p = r + beta p (owned)
              const TV btt = (TV)bt;
#pragma unroll
              for (int i = 0; i < NPT; ++i) {
                const int c = threadIdx.x + i * kBlock;
                if (c < a.dpad) sv[c] = wpre[i] + btt * sv[c];
              }
              for (int i = threadIdx.x; i < nown; i += kBlock)
                own_r[i] = rv[c_lo + i] + btt * own_r[i];
              __syncthreads();
            }
          }
          if (!alive) break;
        } else {
          double rr = rr0;
          TV* vp = (TV*)vbuf;
          while (true) {
            // ---- C1: p = r + beta_cg p_prev (k > 0), staged in LDS over p_prev
            // (every CG workgroup holds the whole of p: the same arithmetic on the
            // same values everywhere).  The loads of r and of the residual
            // partials are all issued before use; the first direction is g.
            TV rv[NPT], pv[NPT];
#pragma unroll
            for (int i = 0; i < NPT; ++i) {
              const int c = threadIdx.x + i * kBlock;
              rv[i] = TV(0);
              pv[i] = TV(0);
              if (c < d) {
                if (k == 0) {
                  rv[i] = co_load(P[0] + c);
                } else {
                  rv[i] = co_load(r + c);
                  pv[i] = vp[c];
                }
              }
            }
            TV bc = TV(0);
            if (k > 0) {
              double rr_new;
              sum2_slots(a.scal, Gc, 3, 3, s_red, rr_new, unused);
              if (rr_new <= stop || k >= a.max_inner) break;
              bc = (TV)(rr_new / rr);
              rr = rr_new;
            }
#pragma unroll
            for (int i = 0; i < NPT; ++i) {
              const int c = threadIdx.x + i * kBlock;
              if (c < a.dpad) {
                const TV p = (k == 0) ? rv[i] : (TV)(rv[i] + bc * pv[i]);
                vp[c] = (c < d) ? p : TV(0);
              }
            }
            for (int c = NPT * kBlock + threadIdx.x; c < a.dpad; c += kBlock) vp[c] = TV(0);
            __syncthreads();
            double rpart = 0.0;
            if (GRAM) {
              // q = H p + lambda p on the owned columns (colbuf <- H p)
              rowdots<TS, TV, EPT>(Hrows, ldhr, 0, nown, d, vp, colbuf);
              __syncthreads();
              double pq = 0.0;
              for (int i = threadIdx.x; i < nown; i += kBlock) {
                const double pc = (double)vp[c_lo + i];
                pq += pc * (colbuf[i] + a.lam * pc);
              }
              pq = block_sum(pq, s_red);
              if (threadIdx.x == 0) co_store(scal_w + 1, pq);
              if (!(alive = cg_sync(a, ep_cg, &s_flag))) break;
              double pqs, unused2;
              sum2_slots(a.scal, Gc, 1, 1, s_red, pqs, unused2);
              const double acg = rr / pqs;
              if (!(pqs > 0.0) || !isfinite(acg)) {
                decision = 2;
                break;
              }
              const TV at = (TV)acg, lt = (TV)a.lam;
              for (int i = threadIdx.x; i < nown; i += kBlock) {
                const TV pc = vp[c_lo + i];
                const TV q = (TV)colbuf[i] + lt * pc;
                own_z[i] = own_z[i] + at * pc;
                const TV rn = own_r[i] - at * q;
                own_r[i] = rn;
                co_store(r + c_lo + i, rn);
                rpart += (double)rn * (double)rn;
              }
            } else {
              TV ssq = TV(0);
              {
                TV acc[EPT];
#pragma unroll
                for (int e = 0; e < EPT; ++e) acc[e] = TV(0);
                rowpass<TS, TV, EPT, false, RS>(SA, a.ldsa, s_r0, s_r1, d, vp, nullptr, acc, ssq);
                wg_store_partial<TS, TV, EPT>(acc, (TV*)rbuf, partS + (int64_t)w * a.dpad, d);
                ssq = wg_sum_ssq(ssq, s_red);
              }
              double pp = 0.0;
              for (int c = c_lo + threadIdx.x; c < c_hi; c += kBlock)
                pp += (double)vp[c] * (double)vp[c];
              pp = block_sum(pp, s_red);
              if (threadIdx.x == 0) {
                co_store(scal_w + 1, pp);
                co_store(scal_w + 2, (double)ssq);
              }
              if (!(alive = cg_sync(a, ep_cg, &s_flag))) break;

              // ---- C2: step length (p^T q = ||u||^2 + lambda ||p||^2) and owner updates
              owned_column_sums(partS, Gc, a.dpad, c_lo, nown, colbuf, scratch);
              double ppn, uu;
              sum2_slots(a.scal, Gc, 1, 2, s_red, ppn, uu);
              const double pq = uu + a.lam * ppn;
              const double acg = rr / pq;
              if (!(pq > 0.0) || !isfinite(acg)) {
                decision = 2;
                break;
              }
              const TV at = (TV)acg, lt = (TV)a.lam;
              for (int i = threadIdx.x; i < nown; i += kBlock) {
                const TV pc = vp[c_lo + i];
                const TV q = (TV)(-colbuf[i]) + lt * pc;
                own_z[i] = own_z[i] + at * pc;
                const TV rn = own_r[i] - at * q;
                own_r[i] = rn;
                co_store(r + c_lo + i, rn);
                rpart += (double)rn * (double)rn;
              }
            }
            rpart = block_sum(rpart, s_red);
            if (threadIdx.x == 0) co_store(scal_w + 3, rpart);
            if (!(alive = cg_sync(a, ep_cg, &s_flag))) break;
            ++k;
          }

        }
        if (!alive) break;
      }
      inner_total += k;
      if (k > inner_max) inner_max = k;

      // ---- U: heavy-ball update on owned columns
      double s0 = 0.0, s1 = 0.0;
      if (decision == 0) {
        for (int i = threadIdx.x; i < nown; i += kBlock) {
          const double xc = own_x[i];
          const double xn = xc + a.alpha * (double)own_z[i] + a.beta * (xc - own_xp[i]);
          own_xp[i] = xc;
          own_x[i] = xn;
          co_store(a.x + c_lo + i, xn);
          s0 += (xn - xc) * (xn - xc);
          s1 += xn * xn;
        }
      }
      s0 = block_sum(s0, s_red);
      s1 = block_sum(s1, s_red);
      if (threadIdx.x == 0) {
        co_store(scal_w + 4, s0);
        co_store(scal_w + 5, s1);
        if (w == 0) co_store(a.status, decision);
      }
    }
    if (!(alive = barrier_hier(a.bar_all, ep_all, G, a.err, &s_flag,
                               in_cg ? a.spin_fast : a.spin_idle)))
      break;
    // the updated x (owners stored it before the barrier), the decision and the
    // step sums: all loads issued before any is used
    double xpre[NPT];
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int c = threadIdx.x + i * kBlock;
      xpre[i] = (c < d) ? co_load(a.x + c) : 0.0;
    }
    decision = __hip_atomic_load(a.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (decision == 1) {
      status = MIHS_CONVERGED;
      break;
    }
    if (decision == 2) {
      status = MIHS_BREAKDOWN;
      break;
    }
    double S0, S1;
    sum2_slots(a.scal, Gc, 4, 5, s_red, S0, S1);
    ++outer;
    last_step = S1 > 0.0 ? sqrt(S0 / S1) : 0.0;
    if (!isfinite(last_step)) {
      status = MIHS_BREAKDOWN;
      break;
    }
    if (a.step_thr > 0.0 && last_step <= a.step_thr) {
      status = MIHS_CONVERGED;
      break;
    }
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int c = threadIdx.x + i * kBlock;
      if (c < a.dpad) vbuf[c] = xpre[i];
    }
    __syncthreads();
  }
  if (!alive) status = MIHS_BARRIER_TIMEOUT;
  // publish the momentum state (the iterate before x) of the owned columns
  for (int i = threadIdx.x; i < nown; i += kBlock) a.xp[c_lo + i] = own_xp[i];
  if (w == 0 && threadIdx.x == 0) {
    a.info->outer_iters = outer;
    a.info->inner_iters_total = inner_total;
    a.info->inner_iters_max = inner_max;
    a.info->rel_step = last_step;
    a.info->grad_norm = last_gnorm;
    a.info->status = status;
    a.info->elapsed_us = 0;
  }
}

// The gradient pass of Algorithm 1 on its own: partial A^T (c - A x) of one row
// block per workgroup (c = b, or none), then a fixed-order column sum that adds
// rhs and subtracts lambda x.  Used by drivers whose inner step is not CG.
template <typename TA, int EPT>
__global__ __launch_bounds__(kBlock) void grad_partial_kernel(const TA* A, int64_t n, int64_t lda,
                                                              int d, int dpad, const double* c,
                                                              const double* x, double* part,
                                                              const int* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  extern __shared__ double smem[];
  double* vbuf = smem;
  double* rbuf = smem + dpad;
  for (int k = threadIdx.x; k < dpad; k += kBlock) vbuf[k] = (k < d) ? x[k] : 0.0;
  __syncthreads();
  const int64_t G = gridDim.x, w = blockIdx.x;
  const int64_t r0 = n * w / G, r1 = n * (w + 1) / G;
  if constexpr (EPT == 64) {
    __shared__ double s_part[2 * kQuarterRows * kWavesPerBlock];
    double acc[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] = 0.0;
    rowpass_quarters<TA, 16, true, kQuarterRows>(A, lda, r0, r1, d, vbuf, c, acc, s_part);
    store_quarters<TA, 16>(acc, part + w * dpad, d);
  } else {
    double acc[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) acc[e] = 0.0;
    double ssq = 0.0;
    rowpass<TA, double, EPT, true, RowsInFlight<TA, EPT>::value>(A, lda, r0, r1, d, vbuf, c,
                                                                   acc, ssq);
    wg_store_partial<TA, double, EPT>(acc, rbuf, part + w * dpad, d);
  }
}

// 32 columns per workgroup; the 8 thread rows of a column sum interleaved
// partials (t = q, q + 8, ...) and meet in LDS in a fixed order.
constexpr int kFinCols = 32;
__global__ __launch_bounds__(kBlock) void grad_finish_kernel(const double* part, int G, int dpad,
                                                             int d, const double* rhs,
                                                             const double* x, double lam,
                                                             double* g, const int* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  __shared__ double red[kBlock / kFinCols][kFinCols];
  constexpr int Q = kBlock / kFinCols;
  const int cl = threadIdx.x % kFinCols, q = threadIdx.x / kFinCols;
  const int k = blockIdx.x * kFinCols + cl;
  double s = 0.0;
  if (k < d)
    for (int t = q; t < G; t += Q) s += part[(int64_t)t * dpad + k];
  red[q][cl] = s;
  __syncthreads();
  if (q == 0 && k < d) {
    double tot = red[0][cl];
    for (int i = 1; i < Q; ++i) tot += red[i][cl];
    if (rhs) tot += rhs[k];
    g[k] = tot - lam * x[k];
  }
}

template <typename TA, int EPT>
int launch_grad_partial(int G, size_t shmem, hipStream_t stream, const TA* A, int64_t n,
                        int64_t lda, int d, int dpad, const double* c, const double* x,
                        double* part, const int* skip) {
  if (hipFuncSetAttribute((const void*)grad_partial_kernel<TA, EPT>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem) != hipSuccess)
    return MIHS_ERR_HIP;
  hipLaunchKernelGGL((grad_partial_kernel<TA, EPT>), dim3(G), dim3(kBlock), shmem, stream, A, n,
                     lda, d, dpad, c, x, part, skip);
  return MIHS_OK;
}

template <typename TA>
int launch_grad_partial_ept(int ept, int G, size_t shmem, hipStream_t stream, const TA* A,
                            int64_t n, int64_t lda, int d, int dpad, const double* c,
                            const double* x, double* part, const int* skip) {
  switch (ept) {
    case 1:
      return launch_grad_partial<TA, 1>(G, shmem, stream, A, n, lda, d, dpad, c, x, part,
                                          skip);
    case 2:
      return launch_grad_partial<TA, 2>(G, shmem, stream, A, n, lda, d, dpad, c, x, part,
                                          skip);
    case 4:
      return launch_grad_partial<TA, 4>(G, shmem, stream, A, n, lda, d, dpad, c, x, part,
                                          skip);
    case 8:
      return launch_grad_partial<TA, 8>(G, shmem, stream, A, n, lda, d, dpad, c, x, part,
                                          skip);
    case 16:
      return launch_grad_partial<TA, 16>(G, shmem, stream, A, n, lda, d, dpad, c, x, part,
                                          skip);
    case 32:
      return launch_grad_partial<TA, 32>(G, shmem, stream, A, n, lda, d, dpad, c, x, part,
                                          skip);
    case 64:
      return launch_grad_partial<TA, 64>(G, shmem, stream, A, n, lda, d, dpad, c, x, part,
                                          skip);
    default: return MIHS_ERR_UNSUPPORTED;
  }
}

__global__ void zero_words(unsigned* p, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0u;
}

typedef void (*SolveKernel)(SolveArgs);

template <typename TA, typename TS, typename TV, bool GRAM>
SolveKernel pick_by_ept(int ept) {
  switch (ept) {
    case 1: return solve_kernel<TA, TS, TV, 1, GRAM>;
    case 2: return solve_kernel<TA, TS, TV, 2, GRAM>;
    case 4: return solve_kernel<TA, TS, TV, 4, GRAM>;
    case 8: return solve_kernel<TA, TS, TV, 8, GRAM>;
    case 16: return solve_kernel<TA, TS, TV, 16, GRAM>;
    case 32: return solve_kernel<TA, TS, TV, 32, GRAM>;
    case 64: return solve_kernel<TA, TS, TV, 64, GRAM>;
    default: return nullptr;
  }
}

// Mixed precision stores the inner solver's operator (SA, or its Gram matrix)
// in FP32, which halves the bytes every inner step streams, and keeps the CG
// recurrences (vectors, step lengths, dot products) in FP64: FP32 recurrences
// lose their conjugacy on ill-conditioned sub-problems (kappa ~ 6e8: 87k inner
// steps against 27k, measured), and in this latency-bound loop the FP64
// vectors cost about 1% at the headline size.
template <bool GRAM>
SolveKernel pick_kernel(int a_f32, int mixed, int ept) {
  if (!a_f32 && !mixed) return pick_by_ept<double, double, double, GRAM>(ept);
  if (!a_f32 && mixed) return pick_by_ept<double, float, double, GRAM>(ept);
  if (a_f32 && !mixed) return pick_by_ept<float, double, double, GRAM>(ept);
  return pick_by_ept<float, float, double, GRAM>(ept);
}

// The CG goes through the Gram matrix when it is no larger than SA (m >= d).
bool use_gram(int64_t m, int64_t d) { return m >= d; }

struct SolveLayout {
  size_t partA, partS, scal, vecs, xp, bar, gram, yrow, total;
};

// Barrier region: line 0 = top counter of the all-workgroup barrier, lines 1-8
// its group counters, line 9 = inner-solve group counter, line 10 = error flag,
// line 11 = status word, lines 12-20 = top and group counters of the two-level
// inner-solve barrier (128-byte lines).
constexpr size_t kBarLines = 21;

// gram_bytes: size of the Gram matrix region (0 when the CG streams SA).
SolveLayout layout(int G, int Gc, int64_t dpad, size_t gram_bytes, int64_t m) {
  SolveLayout L;
  size_t off = 0;
  L.partA = off; off = align_up(off + (size_t)G * dpad * 8, 256);
  L.partS = off; off = align_up(off + (size_t)Gc * dpad * 8, 256);
  L.scal = off;  off = align_up(off + (size_t)G * kScal * 8, 256);
  L.vecs = off;  off = align_up(off + 4 * (size_t)dpad * 8, 256);
  L.xp = off;    off = align_up(off + (size_t)dpad * 8, 256);
  L.bar = off;   off = align_up(off + kBarLines * 128, 256);
  L.gram = off;  off = align_up(off + gram_bytes, 256);
  L.yrow = off;  off = align_up(off + (size_t)m * 8, 256);
  L.total = off;
  return L;
}

size_t gram_bytes_for(int64_t m, int64_t d, int mixed) {
  if (!use_gram(m, d)) return 0;
  const size_t dp = (size_t)dpad_for(d);
  return dp * dp * (mixed ? sizeof(float) : sizeof(double));
}

int max_grid(const mihs_handle* h) { return h->num_cu * kMaxBlocksPerCU; }

// Size of the inner-solve subgroup: enough workgroups to stream the operator
// quickly, few enough that its barrier stays cheap.  Operators of 8 MB and
// more take 256 workgroups (one per CU for the usual 512-workgroup grid) with
// the two-level barrier: measured at 2^18 x 2048 (16 MB FP32 Gram matrix,
// per CG step 4.2 -> 2.9 us of row products) and at 2^20 x 4096 (64 MB,
// 19.2 -> 13.4 us), the barrier costing no more than a flat one over 128.
// `forced` > 0 fixes the size.
int pick_cg_groups(int64_t m, int64_t d, int sa_bytes, int G, bool gram, int forced) {
  int gc;
  if (forced > 0) {
    gc = forced;
  } else {
    // bytes one CG step streams: the Gram matrix (m >= d) or SA
    const double mb = (double)(gram ? d : m) * (double)d * sa_bytes / (1024.0 * 1024.0);
    gc = mb >= 8.0 ? 256 : (mb >= 4.0 ? 64 : (mb >= 1.0 ? 32 : 16));
    // each CG workgroup should own at least a few rows
    const int64_t by_rows = (m + 3) / 4;
    if (gc > by_rows) gc = (int)(by_rows < 1 ? 1 : by_rows);
  }
  if (gc > G) gc = G;
  if (gc < 1) gc = 1;
  return gc;
}

}  // namespace

// ---- scratch of the entry point without a workspace argument -------------
// mihs_solve_noalloc runs the solve kernels on this array instead of a caller
// workspace: one copy per GPU, held by the loaded code object until the process
// ends.  In host code the name is only a stand-in for the symbol (passing it
// to a kernel would make the kernel fault): every host use goes through the
// device address that noalloc_scratch_address() returns, which differs per GPU.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

int noalloc_scratch_address(void** ptr) {
  // call with the handle's device current: each GPU holds its own copy
  *ptr = nullptr;
  if (hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch)) != hipSuccess || *ptr == nullptr)
    return MIHS_ERR_HIP;
  return MIHS_OK;
}

int ept_for(int64_t d) {
  int e = 1;
  while (64 * (int64_t)e < d) e *= 2;
  return e;
}

size_t solve_workspace_bytes(const mihs_handle* h, int64_t n, int64_t d, int64_t m, int mixed,
                             int no_gram) {
  (void)n;
  const int G = max_grid(h);
  return layout(G, G, dpad_for(d), no_gram ? 0 : gram_bytes_for(m, d, mixed), m).total;
}

int grad_partials(const mihs_handle* h, int64_t n, int64_t d) {
  int64_t g = (int64_t)h->num_cu * kMaxBlocksPerCU;
  const int64_t by_rows = (n + 63) / 64;
  if (g > by_rows) g = by_rows < 1 ? 1 : by_rows;
  (void)d;
  return (int)g;
}

size_t grad_workspace_bytes(const mihs_handle* h, int64_t n, int64_t d) {
  return align_up((size_t)grad_partials(h, n, d) * (size_t)dpad_for(d) * 8, 256);
}

int launch_grad(const mihs_handle* h, const void* A, int a_f32, int64_t n, int64_t d,
                int64_t lda, const double* c, const double* rhs, const double* x, double lam,
                double* g, void* ws, size_t ws_bytes, const int* skip, hipStream_t stream) {
  const int ept = ept_for(d);
  if (ept > 64) return MIHS_ERR_UNSUPPORTED;
  if (ws_bytes < grad_workspace_bytes(h, n, d) || ws == nullptr) return MIHS_ERR_WORKSPACE;
  const int dpad = (int)dpad_for(d);
  const size_t shmem = 2 * (size_t)dpad * sizeof(double);
  const int G = grad_partials(h, n, d);
  double* part = (double*)ws;
  const int rc = a_f32 ? launch_grad_partial_ept<float>(ept, G, shmem, stream, (const float*)A, n,
                                                        lda, (int)d, dpad, c, x, part, skip)
                       : launch_grad_partial_ept<double>(ept, G, shmem, stream, (const double*)A,
                                                         n, lda, (int)d, dpad, c, x, part, skip);
  if (rc) return rc;
  hipLaunchKernelGGL(grad_finish_kernel, dim3((unsigned)((d + kFinCols - 1) / kFinCols)),
                     dim3(kBlock), 0, stream, part, G, dpad, (int)d, rhs, x, lam, g, skip);
  return hipGetLastError() == hipSuccess ? MIHS_OK : MIHS_ERR_HIP;
}

int launch_solve(const mihs_handle* h, const SolveDesc& s, void* ws, size_t ws_bytes,
                 hipStream_t stream) {
  const int ept = ept_for(s.d);
  if (ept > 64) return MIHS_ERR_UNSUPPORTED;
  // AAb_Solver needs M v and M^T p separately: it always streams SA
  const bool gram = !s.no_gram && !s.aab && use_gram(s.m, s.d);
  SolveKernel kern = gram ? pick_kernel<true>(s.a_f32, s.mixed, ept)
                          : pick_kernel<false>(s.a_f32, s.mixed, ept);
  if (!kern) return MIHS_ERR_UNSUPPORTED;
  const int64_t dpad = dpad_for(s.d);
  // Pick the grid: try two workgroups per CU, then one; the inner-solve group
  // size (and with it the LDS request) depends on the grid.
  int G = 0, Gc = 0, cpw = 0;
  size_t shmem = 0;
  // keep >= ~64 rows of A per workgroup (unless the caller fixes another count)
  const int64_t rows_per_wg = s.rows_per_wg > 0 ? s.rows_per_wg : 64;
  const int64_t g_rows = (s.n + rows_per_wg - 1) / rows_per_wg;
  for (int occ_try = kMaxBlocksPerCU; occ_try >= 1; --occ_try) {
    int g = h->num_cu * occ_try;
    if ((int64_t)g > g_rows) g = (int)(g_rows < 1 ? 1 : g_rows);
    const int gc = pick_cg_groups(s.m, s.d, s.mixed ? 4 : 8, g, gram, s.cg_groups);
    const int cp = (int)((s.d + gc - 1) / gc);
    const size_t sh = (2 * (size_t)dpad + 6 * (size_t)cp + kBlock) * sizeof(double);
    if (sh > 160 * 1024) continue;
    if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sh) != hipSuccess)
      return MIHS_ERR_HIP;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kBlock, sh) != hipSuccess)
      return MIHS_ERR_HIP;
    if (occ >= occ_try || (occ >= 1 && (int64_t)g <= (int64_t)h->num_cu * occ)) {
      G = g;
      Gc = gc;
      cpw = cp;
      shmem = sh;
      break;
    }
  }
  if (G == 0) return MIHS_ERR_UNSUPPORTED;
  const SolveLayout L = layout(G, Gc, dpad, gram ? gram_bytes_for(s.m, s.d, s.mixed) : 0, s.m);
  if (ws_bytes < L.total || ws == nullptr) return MIHS_ERR_WORKSPACE;

  char* base = (char*)ws;
  SolveArgs a;
  a.A = s.A;
  a.n = s.n;
  a.lda = s.lda;
  a.b = s.b;
  a.rhs = s.rhs;
  a.SA = s.SA;
  a.m = s.m;
  a.ldsa = s.ldsa;
  a.lam = s.lam;
  a.alpha = s.alpha;
  a.beta = s.beta;
  a.eps_sub = s.eps_sub;
  a.step_thr = (s.tol > 0.0 && s.beta > 0.0 && s.beta < 1.0)
                   ? s.tol * (1.0 - sqrt(s.beta)) / sqrt(s.beta)
                   : (s.tol > 0.0 ? s.tol : 0.0);
  a.max_outer = s.max_outer;
  a.max_inner = s.max_inner;
  a.x = s.x;
  a.xp = s.x_prev ? s.x_prev : (double*)(base + L.xp);
  a.xp_from_x = s.x_prev ? 0 : 1;
  a.info = s.info;
  a.partA = (double*)(base + L.partA);
  a.partS = (void*)(base + L.partS);
  a.scal = (double*)(base + L.scal);
  a.r = (void*)(base + L.vecs);
  a.z = (void*)(base + L.vecs + (size_t)dpad * 8);
  a.p0 = (void*)(base + L.vecs + 2 * (size_t)dpad * 8);
  a.p1 = (void*)(base + L.vecs + 3 * (size_t)dpad * 8);
  unsigned* bar = (unsigned*)(base + L.bar);
  a.bar_all = bar;
  a.bar_cg = bar + 9 * 32;
  a.bar_cgh = bar + 12 * 32;
  a.cg_hier = Gc > 128 ? 1 : 0;
  for (int k = 0; k < kXcds; ++k) a.xw[k] = h->row_weight[k];
  a.err = (int*)(bar + 10 * 32);
  a.status = (int*)(bar + 11 * 32);
  a.d = (int)s.d;
  a.dpad = (int)dpad;
  a.G = G;
  a.Gc = Gc;
  a.cpw = cpw;
  a.spin_fast.limit = 1L << 26;  // ~64-clock polls: a few seconds at most
  a.spin_fast.sleep = 1;
  a.spin_idle.limit = 1L << 24;  // ~1000-clock polls while the inner solve runs
  a.spin_idle.sleep = 16;
  a.H = gram ? (const void*)(base + L.gram) : nullptr;
  a.ldh = dpad;
  // One barrier per CG step pays off where the CG is latency-bound (headline,
  // FP64: 32.2 -> 29.4 ms per solve); the two-reduction form keeps fewer steps
  // on very ill-conditioned solves (measured on the CountSketch workload,
  // kappa ~ 6e8: FP64 22k vs 27-38k steps; FP32 breaks down), so the kernel
  // takes the single-reduction form only where trace(H) / lambda is small.
  a.cg1 = 1;
  a.aab = s.aab ? 1 : 0;
  a.yrow = (double*)(base + L.yrow);
  a.skip = s.skip;
  if (gram && !s.gram_ready) {
    const int rc = launch_gram(s.SA, s.mixed, s.m, s.d, s.ldsa, base + L.gram, s.mixed, dpad,
                               stream);
    if (rc) return rc;
  }

  hipLaunchKernelGGL(zero_words, dim3(1), dim3(256), 0, stream, bar, (int)(kBarLines * 32));
  if (hipGetLastError() != hipSuccess) return MIHS_ERR_HIP;
  void* args[] = {&a};
  if (hipLaunchCooperativeKernel((const void*)kern, dim3(G), dim3(kBlock), args, shmem, stream) !=
      hipSuccess)
    return MIHS_ERR_HIP;
  return MIHS_OK;
}

// ---- per-XCD row weights of the gradient pass --------------------------------
// The gradient pass streams A once per outer iteration in contiguous row ranges,
// one workgroup per CU; its length is that of the slowest workgroup.  XCDs do
// not all stream from HBM at the same rate: on MI355X, with equal shares of an
// FP64 matrix of 2048 columns, the odd-numbered XCDs took 6-8% longer than the
// even ones, on every pass (a plain 16-byte stream shows about half of that, so
// the measurement below runs the gradient pass's own row loop).  The rows are
// shared out by per-XCD weights measured here.

constexpr int kCalCols = 2048;                      // FP64 columns of the timing matrix
constexpr int64_t kCalRows = (int64_t)1 << 17;      // 2 GiB (> the Infinity Cache)
constexpr int kCalWarm = 6;    // untimed passes (the first calibration of a process,
                               // with 2, sometimes saw a 14% spread instead of 10%)
constexpr int kCalPasses = 15;  // timed passes; per XCD the median pass counts
constexpr long kRowWeightStep = 4;                  // weights are multiples of this
constexpr size_t kCalLds = 96 * 1024;               // keeps one workgroup per CU

// One workgroup per CU runs the gradient pass's row loop (x = 0) over its equal
// share of the rows and records its start and end wall clock (clk[2w],
// clk[2w + 1]).
__global__ __launch_bounds__(kBlock) void xcd_rowpass_kernel(const double* __restrict__ M,
                                                             long long* clk, double* sink) {
  extern __shared__ double v[];  // kCalCols zeros, then padding
  for (int c = threadIdx.x; c < kCalCols; c += kBlock) v[c] = 0.0;
  __syncthreads();
  const int G = gridDim.x, w = blockIdx.x;
  const long long t0 = wall_clock64();
  constexpr int EPT = kCalCols / kWave;
  double acc[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) acc[e] = 0.0;
  double ssq = 0.0;
  rowpass<double, double, EPT, true, RowsInFlight<double, EPT>::value>(
      M, kCalCols, kCalRows * w / G, kCalRows * (w + 1) / G, kCalCols, v, nullptr, acc, ssq);
  __syncthreads();
  if (threadIdx.x == 0) {
    clk[2 * w] = t0;
    clk[2 * w + 1] = wall_clock64();
  }
  // keeps the arithmetic (never true: the matrix is zero)
  double t = ssq;
#pragma unroll
  for (int e = 0; e < EPT; ++e) t += acc[e];
  if (t == 1.25e300) sink[w] = t;
}

int calibrate_rows(mihs_handle* h) {
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(h->device) != hipSuccess)
    return MIHS_ERR_HIP;
  const int G = h->num_cu;
  char* buf = nullptr;
  const size_t bytes = (size_t)kCalRows * kCalCols * sizeof(double);
  const size_t clk_off = bytes, sink_off = bytes + (size_t)G * 16;
  int rc = MIHS_OK;
  if (G < kXcds || hipMalloc(&buf, sink_off + (size_t)G * 8) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipSetDevice(prev);
    return MIHS_ERR_HIP;
  }
  std::vector<long long> clk((size_t)2 * G);
  std::vector<double> tpass[kXcds];  // per XCD: mean workgroup time of each pass
  if (hipMemset(buf, 0, bytes) != hipSuccess ||
      hipFuncSetAttribute((const void*)xcd_rowpass_kernel,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCalLds) != hipSuccess)
    rc = MIHS_ERR_HIP;
  for (int pass = 0; pass < kCalWarm + kCalPasses && rc == MIHS_OK; ++pass) {
    hipLaunchKernelGGL(xcd_rowpass_kernel, dim3(G), dim3(kBlock), kCalLds, 0, (const double*)buf,
                       (long long*)(buf + clk_off), (double*)(buf + sink_off));
    if (hipGetLastError() != hipSuccess ||
        hipMemcpy(clk.data(), buf + clk_off, clk.size() * sizeof(long long),
                  hipMemcpyDeviceToHost) != hipSuccess) {
      rc = MIHS_ERR_HIP;
      break;
    }
    if (pass < kCalWarm) continue;
    double sum[kXcds] = {0.0};
    int cnt[kXcds] = {0};
    for (int w = 0; w < G; ++w) {
      sum[w % kXcds] += (double)(clk[2 * w + 1] - clk[2 * w]);
      cnt[w % kXcds] += 1;
    }
    for (int k = 0; k < kXcds; ++k) tpass[k].push_back(sum[k] / (double)cnt[k]);
  }
  (void)hipFree(buf);
  (void)hipSetDevice(prev);
  if (rc != MIHS_OK) return rc;
  // Weight (t_min / t)^(3/4) of the fastest XCD's kRowWeightMax, at most a 2:1
  // spread, in steps of kRowWeightStep.  With equal shares the slow XCDs also
  // stream faster once the fast ones are done, so the time ratio overstates the
  // rate ratio under a balanced load: on the headline solve (odd XCDs 7-9%
  // slower at equal shares) weights 64/60 by XCD parity gave 25.10-25.26 ms
  // per solve, 64/56 25.47 ms, equal weights 25.56-25.67 ms.  The steps keep
  // the 1-2% drift of the means between calibrations from moving the split
  // (64/60 with one even XCD at 63 measured 25.36 ms).
  double tk[kXcds], tmin = 0.0;
  for (int k = 0; k < kXcds; ++k) {
    std::vector<double>& v = tpass[k];
    std::nth_element(v.begin(), v.begin() + v.size() / 2, v.end());
    tk[k] = v[v.size() / 2];
    if (!(tk[k] > 0.0)) return MIHS_ERR_HIP;
    if (k == 0 || tk[k] < tmin) tmin = tk[k];
  }
  for (int k = 0; k < kXcds; ++k) {
    const double t = tk[k];
    const long wk =
        kRowWeightStep * lround((double)(kRowWeightMax / kRowWeightStep) * pow(tmin / t, 0.75));
    h->row_weight[k] = (int32_t)std::min<long>(kRowWeightMax, std::max<long>(kRowWeightMax / 2, wk));
  }
  return MIHS_OK;
}

}  // namespace mihs
