// Block M-IHS: many problems, each with up to 16 right-hand sides that share
// one pass over A per outer iteration (a lambda-path shares A, b and SA; the
// backward's adjoint systems share A, SA and lambda).
//
// Before the solve, the Gram matrix H = (SA)^T SA (d x d, FP64) of every
// distinct sketch is formed on the matrix cores; the inner CG applies the
// sub-problem operator as q = H p + lambda p, which costs d^2 per column instead
// of the 2 m d of two passes over SA and needs no reduction across workgroups.
//
// One persistent cooperative launch.  The host scheduler gives each large
// problem a dedicated team of workgroups (synchronised by a team barrier) and
// packs small problems into single-workgroup bins that run them one after the
// other.  Per entry (problem x group of 16 columns) and outer iteration:
//
//   A     for each 16-row tile of A: stage it in LDS, U = C - A_tile X on the
//         matrix cores (v_mfma_f64_16x16x4; the four waves split the d-range and
//         add their partial U in LDS), then G += A_tile^T U for each wave's
//         d-slice; G = A^T (B - A X) (+ RHS) - X diag(lambda), reduced over the team.
//   CG    16 CGs in lockstep on (H + lambda_j I) on the first tcg members of the
//         team (own barrier), each owning a 16-aligned range of columns of q;
//         per-column step lengths and convergence masks; two barriers each.
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
  const void* H;      // Gram matrix (SA)^T SA, dp x dp (FP64, or FP32 with FP32 sketches)
  int64_t ldh;
  double* X;          // X[c * ldx + j], in: start, out: result
  int64_t ldx;
  const double* lam;
  const double* alpha;
  const double* beta;
  mihs_info_t* info;  // ncols records
  double* work;       // per-entry scratch (see entry_layout)
  double* fac;        // exact sub-solves: ncols Cholesky factors, dp x dp each (or null)
  int* fac_bad;       // set when a factorization met a non-positive pivot
  unsigned* bar;      // team barrier counter (own 128-byte line)
  unsigned* bar_cg;   // CG sub-team barrier counter (own 128-byte line)
  int d, dp, ncols;
  int team0, tsize, tcg;
};

struct BatchArgs {
  const BatchEntry* entries;
  const int* wg_items;  // per workgroup: entry indices, -1 terminated
  int items_stride;
  int* err;
  int a_f32, h_f32;
  int a_dma;     // 1: direct-to-LDS row groups where rows are 1-4 KiB
  int exact;     // 1: exact sub-solves with the entries' Cholesky factors
  int wall_khz;  // rate of wall_clock64()
  double eps_sub, tol;
  int64_t max_outer, max_inner;
  BarrierSpin spin, spin_idle;
};

// Scratch of one entry, in doubles: partial block vectors of every team member,
// then R, Z, Q, XP (dp x KR each), then scalar partial slots.
struct EntryLayout {
  size_t part, R, Z, Q, XP, scal, total;
};
__host__ __device__ inline EntryLayout entry_layout(int dp, int tsize) {
  EntryLayout L;
  const size_t blk = (size_t)dp * KR;
  size_t o = 0;
  L.part = o; o += (size_t)tsize * blk;
  L.R = o; o += blk;
  L.Z = o; o += blk;
  L.Q = o; o += blk;
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
// One instance per workgroup, visible to the out-of-line solver phases too.
static __shared__ Shared g_sh;

__device__ __forceinline__ bool group_sync(unsigned* bar, int size, unsigned& epoch, int* err,
                                           int* s_flag, BarrierSpin spin) {
  if (size <= 1) {
    __threadfence_block();
    __syncthreads();
    return true;
  }
  return barrier_flat(bar, epoch, (unsigned)size, err, s_flag, spin);
}

// Sum over the first T slots: out[j] = sum_t scal[t * kNScal + s0 + j], j < KR
// (scal in global memory, out and red in LDS).
__device__ __forceinline__ void team_slot_sums(const double* scal, int T, int s0, double* out,
                                               double* red) {
  // thread (j, q) with j = tid % 16 sums t = q, q + 16, ... ; fixed tree over q
  const int j = threadIdx.x % KR, q = threadIdx.x / KR;
  double v = 0.0;
  for (int t = q; t < T; t += kBlock / KR) v += co_load(scal + (int64_t)t * kNScal + s0 + j);
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

// Per-column sums of values held by all threads (thread tid owns column tid % 16),
// into the global slots `out`.
__device__ __forceinline__ void column_partials(double v, double* out, double* red) {
  __syncthreads();
  red[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x < KR) {
    double a = red[threadIdx.x];
    for (int i = 1; i < kBlock / KR; ++i) a += red[i * KR + threadIdx.x];
    co_store(out + threadIdx.x, a);
  }
  __syncthreads();
}

// Columns of the A pass per wave: the four waves split [0, d) into 16-aligned
// slices (at most DP / 4 each), so a padded width costs nothing past d.
__device__ __forceinline__ int wave_cols(int d, int dp) {
  const int w = ((d + 3) / 4 + 15) / 16 * 16;
  return w < dp / 4 ? w : dp / 4;
}

// Staging of one 16-row tile of M: each thread moves NCH 16-byte chunks
// (coalesced across the workgroup) from global memory into registers, and later
// from registers into the LDS tile (kept in M's own precision, row stride LDT).
template <typename TM, int DP>
struct TileCfg {
  static constexpr int VE = 16 / (int)sizeof(TM);             // elements per chunk
  static constexpr int CPR = DP / VE;                         // chunks per row
  static constexpr int NCH = TROWS * CPR / kBlock;            // chunks per thread
  static constexpr int LDT = DP + (sizeof(TM) == 4 ? 4 : 2);  // LDS row stride (elements)
  static_assert(NCH >= 1 && TROWS * CPR % kBlock == 0, "tile shape");
};

template <typename TM, int DP, bool NT>
__device__ __forceinline__ void tile_load(const TM* __restrict__ M, int64_t ld, int64_t rows,
                                          int d, int64_t row0,
                                          uint4 (&buf)[TileCfg<TM, DP>::NCH]) {
  typedef TileCfg<TM, DP> C;
#pragma unroll
  for (int i = 0; i < C::NCH; ++i) {
    const int ch = i * kBlock + (int)threadIdx.x;
    const int r = ch / C::CPR, c = (ch % C::CPR) * C::VE;
    const int64_t gr = row0 + r;
    // rows are 16-byte aligned (checked at the boundary), so a chunk that starts
    // before column d lies inside the row's aligned span
    if (gr < rows && c < d) {
      typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
      const u32x4* src = (const u32x4*)(M + gr * ld + c);
      const u32x4 v = NT ? __builtin_nontemporal_load(src) : *src;
      buf[i] = make_uint4(v.x, v.y, v.z, v.w);
    } else {
      buf[i] = make_uint4(0u, 0u, 0u, 0u);
    }
  }
}

template <typename TM, int DP>
__device__ __forceinline__ void tile_store(const uint4 (&buf)[TileCfg<TM, DP>::NCH], int d,
                                           TM* tile) {
  typedef TileCfg<TM, DP> C;
#pragma unroll
  for (int i = 0; i < C::NCH; ++i) {
    const int ch = i * kBlock + (int)threadIdx.x;
    const int r = ch / C::CPR, c = (ch % C::CPR) * C::VE;
    union {
      uint4 u;
      TM v[C::VE];
    } x;
    x.u = buf[i];
    if (c + C::VE > d) {
#pragma unroll
      for (int e = 0; e < C::VE; ++e)
        if (c + e >= d) x.v[e] = (TM)0;
    }
    *(uint4*)(tile + r * C::LDT + c) = x.u;
  }
}

// One pass over rows [0, rows) of M (tiles t = rank, rank + T, ...):
//   U = C - M_tile V (C from B), Gacc (this wave's d-slice) += M_tile^T U.
// V is the B operand in registers: Vreg[s] = V[kbase + 4 s + lane/16][lane % 16].
// The global loads of the next one or two tiles are in flight while a tile is
// computed.  ured (4 x 256 doubles)
// and ufin (256 doubles) are LDS scratch.
template <typename TM, int DP, bool NT>
__device__ __forceinline__ void block_pass(const TM* __restrict__ M, int64_t ld, int64_t rows,
                                           int d, int rank, int T, const double* __restrict__ B,
                                           int64_t ldb, int64_t ldbc, int ncols,
                                           const double (&Vreg)[DP / 16],
                                           f64x4 (&Gacc)[DP / 64], void* tile_raw, double* ured,
                                           double* ufin) {
  typedef TileCfg<TM, DP> C;
  constexpr int DQ = DP / 4;   // columns per wave
  constexpr int KS = DQ / 4;   // k-steps per wave
  constexpr int NB = DQ / 16;  // 16-column output blocks per wave
  TM* tile = (TM*)tile_raw;
  const int lane = lane_id(), wave = wave_id();
  const int dqe = wave_cols(d, DP);
  const int kbase = wave * dqe;
  const int rr = threadIdx.x / KR, jj = threadIdx.x % KR;  // (row, column) of U per thread
  const int64_t ntiles = (rows + TROWS - 1) / TROWS;
  // PF tiles in flight: while tile t is computed, t + T (.. t + PF T) are loading;
  // one for the widest rows, where a second register buffer would spill
  constexpr int PF = DP >= 1024 ? 1 : 2;
  auto step = [&](uint4 (&buf)[C::NCH], int64_t t) {
    const int64_t row0 = t * TROWS;
    __syncthreads();  // previous tile fully consumed
    tile_store<TM, DP>(buf, d, tile);
    const int64_t gr = row0 + rr;
    const double cval = (B && gr < rows && jj < ncols) ? B[gr * ldb + jj * ldbc] : 0.0;
    __syncthreads();
    if (t + PF * T < ntiles) tile_load<TM, DP, NT>(M, ld, rows, d, (t + PF * T) * TROWS, buf);
    // partial U over this wave's k-range
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    // (dqe is a multiple of 16: groups of four k-steps are all in or all out)
#pragma unroll
    for (int s4 = 0; s4 < KS; s4 += 4) {
      if (4 * s4 < dqe) {
#pragma unroll
        for (int s = s4; s < s4 + 4; ++s) {
          const double a = (double)tile[(lane & 15) * C::LDT + kbase + 4 * s + (lane >> 4)];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Vreg[s], acc, 0, 0, 0);
        }
      }
      if ((s4 & 7) == 4) __builtin_amdgcn_sched_barrier(0);
    }
    // result register r of lane l: row l/16 + 4 r, column l % 16
#pragma unroll
    for (int r = 0; r < 4; ++r)
      ured[wave * TROWS * KR + ((lane >> 4) + 4 * r) * KR + (lane & 15)] = acc[r];
    __syncthreads();
    {
      double su = 0.0;
#pragma unroll
      for (int w = 0; w < kWavesPerBlock; ++w) su += ured[w * TROWS * KR + rr * KR + jj];
      ufin[rr * KR + jj] = (gr < rows && jj < ncols) ? cval - su : 0.0;
    }
    __syncthreads();
    // Gacc[b] += M_tile[:, slice block b]^T U
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int r2 = 4 * s + (lane >> 4);
        const double a = (double)tile[r2 * C::LDT + kbase + 16 * b + (lane & 15)];
        const double bv = ufin[r2 * KR + (lane & 15)];
        if (16 * b < dqe) Gacc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, Gacc[b], 0, 0, 0);
      }
      if ((b & 1) == 1) __builtin_amdgcn_sched_barrier(0);
    }
  };
  uint4 buf0[C::NCH];
  if (rank < ntiles) tile_load<TM, DP, NT>(M, ld, rows, d, rank * TROWS, buf0);
  if (PF == 1) {
    for (int64_t t = rank; t < ntiles; t += T) step(buf0, t);
  } else {
    uint4 buf1[C::NCH];
    if (rank + T < ntiles) tile_load<TM, DP, NT>(M, ld, rows, d, (rank + T) * TROWS, buf1);
    for (int64_t t = rank; t < ntiles; t += 2 * T) {
      step(buf0, t);
      if (t + T >= ntiles) break;
      step(buf1, t + T);
    }
  }
}

// Store this wave's Gacc (d-slice x 16) to out[c * KR + j].
template <int DP>
__device__ __forceinline__ void store_block(const f64x4 (&Gacc)[DP / 64], int d, double* out) {
  constexpr int DQ = DP / 4;
  const int dqe = wave_cols(d, DP);
  const int lane = lane_id(), kbase = wave_id() * dqe;
#pragma unroll
  for (int b = 0; b < DQ / 16; ++b)
    if (16 * b < dqe) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = kbase + 16 * b + (lane >> 4) + 4 * r;
        co_store(out + (int64_t)c * KR + (lane & 15), Gacc[b][r]);
      }
    }
}

// LDS: the tile region (the two DMA tile buffers of 64 KiB, or 16 rows of the
// widest entry for the register-staged pass; it doubles as the d x 16 vector
// stage), then the U reduction scratch (4 x 256 + 256 doubles) at a fixed offset.
__host__ __device__ constexpr size_t tile_region(int dp) {
  return (size_t)TROWS * (dp + 2) * sizeof(double);
}
constexpr size_t kDmaRegion = 2 * (65536 + 16 * 64);  // two 64 KiB buffers + row padding
constexpr size_t kUredOffset = kDmaRegion > 16 * (1024 + 2) * 8 ? kDmaRegion : 16 * (1024 + 2) * 8;
constexpr size_t kUredBytes = (size_t)(kWavesPerBlock + 1) * TROWS * KR * sizeof(double);
__host__ __device__ constexpr size_t lds_bytes(int dpmax) {
  return (dpmax > 0 ? kUredOffset : 0) + kUredBytes;
}

// Direct-to-LDS tile pipeline (rows of 1-4 KiB): a group of ROWS rows (64 KiB of
// A) lands in one of two LDS buffers through global_load_lds_dwordx4 (64 lanes
// x 16 bytes per instruction, no registers), while the other buffer is computed.
template <typename TM, int DP>
struct DmaCfg {
  static constexpr int RB = DP * (int)sizeof(TM);           // row bytes
  static constexpr bool ok = RB >= 1024 && RB <= 4096;
  static constexpr int ROWS = ok ? 65536 / RB : TROWS;      // rows per group
  static constexpr int TB = ROWS / TROWS;                   // 16-row tiles per group
  static constexpr int CPR = ok ? RB / 1024 : 1;            // 1 KiB chunks per row
  static constexpr int LDB = RB + 16;                       // LDS row stride (bytes)
  static constexpr int LDT = LDB / (int)sizeof(TM);         // ... in elements
  static constexpr int NI = ROWS * CPR / kWavesPerBlock;    // instructions per wave per group
  static constexpr int BUF = ROWS * LDB;                    // bytes per buffer
  static_assert(!ok || (NI == 16 && 2 * BUF <= (int)kDmaRegion), "dma layout");
  static_assert(!ok || (LDB / 4) % 64 == 4, "the LDS row pitch shifts by 4 banks per row");
};

typedef __attribute__((address_space(3))) char lds_char;

// Cache policy of the A-stream loads: non-temporal (A is read once per outer
// iteration; the Gram matrices the inner CG re-reads every step should stay in
// the caches instead).
constexpr int kStreamAux = 2;

// Issue the DMA of rows [row0, row0 + ROWS) into buffer `dst`: lane l of the
// instruction for (row r, chunk c) moves 16 bytes at column c*1024/s + 16 l/s.
// Rows past the end and columns past d read finite in-bounds data instead
// (row rows-1, column 0): their products meet zero operands or are discarded.
template <typename TM, int DP>
__device__ __forceinline__ void dma_group(const TM* __restrict__ M, int64_t ld, int64_t rows,
                                          int d, int64_t row0, lds_char* dst) {
  typedef DmaCfg<TM, DP> C;
  const int lane = lane_id(), wave = wave_id();
#pragma unroll
  for (int i = 0; i < C::NI; ++i) {
    const int q = wave * C::NI + i;
    const int r = q / C::CPR, c = q % C::CPR;
    const int64_t gr = min(row0 + r, rows - 1);
    const int col = c * (1024 / (int)sizeof(TM)) + lane * (16 / (int)sizeof(TM));
    const TM* src = M + gr * ld + (col < d ? col : 0);
    __builtin_amdgcn_global_load_lds((const void*)src, (__attribute__((address_space(3))) void*)(dst + r * C::LDB + c * 1024), 16, 0, kStreamAux);
  }
}

// Waits: vmcnt(16) (16 DMA instructions may stay in flight) and lgkmcnt(0)
// (LDS traffic of this wave done).  Workgroup barriers without the
// memory fence of __syncthreads (whose release would wait for the DMA in
// flight); the empty asm statements keep the compiler from moving memory
// accesses across them.
__device__ __forceinline__ void wait_vm16() { __builtin_amdgcn_s_waitcnt(0x4F70); }
__device__ __forceinline__ void wait_lgkm0() { __builtin_amdgcn_s_waitcnt(0xC07F); }
__device__ __forceinline__ void raw_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <typename TM, int DP>
__device__ __forceinline__ void block_pass_dma(const TM* __restrict__ M, int64_t ld, int64_t rows,
                                               int d, int rank, int T,
                                               const double* __restrict__ B, int64_t ldb,
                                               int64_t ldbc, int ncols,
                                               const double (&Vreg)[DP / 16],
                                               f64x4 (&Gacc)[DP / 64], lds_char* lbase,
                                               double* ured, double* ufin) {
  typedef DmaCfg<TM, DP> C;
  constexpr int DQ = DP / 4, KS = DQ / 4, NB = DQ / 16;
  constexpr int VE = 16 / (int)sizeof(TM);
  const int lane = lane_id(), wave = wave_id();
  const int dqe = wave_cols(d, DP);
  const int kbase = wave * dqe;
  const int rr = threadIdx.x / KR, jj = threadIdx.x % KR;
  const int64_t ngroups = (rows + C::ROWS - 1) / C::ROWS;
  const int dz = (d + VE - 1) / VE * VE;  // columns [d, dz) share a 16-byte chunk with d - 1
  // classic double buffer: group g is computed from one buffer while group g + T
  // lands in the other; the C values of g + T are loaded just before its DMA, so
  // no wait inside the computation involves the DMA in flight
  double cv[2][C::TB];
  auto load_c = [&](double (&c)[C::TB], int64_t g) {
#pragma unroll
    for (int t = 0; t < C::TB; ++t) {
      const int64_t gr = g * C::ROWS + t * TROWS + rr;
      c[t] = (g < ngroups && B && gr < rows && jj < ncols) ? B[gr * ldb + jj * ldbc] : 0.0;
    }
  };
  auto step = [&](double (&c)[C::TB], double (&cnext)[C::TB], int64_t g, lds_char* bufg,
                  lds_char* bufn) {
    const int64_t row0 = g * C::ROWS;
    TM* tileg = (TM*)bufg;
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this group and its C values
    raw_barrier();
    if (dz != d) {  // zero the bytes the last 16-byte chunk carried past d
      for (int e = threadIdx.x; e < C::ROWS * (dz - d); e += kBlock)
        tileg[(e / (dz - d)) * C::LDT + d + e % (dz - d)] = TM(0);
      wait_lgkm0();
      raw_barrier();
    }
    if (g + T < ngroups) {
      load_c(cnext, g + T);
      dma_group<TM, DP>(M, ld, rows, d, (g + T) * C::ROWS, bufn);
    }
#pragma unroll
    for (int t = 0; t < C::TB; ++t) {
      const TM* tile = tileg + t * TROWS * C::LDT;
      const int64_t gr = row0 + t * TROWS + rr;
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
      // (dqe is a multiple of 16: groups of four k-steps are all in or all out).
      // Software pipeline: the tile values of group q + 1 are read from LDS
      // (unconditionally: the tile row is DP wide) before the products of
      // group q, so each group waits only for reads issued one group earlier.
      const TM* arow = tile + (lane & 15) * C::LDT + kbase + (lane >> 4);
      double abuf[2][4];
#pragma unroll
      for (int i = 0; i < 4; ++i) abuf[0][i] = (double)arow[4 * i];
#pragma unroll
      for (int q = 0; q < KS / 4; ++q) {
        if (q + 1 < KS / 4) {
#pragma unroll
          for (int i = 0; i < 4; ++i) abuf[(q + 1) & 1][i] = (double)arow[4 * (4 * (q + 1) + i)];
        }
        if (16 * q < dqe) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(abuf[q & 1][i], Vreg[4 * q + i], acc, 0,
                                                       0, 0);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
        ured[wave * TROWS * KR + ((lane >> 4) + 4 * r) * KR + (lane & 15)] = acc[r];
      wait_lgkm0();
      raw_barrier();
      {
        double su = 0.0;
#pragma unroll
        for (int w = 0; w < kWavesPerBlock; ++w) su += ured[w * TROWS * KR + rr * KR + jj];
        ufin[rr * KR + jj] = (gr < rows && jj < ncols) ? c[t] - su : 0.0;
      }
      wait_lgkm0();
      raw_barrier();
      // G += tile^T U: the U operand is the same for every block b (read once);
      // the tile values of block b + 1 are read before the products of block b.
      // k slot g of product s is tile row s + 4 (g >> 1) + 8 (g & 1): the rows
      // that share an LDS pass (k slots 0, 1 and 2, 3) then sit 8 rows, i.e.
      // 32 banks, apart (the row pitch shifts by 4 banks), so no reads collide
      const int g4 = 4 * ((lane >> 5) & 1) + 8 * ((lane >> 4) & 1);
      double bvu[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) bvu[s] = ufin[(s + g4) * KR + (lane & 15)];
      const TM* gcol = tile + g4 * C::LDT + kbase + (lane & 15);
      double gbuf[2][4];
#pragma unroll
      for (int s = 0; s < 4; ++s) gbuf[0][s] = (double)gcol[s * C::LDT];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (b + 1 < NB) {
#pragma unroll
          for (int s = 0; s < 4; ++s)
            gbuf[(b + 1) & 1][s] = (double)gcol[s * C::LDT + 16 * (b + 1)];
        }
        if (16 * b < dqe) {
#pragma unroll
          for (int s = 0; s < 4; ++s)
            Gacc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(gbuf[b & 1][s], bvu[s], Gacc[b], 0, 0,
                                                           0);
        }
      }
      wait_lgkm0();
      raw_barrier();  // ured / ufin (and after the last tile, this buffer) free again
    }
  };
  if (rank < ngroups) {
    load_c(cv[0], rank);
    dma_group<TM, DP>(M, ld, rows, d, rank * C::ROWS, lbase);
  }
  for (int64_t g = rank; g < ngroups; g += 2 * T) {
    step(cv[0], cv[1], g, lbase, lbase + C::BUF);
    if (g + T >= ngroups) break;
    step(cv[1], cv[0], g + T, lbase + C::BUF, lbase);
  }
  __syncthreads();
}

// The whole A pass of one team member, out of line so that its registers
// (the X operand, the Gram-block accumulators and the tile in flight) do not
// compete with the solver state around it:
//   part_out = A_rows^T (C - A_rows X) over this member's tiles (d x 16, FP64).
template <typename TM, int DP, bool DMA>
__device__ __attribute__((noinline)) void a_pass(const TM* __restrict__ M, int64_t ld,
                                                 int64_t rows, int d, int rank, int T,
                                                 const double* __restrict__ B, int64_t ldb,
                                                 int64_t ldbc, int ncols,
                                                 const double* __restrict__ X, int64_t ldx,
                                                 double* __restrict__ part_out) {
  // dynamic LDS: the tile region, then the U reduction scratch
  extern __shared__ uint4 lds_raw[];
  double* ured = (double*)((char*)lds_raw + kUredOffset);
  double* ufin = ured + kWavesPerBlock * TROWS * KR;
  constexpr int DQ = DP / 4;
  constexpr int KS = DQ / 4;
  constexpr int NB = DQ / 16;
  double* stage = (double*)lds_raw;
  const int lane = lane_id(), kbase = wave_id() * wave_cols(d, DP);
  // X through the LDS stage (row-major d x 16 is the B-operand order)
  __syncthreads();
#pragma unroll 8
  for (int i = 0; i < DP * KR / kBlock; ++i) {
    const int idx = i * kBlock + (int)threadIdx.x;
    const int c = idx / KR, j = idx % KR;
    stage[idx] = (c < d && j < ncols) ? co_load(X + (int64_t)c * ldx + j) : 0.0;
  }
  __syncthreads();
  double Vreg[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) Vreg[s] = stage[(kbase + 4 * s) * KR + lane];
  f64x4 Gacc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) Gacc[b] = (f64x4){0.0, 0.0, 0.0, 0.0};
  if (DmaCfg<TM, DP>::ok && DMA)
    block_pass_dma<TM, DP>(M, ld, rows, d, rank, T, B, ldb, ldbc, ncols, Vreg, Gacc,
                           (lds_char*)lds_raw, ured, ufin);
  else
    block_pass<TM, DP, true>(M, ld, rows, d, rank, T, B, ldb, ldbc, ncols, Vreg, Gacc, lds_raw,
                             ured, ufin);
  store_block<DP>(Gacc, d, part_out);
}

// q = H p + lambda p on the owned columns [c_lo, c_hi) (16-aligned blocks), p
// (d x 16) in the LDS stage.  The waves split the
// k-range: lane (r, g) reads row cb + r of H over k = kbase + g KS + s (contiguous)
// with 16-byte loads, one block ahead of the matrix-core work.  Returns this
// thread's share of sum_c p_cj q_cj for its column j = tid % 16.
template <typename TH, int DP>
__device__ __forceinline__ double h_matvec(const TH* __restrict__ H, int64_t ldh, int c_lo,
                                                   int c_hi, const double* lam,
                                                   double* __restrict__ Q) {
  extern __shared__ uint4 lds_raw[];
  const double* stage = (const double*)lds_raw;
  double* ured = (double*)((char*)lds_raw + kUredOffset);
  constexpr int DQ = DP / 4;
  constexpr int KS = DQ / 4;
  constexpr int VE = 16 / (int)sizeof(TH);
  constexpr int NL = KS >= VE ? KS / VE : 1;
  constexpr int KSP = NL * VE;  // register slots per lane (>= KS)
  const int lane = lane_id(), wave = wave_id();
  const int kbase = wave * DQ;
  const int rr = threadIdx.x / KR, j = threadIdx.x % KR;
  const double lj = lam[j];
  const double* prow = stage + (kbase + (lane >> 4) * KS) * KR + (lane & 15);
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  auto load = [&](TH (&hv)[KSP], int cb) {
    const TH* hrow = H + (int64_t)(cb + (lane & 15)) * ldh + kbase + (lane >> 4) * KS;
    if (KS >= VE) {
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        union {
          u32x4 u;
          TH v[VE];
        } x;
        x.u = *(const u32x4 __attribute__((address_space(1)))*)(hrow + i * VE);
#pragma unroll
        for (int e = 0; e < VE; ++e) hv[i * VE + e] = x.v[e];
      }
    } else {
#pragma unroll
      for (int s = 0; s < KSP; ++s) hv[s] = s < KS ? hrow[s] : TH(0);
    }
  };
  double pq = 0.0;
  auto step = [&](TH (&hv)[KSP], int cb) {
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < KS; ++s)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)hv[s], prow[s * KR], acc, 0, 0, 0);
    if (cb + 32 < c_hi) load(hv, cb + 32);  // the block after next, into this buffer
#pragma unroll
    for (int r = 0; r < 4; ++r)
      ured[wave * TROWS * KR + ((lane >> 4) + 4 * r) * KR + (lane & 15)] = acc[r];
    __syncthreads();
    const int c = cb + rr;
    if (c < c_hi) {
      double qv = 0.0;
#pragma unroll
      for (int w = 0; w < kWavesPerBlock; ++w) qv += ured[w * TROWS * KR + rr * KR + j];
      const double pv = stage[c * KR + j];
      qv += lj * pv;
      ((double __attribute__((address_space(1)))*)Q)[(int64_t)c * KR + j] = qv;
      pq += pv * qv;
    }
    __syncthreads();
  };
  TH h0[KSP], h1[KSP];
  if (c_lo < c_hi) load(h0, c_lo);
  if (c_lo + 16 < c_hi) load(h1, c_lo + 16);
  for (int cb = c_lo; cb < c_hi; cb += 32) {
    step(h0, cb);
    if (cb + 16 >= c_hi) break;
    step(h1, cb + 16);
  }
  return pq;
}

// The lockstep CG of one outer iteration on a CG member (out of line, like
// a_pass: its registers are saved once per outer iteration, not per step).
// On entry R holds g (the member's columns), Z = 0, g_sh.rr / rr0 / active /
// bcg are set.  Returns the number of steps taken, or -1 if a barrier timed
// out; the caller advances its barrier epoch by two per step.
template <typename TH, int DP>
__device__ __attribute__((noinline)) int64_t cg_solve(const TH* __restrict__ H, int64_t ldh, int d,
                                                      int c_lo, int c_hi, double* Rp, double* Zp,
                                                      double* Qp, const double* scal,
                                                      double* myscal, int Tc, unsigned* bar_cg,
                                                      unsigned epoch, int* err, BarrierSpin spin,
                                                      double eps_sub, int64_t max_inner) {
  extern __shared__ uint4 lds_raw[];
  double* stage = (double*)lds_raw;
  // R and Z are exchanged with the other members (co_load / co_store); Q stays
  // with this member (its own rows), addressed as global memory
  typedef double __attribute__((address_space(1)))* gdbl;
  const gdbl Q = (gdbl)Qp;
  Shared& sh = g_sh;
  const int nown = c_hi - c_lo;
  int64_t k = 0;
  while (true) {
    int any = 0;
    for (int j = 0; j < KR; ++j) any |= sh.active[j];
    if (!any || k >= max_inner) break;
    // p = r (first step) or r + beta_cg p over all d, in place in the stage
    __syncthreads();
    {
      const int j = threadIdx.x % KR;  // fixed column per thread
      const bool act = sh.active[j] != 0;
      const double bc = sh.bcg[j];
#pragma unroll 8
      for (int i = 0; i < DP * KR / kBlock; ++i) {
        const int idx = i * kBlock + (int)threadIdx.x;
        const int c = idx / KR;
        double v = 0.0;
        if (c < d && act) v = (k == 0) ? co_load(Rp + idx) : co_load(Rp + idx) + bc * stage[idx];
        stage[idx] = v;
      }
    }
    __syncthreads();
    // q = H p + lambda p on the owned 16-column blocks
    const double pq_lane = h_matvec<TH, DP>(H, ldh, c_lo, c_hi, sh.lam, Qp);
    column_partials(pq_lane, myscal + KR, sh.red);
    if (!group_sync(bar_cg, Tc, epoch, err, &sh.flag, spin)) return -1;
    team_slot_sums(scal, Tc, KR, sh.ufin, sh.red);  // ufin[0..15] <- p_j^T q_j
    if (threadIdx.x < KR) {
      const int j = threadIdx.x;
      const double pq = sh.ufin[j];
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
    // owners: z += alpha p, r -= alpha q
    double rr_lane = 0.0;
    for (int idx = threadIdx.x; idx < nown * KR; idx += kBlock) {
      const int c = c_lo + idx / KR, j = idx % KR;
      const int64_t o = (int64_t)c * KR + j;
      double rv = co_load(Rp + o);
      if (sh.active[j]) {
        const double al = sh.acg[j];
        co_store(Zp + o, co_load(Zp + o) + al * stage[o]);
        rv -= al * Q[o];
        co_store(Rp + o, rv);
      }
      rr_lane += rv * rv;
    }
    column_partials(rr_lane, myscal + 0, sh.red);
    if (!group_sync(bar_cg, Tc, epoch, err, &sh.flag, spin)) return -1;
    team_slot_sums(scal, Tc, 0, sh.ufin, sh.red);  // ufin[0..15] <- new ||r_j||^2
    ++k;
    if (threadIdx.x < KR) {
      const int j = threadIdx.x;
      if (sh.active[j]) {
        const double rn = sh.ufin[j];
        sh.bcg[j] = rn / sh.rr[j];
        sh.rr[j] = rn;
        sh.kin[j] = k;
        if (rn <= eps_sub * eps_sub * sh.rr0[j]) sh.active[j] = 0;
      }
    }
    __syncthreads();
  }
  return k;
}


// The lockstep CG of an entry whose inner solve runs on one workgroup
// (sub-team of one): every vector stays in the workgroup.  Thread (wave w,
// lane l) owns rows 16 (4 b + w) + l / 16 + 4 i (i < 4, b < DP / 64) of
// column j = l % 16 -- the rows of the matrix-core result block it holds -- so
// r and z live in registers, p (the MFMA operand) and q in LDS, and the
// per-column sums go through two LDS buffers in a fixed order.  Each wave forms
// whole rows of H p for its own 16-row blocks (no reduction across waves) and
// skips the blocks and k-chunks at or beyond d, where H is zero.  H streams
// through a ring of register buffers: every load is unconditional (past the
// last chunk the ring already fetches the next step's first chunks; H does not
// change between steps), nothing else in the step touches global memory, and
// the barriers wait for LDS traffic only, so the waits before the products
// count exactly the chunks still in flight.  Same iteration as cg_solve (step
// lengths, masks, breakdown and stop rule per column); z ends in the entry's Z
// buffer.
template <typename TH, int DP>
__device__ __attribute__((noinline)) int64_t cg_solve_local(const TH* __restrict__ H, int64_t ldh,
                                                            int d, const double* __restrict__ R,
                                                            double* __restrict__ Z, double eps_sub,
                                                            int64_t max_inner) {
  extern __shared__ uint4 lds_raw[];
  double* stage = (double*)lds_raw;      // p, DP x 16
  double* ql = stage + DP * KR;          // q, DP x 16
  double* red0 = (double*)((char*)lds_raw + kUredOffset);
  double* red1 = red0 + kBlock;
  Shared& sh = g_sh;
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  typedef const u32x4 __attribute__((address_space(1)))* gvec;
  constexpr int NBW = DP / 64;                    // 16-row blocks per wave
  constexpr int NV = 4 * NBW;                     // owned entries per vector
  constexpr int VE = 16 / (int)sizeof(TH);        // elements per 16-byte load
  constexpr int KQ = DP / 4;
  constexpr int NLD = (KQ * (int)sizeof(TH) / 16) < 4 ? KQ * (int)sizeof(TH) / 16 : 4;
  constexpr int CE = NLD * VE;                    // k elements per lane and chunk
  constexpr int NRING = 4;                        // chunks in flight per lane
  const int lane = lane_id(), wave = wave_id();
  const int j = lane & 15, g = lane >> 4;
  const int tid = (int)threadIdx.x;
  // active blocks of this wave and k-chunks (chunk c covers k in [c 4 CE, (c+1) 4 CE))
  const int nbw = d > 16 * wave ? min(NBW, (d - 16 * wave + 63) / 64) : 0;
  const int nch = min(KQ / CE, (d + 4 * CE - 1) / (4 * CE));
  const int T = nbw * nch;  // chunks of one product, in order t = b nch + c
  // each step walks Tp positions (T rounded up to whole rings; the extra ones
  // are dummy reads), so ring slot u always holds a position congruent to u
  const int Tp = T > 0 ? (T + NRING - 1) / NRING * NRING : 0;
  // element i of a 16 x 16 x 4 FP64 MFMA result is row l / 16 + 4 i, column l % 16
  auto row_of = [&](int v) { return 16 * (4 * (v >> 2) + wave) + g + 4 * (v & 3); };
  union Chunk {
    u32x4 u[NLD];
    TH v[CE];
  };
  // the fetch cursor walks the positions of every step in turn; dummy
  // positions (and a wave with no active block) read row j (valid, cached)
  int pos = 0, fb = 0, fc = 0;
  auto fetch = [&](Chunk& dst) {
    const bool in = pos < T;
    const int row = in ? 16 * (4 * fb + wave) + j : j;
    const gvec src = (gvec)(H + (int64_t)row * ldh + (in ? fc : 0) * 4 * CE + g * CE);
#pragma unroll
    for (int i = 0; i < NLD; ++i) dst.u[i] = src[i];
    if (++pos >= Tp) {
      pos = 0;
      fb = 0;
      fc = 0;
    } else if (++fc == nch) {
      fc = 0;
      ++fb;
    }
  };
  Chunk ring[NRING];
#pragma unroll
  for (int u = 0; u < NRING; ++u) fetch(ring[u]);

  double r[NV], z[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int row = row_of(v);
    r[v] = row < d ? co_load(R + row * KR + j) : 0.0;
    z[v] = 0.0;
  }
  const double lj = sh.lam[j];
  bool act = sh.active[j] != 0;
  double rr = sh.rr[j], bc = 0.0;
  const double rr0 = sh.rr0[j];
  int64_t k = 0, kin = 0;

  while (true) {
    int any = 0;
    for (int jj = 0; jj < KR; ++jj) any |= sh.active[jj];
    if (!any || k >= max_inner) break;
    // p = r (first step) or r + beta_cg p; inactive columns carry p = 0
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int o = row_of(v) * KR + j;
      stage[o] = act ? ((k == 0) ? r[v] : r[v] + bc * stage[o]) : 0.0;
    }
    wait_lgkm0();
    raw_barrier();
    // q = H p + lambda p on the owned blocks (into LDS), p . q per column
    double pq = 0.0;
    {
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
      int b = 0, c = 0;
      for (int t0 = 0; t0 < Tp; t0 += NRING) {
#pragma unroll
        for (int u = 0; u < NRING; ++u) {
          if (t0 + u < T) {
            const double* pk = stage + (c * 4 * CE + g * CE) * KR + j;
#pragma unroll
            for (int e = 0; e < CE; ++e)
              acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)ring[u].v[e], pk[e * KR], acc,
                                                         0, 0, 0);
            if (++c == nch) {
              const int row0 = 16 * (4 * b + wave) + g;
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int o = (row0 + 4 * i) * KR + j;
                const double pv = stage[o];
                const double qv = acc[i] + lj * pv;
                ql[o] = qv;
                pq += pv * qv;
              }
              acc = (f64x4){0.0, 0.0, 0.0, 0.0};
              c = 0;
              ++b;
            }
          }
          // the slot's next position (this step's or the next step's)
          fetch(ring[u]);
        }
      }
    }
    red0[tid] = pq;
    wait_lgkm0();
    raw_barrier();
    double spq = 0.0;
#pragma unroll
    for (int t = 0; t < 16; ++t) spq += red0[t * 16 + j];
    double al = 0.0;
    if (act) {
      al = rr / spq;
      if (!(spq > 0.0) || !isfinite(al)) {
        al = 0.0;
        act = false;  // breakdown in this column: keep the current step
      }
    }
    double rrp = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      // rows of blocks this wave skipped (at or beyond d) keep r = 0
      if (act && (v >> 2) < nbw) {
        const int o = row_of(v) * KR + j;
        z[v] += al * stage[o];
        r[v] -= al * ql[o];
      }
      rrp += r[v] * r[v];
    }
    red1[tid] = rrp;
    wait_lgkm0();
    raw_barrier();
    double rn = 0.0;
#pragma unroll
    for (int t = 0; t < 16; ++t) rn += red1[t * 16 + j];
    ++k;
    if (act) {
      bc = rn / rr;
      rr = rn;
      kin = k;
      if (rn <= eps_sub * eps_sub * rr0) act = false;
    }
    if (tid < KR) sh.active[tid] = act ? 1 : 0;
    wait_lgkm0();
    raw_barrier();
  }
  if (tid < KR) sh.kin[tid] = kin;
  // z to the entry's buffer (read by the update with another thread mapping);
  // the ring's look-ahead loads are waited for before the registers go
#pragma unroll
  for (int v = 0; v < NV; ++v) co_store(Z + row_of(v) * KR + j, z[v]);
  __builtin_amdgcn_s_waitcnt(0);
  __threadfence_block();
  __syncthreads();
  return k;
}

// The one-workgroup CG above spread over a sub-team of Tc workgroups (rank
// 0 .. Tc - 1 of the problem's team).  The 16-row blocks are grouped in fours
// (a quad: one block per wave, as above), and member `rank` owns quads
// rank, rank + Tc, ...: each of its waves forms whole rows of H p for its own
// blocks from the same register ring, and keeps r and z of its rows in
// registers.  Per step, two sub-team barriers: one after each member has
// stored its per-column sums p . q (scalar slots), one after it has stored its
// rows of the new r and its per-column sums r . r; every member then reads the
// whole r back and forms the whole p = r + beta p in LDS for the next
// products.  Every member sums the slots in member order, so all of them take
// the same step lengths, masks and stop decision.  A last barrier publishes
// the members' rows of z to the row owners of the heavy-ball update.  With two
// or more members a member owns at most half the quads, so its r and z take
// half the registers of the one-workgroup form.  Returns the number of steps
// (the caller advances its barrier epoch by 2 k + 1), or -1 if a barrier timed
// out.
template <typename TH, int DP>
__device__ __attribute__((noinline)) int64_t cg_solve_team(
    const TH* __restrict__ H, int64_t ldh, int d, int rank, int Tc, double* R, double* Z,
    const double* scal, double* myscal, unsigned* bar_cg, unsigned epoch, int* err,
    BarrierSpin spin, double eps_sub, int64_t max_inner) {
  extern __shared__ uint4 lds_raw[];
  double* stage = (double*)lds_raw;      // p, DP x 16 (all rows)
  double* ql = stage + DP * KR;          // q, DP x 16 (this member's rows)
  double* red0 = (double*)((char*)lds_raw + kUredOffset);
  double* red1 = red0 + kBlock;
  Shared& sh = g_sh;
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  typedef const u32x4 __attribute__((address_space(1)))* gvec;
  constexpr int NBW = DP / 128 > 0 ? DP / 128 : 1;  // quads per member (Tc >= 2)
  constexpr int NV = 4 * NBW;
  constexpr int VE = 16 / (int)sizeof(TH);
  constexpr int KQ = DP / 4;
  constexpr int NLD = (KQ * (int)sizeof(TH) / 16) < 4 ? KQ * (int)sizeof(TH) / 16 : 4;
  constexpr int CE = NLD * VE;
  constexpr int NRING = 4;
  const int lane = lane_id(), wave = wave_id();
  const int j = lane & 15, g = lane >> 4;
  const int tid = (int)threadIdx.x;
  // this wave's blocks: 4 (rank + Tc b) + wave for b < nbw (those starting below d)
  auto block_row0 = [&](int b) { return 16 * (4 * (rank + Tc * b) + wave); };
  int nbw = 0;
  while (nbw < NBW && block_row0(nbw) < d) ++nbw;
  const int nch = min(KQ / CE, (d + 4 * CE - 1) / (4 * CE));
  const int T = nbw * nch;
  const int Tp = T > 0 ? (T + NRING - 1) / NRING * NRING : 0;
  auto row_of = [&](int v) { return block_row0(v >> 2) + g + 4 * (v & 3); };
  union Chunk {
    u32x4 u[NLD];
    TH v[CE];
  };
  int pos = 0, fb = 0, fc = 0;
  auto fetch = [&](Chunk& dst) {
    const bool in = pos < T;
    const int row = in ? block_row0(fb) + j : j;
    const gvec src = (gvec)(H + (int64_t)row * ldh + (in ? fc : 0) * 4 * CE + g * CE);
#pragma unroll
    for (int i = 0; i < NLD; ++i) dst.u[i] = src[i];
    if (++pos >= Tp) {
      pos = 0;
      fb = 0;
      fc = 0;
    } else if (++fc == nch) {
      fc = 0;
      ++fb;
    }
  };
  Chunk ring[NRING];
#pragma unroll
  for (int u = 0; u < NRING; ++u) fetch(ring[u]);

  double r[NV], z[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int row = row_of(v);
    r[v] = ((v >> 2) < nbw && row < d) ? co_load(R + row * KR + j) : 0.0;
    z[v] = 0.0;
  }
  const double lj = sh.lam[j];
  bool act = sh.active[j] != 0;
  double rr = sh.rr[j], bc = 0.0;
  const double rr0 = sh.rr0[j];
  int64_t k = 0, kin = 0;

  while (true) {
    int any = 0;
    for (int jj = 0; jj < KR; ++jj) any |= sh.active[jj];
    if (!any || k >= max_inner) break;
    // p = r (first step) or r + beta_cg p over all rows, r as published by
    // the members; inactive columns carry p = 0
    for (int idx = tid; idx < DP * KR; idx += kBlock) {
      const int c = idx / KR;  // column idx % KR == j for this thread
      double v = 0.0;
      if (c < d && act) v = (k == 0) ? co_load(R + idx) : co_load(R + idx) + bc * stage[idx];
      stage[idx] = v;
    }
    __syncthreads();
    // q = H p + lambda p on this member's blocks, p . q per column
    double pq = 0.0;
    {
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
      int b = 0, c = 0;
      for (int t0 = 0; t0 < Tp; t0 += NRING) {
#pragma unroll
        for (int u = 0; u < NRING; ++u) {
          if (t0 + u < T) {
            const double* pk = stage + (c * 4 * CE + g * CE) * KR + j;
#pragma unroll
            for (int e = 0; e < CE; ++e)
              acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)ring[u].v[e], pk[e * KR], acc,
                                                         0, 0, 0);
            if (++c == nch) {
              const int row0 = block_row0(b) + g;
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int o = (row0 + 4 * i) * KR + j;
                const double pv = stage[o];
                const double qv = acc[i] + lj * pv;
                ql[o] = qv;
                pq += pv * qv;
              }
              acc = (f64x4){0.0, 0.0, 0.0, 0.0};
              c = 0;
              ++b;
            }
          }
          fetch(ring[u]);
        }
      }
    }
    red0[tid] = pq;
    __syncthreads();
    if (tid < KR) {
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < 16; ++t) s += red0[t * 16 + tid];
      co_store(myscal + KR + tid, s);
    }
    if (!group_sync(bar_cg, Tc, epoch, err, &sh.flag, spin)) return -1;
    double spq = 0.0;
    for (int m = 0; m < Tc; ++m) spq += co_load(scal + (int64_t)m * kNScal + KR + j);
    double al = 0.0;
    if (act) {
      al = rr / spq;
      if (!(spq > 0.0) || !isfinite(al)) {
        al = 0.0;
        act = false;  // breakdown in this column: keep the current step
      }
    }
    double rrp = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if ((v >> 2) < nbw) {
        const int row = row_of(v);
        const int o = row * KR + j;
        if (act) {
          z[v] += al * stage[o];
          r[v] -= al * ql[o];
        }
        if (row < d) co_store(R + o, r[v]);
      }
      rrp += r[v] * r[v];
    }
    red1[tid] = rrp;
    __syncthreads();
    if (tid < KR) {
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < 16; ++t) s += red1[t * 16 + tid];
      co_store(myscal + tid, s);
    }
    if (!group_sync(bar_cg, Tc, epoch, err, &sh.flag, spin)) return -1;
    double rn = 0.0;
    for (int m = 0; m < Tc; ++m) rn += co_load(scal + (int64_t)m * kNScal + j);
    ++k;
    if (act) {
      bc = rn / rr;
      rr = rn;
      kin = k;
      if (rn <= eps_sub * eps_sub * rr0) act = false;
    }
    if (tid < KR) sh.active[tid] = act ? 1 : 0;
    __syncthreads();
  }
  if (tid < KR) sh.kin[tid] = kin;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int row = row_of(v);
    if ((v >> 2) < nbw && row < d) co_store(Z + row * KR + j, z[v]);
  }
  __builtin_amdgcn_s_waitcnt(0);  // the ring's look-ahead loads too
  if (!group_sync(bar_cg, Tc, epoch, err, &sh.flag, spin)) return -1;
  return k;
}

// Lane l's value of v in every lane (l a compile-time constant after
// unrolling: two v_readlane into scalar registers, no LDS round trip).
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Partial dot product of one factor row with the solved vector over the
// 16-column blocks [m0, m1): this lane's k slot g covers k = 16 m + 4 g + 0..3.
// Four blocks per step with separate sums keep eight 16-byte loads in flight.
__device__ __forceinline__ double row_dot(const double* __restrict__ Fr,
                                          const double* __restrict__ y, int m0, int m1, int g) {
  typedef double dbl2 __attribute__((ext_vector_type(2)));
  typedef const dbl2 __attribute__((address_space(1)))* gd2;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  int m = m0;
  for (; m + 4 <= m1; m += 4) {
    dbl2 f[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k0 = 16 * (m + u) + 4 * g;
      f[u][0] = ((gd2)(Fr + k0))[0];
      f[u][1] = ((gd2)(Fr + k0))[1];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k0 = 16 * (m + u) + 4 * g;
      s[u] += f[u][0].x * y[k0] + f[u][0].y * y[k0 + 1] + f[u][1].x * y[k0 + 2] +
              f[u][1].y * y[k0 + 3];
    }
  }
  for (; m < m1; ++m) {
    const int k0 = 16 * m + 4 * g;
    const dbl2 f0 = ((gd2)(Fr + k0))[0], f1 = ((gd2)(Fr + k0))[1];
    s[0] += f0.x * y[k0] + f0.y * y[k0 + 1] + f1.x * y[k0 + 2] + f1.y * y[k0 + 3];
  }
  return (s[0] + s[1]) + (s[2] + s[3]);
}
// Sum over the four k slots (lanes r, r + 16, r + 32, r + 48).
__device__ __forceinline__ double slot_sum(double s) {
  s += __shfl_xor(s, 16);
  return s + __shfl_xor(s, 32);
}

// Exact sub-solve of one outer step (Exact M-IHS: Table 2, Section 4.2): for every active
// column j, z_j = (L_j L_j^T)^{-1} r_j with the column's Cholesky factor F_j
// (L_j in the lower triangle, L_j^T mirrored into the upper one, zero at
// indices >= d).  Member `rank` of a sub-team of `tc` workgroups takes columns
// rank, rank + tc, ..., handed to its waves in turn; the column's vector lives
// in the wave's slice of LDS.  z goes to Zt column-major (column j at Zt + j ld,
// ld the entry's padded width), so that no cache line holds results of two
// workgroups.  Both substitutions run by 16-row blocks, each
// block first taking the dot products of its rows with the already solved part
// (lane = row + 16 k-slot, four consecutive k per lane and 16-column step,
// summed over the four slots), then solving its 16 x 16 diagonal block in
// registers, one lane broadcast per column.
template <int DP>
__device__ __attribute__((noinline)) void tri_solve_local(const double* __restrict__ Fb,
                                                          int64_t ld, int d,
                                                          const double* __restrict__ R,
                                                          double* __restrict__ Zt, int rank,
                                                          int tc) {
  extern __shared__ uint4 lds_raw[];
  Shared& sh = g_sh;
  const int lane = lane_id(), wave = wave_id();
  const int r = lane & 15, g = lane >> 4;
  double* y = (double*)lds_raw + wave * DP;
  const int nb = (d + 15) / 16;
  for (int q = wave; rank + q * tc < KR; q += kWavesPerBlock) {
    const int j = rank + q * tc;
    if (!sh.active[j]) continue;
    const double* F = Fb + (int64_t)j * ld * ld;
    for (int k = lane; k < DP; k += kWave) y[k] = k < d ? co_load(R + (int64_t)k * KR + j) : 0.0;
    // forward substitution L u = r (u overwrites y block by block)
    for (int I = 0; I < nb; ++I) {
      const int row = 16 * I + r;
      const double* Fr = F + (int64_t)(row < d ? row : 0) * ld;
      const double s = slot_sum(row < d ? row_dot(Fr, y, 0, I, g) : 0.0);
      double dr[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) dr[c] = 16 * I + c < d ? Fr[16 * I + c] : 1.0;
      double x = row < d ? y[row] - s : 0.0;
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (16 * I + c < d) {
          if (r == c) x /= dr[c];
          const double xc = lane_value(x, c);
          if (r > c) x -= dr[c] * xc;
        }
      if (g == 0 && row < d) y[row] = x;
    }
    // backward substitution L^T z = u, reading the rows of L^T
    for (int I = nb - 1; I >= 0; --I) {
      const int row = 16 * I + r;
      const double* Fr = F + (int64_t)(row < d ? row : 0) * ld;
      const double s = slot_sum(row < d ? row_dot(Fr, y, I + 1, nb, g) : 0.0);
      double dr[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) dr[c] = 16 * I + c < d ? Fr[16 * I + c] : 1.0;
      double x = row < d ? y[row] - s : 0.0;
#pragma unroll
      for (int c = 15; c >= 0; --c)
        if (16 * I + c < d) {
          if (r == c) x /= dr[c];
          const double xc = lane_value(x, c);
          if (r < c) x -= dr[c] * xc;
        }
      if (g == 0 && row < d) y[row] = x;
    }
    for (int k = lane; k < d; k += kWave) co_store(Zt + (int64_t)j * ld + k, y[k]);
  }
  if (threadIdx.x < KR) sh.kin[threadIdx.x] = sh.active[threadIdx.x] ? 1 : 0;
  __threadfence_block();
  __syncthreads();
}

template <int DP>
__device__ void run_entry(const BatchArgs& a, const BatchEntry& e, int rank, void* tile,
                          Shared& sh) {
  constexpr int DQ = DP / 4;
  constexpr int KS = DQ / 4;
  constexpr int NB = DQ / 16;
  const int T = e.tsize, Tc = e.tcg;
  const int d = e.d;
  const int lane = lane_id(), wave = wave_id();
  const int kbase = wave * DQ;
  const EntryLayout L = entry_layout(DP, T);
  double* W = e.work;
  double* part = W + L.part;
  double* R = W + L.R;
  double* Z = W + L.Z;
  double* Q = W + L.Q;
  double* XP = W + L.XP;
  double* scal = W + L.scal;
  double* myscal = scal + (int64_t)rank * kNScal;
  double* stage = (double*)tile;  // d x 16 vectors (row-major = MFMA B-operand order)
  const bool cg = rank < Tc;
  // a one-workgroup CG keeps p and q in LDS (2 x DP x 16 doubles within the
  // tile region)
  const bool local_cg = Tc == 1 && 2 * (size_t)DP * KR * sizeof(double) <= kUredOffset;
  // a larger sub-team runs the same form, each member on its share of the rows
  const bool team_cg = Tc > 1 && 2 * (size_t)DP * KR * sizeof(double) <= kUredOffset;
  // CG members own 16-aligned column ranges of R, Z, Q, XP and X
  const int cpw = ((d + Tc - 1) / Tc + 15) / 16 * 16;
  const int c_lo = cg ? min(d, rank * cpw) : d;
  const int c_hi = cg ? min(d, c_lo + cpw) : d;
  const int nown = c_hi - c_lo;
  unsigned ep_all = 0, ep_cg = 0;
  int* s_flag = &sh.flag;
  bool alive = true;
  const long long t_start = wall_clock64();

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
    XP[(int64_t)c * KR + j] = (j < e.ncols) ? co_load(e.X + (int64_t)c * e.ldx + j) : 0.0;
  }
  __syncthreads();

  int64_t outer = 0;
  for (; outer < a.max_outer; ++outer) {
    // ---- A pass: G partial = A^T (C - A X) over this member's tiles
    // (the direct-to-LDS and register-staged passes are separate functions,
    // each with its own register allocation)
    double* my_part = part + (int64_t)rank * DP * KR;
    if (a.a_f32) {
      if (a.a_dma)
        a_pass<float, DP, true>((const float*)e.A, e.lda, e.n, d, rank, T, e.B, e.ldb, e.ldbc,
                                e.ncols, e.X, e.ldx, my_part);
      else
        a_pass<float, DP, false>((const float*)e.A, e.lda, e.n, d, rank, T, e.B, e.ldb, e.ldbc,
                                 e.ncols, e.X, e.ldx, my_part);
    } else {
      if (a.a_dma)
        a_pass<double, DP, true>((const double*)e.A, e.lda, e.n, d, rank, T, e.B, e.ldb,
                                 e.ldbc, e.ncols, e.X, e.ldx, my_part);
      else
        a_pass<double, DP, false>((const double*)e.A, e.lda, e.n, d, rank, T, e.B, e.ldb,
                                  e.ldbc, e.ncols, e.X, e.ldx, my_part);
    }
    if (!(alive = group_sync(e.bar, T, ep_all, a.err, s_flag, a.spin))) break;

    // ---- every member reduces the partials of a slice of columns:
    // g = sum of partials + rhs - lambda x; CG start r = g, z = 0
    {
      const int cpa = (d + T - 1) / T;
      const int a_lo = min(d, rank * cpa), a_hi = min(d, a_lo + cpa);
      double rr_lane = 0.0;
      for (int idx = threadIdx.x; idx < (a_hi - a_lo) * KR; idx += kBlock) {
        const int c = a_lo + idx / KR, j = idx % KR;
        double g = 0.0;
#pragma unroll 8
        for (int t = 0; t < T; ++t) g += co_load(part + ((int64_t)t * DP + c) * KR + j);
        if (j < e.ncols) {
          if (e.RHS) g += e.RHS[(int64_t)c * e.ldr + j];
          g -= sh.lam[j] * co_load(e.X + (int64_t)c * e.ldx + j);
        }
        if (sh.done[j]) g = 0.0;
        const int64_t o = (int64_t)c * KR + j;
        co_store(R + o, g);
        co_store(Z + o, 0.0);
        rr_lane += g * g;
      }
      column_partials(rr_lane, myscal + 0, sh.red);
    }
    if (!(alive = group_sync(e.bar, T, ep_all, a.err, s_flag, a.spin))) break;

    if (cg) {
      team_slot_sums(scal, T, 0, sh.rr0, sh.red);
      if (threadIdx.x < KR) {
        const int j = threadIdx.x;
        sh.rr[j] = sh.rr0[j];
        sh.gnorm[j] = sh.done[j] ? sh.gnorm[j] : sqrt(sh.rr0[j]);
        sh.active[j] = (!sh.done[j] && sh.rr0[j] > 0.0) ? 1 : 0;
        sh.bcg[j] = 0.0;
        sh.kin[j] = 0;
      }
      __syncthreads();

      // ---- lockstep CG on (H + lambda_j I): in the workgroup when the CG
      // sub-team is one workgroup, else on the team
      int64_t k;
      const bool exact = a.exact && e.fac && !*(volatile int*)e.fac_bad;
      if (exact) {
        // the columns split over the sub-team, z column-major in Q (unused by
        // the exact path); the barrier publishes it to the row owners
        tri_solve_local<DP>(e.fac, e.dp, d, R, Q, rank, Tc);
        k = group_sync(e.bar_cg, Tc, ep_cg, a.err, s_flag, a.spin) ? 1 : -1;
      } else if (local_cg)
        k = a.h_f32 ? cg_solve_local<float, DP>((const float*)e.H, e.ldh, d, R, Z, a.eps_sub,
                                                a.max_inner)
                    : cg_solve_local<double, DP>((const double*)e.H, e.ldh, d, R, Z, a.eps_sub,
                                                 a.max_inner);
      else if (team_cg)
        k = a.h_f32 ? cg_solve_team<float, DP>((const float*)e.H, e.ldh, d, rank, Tc, R, Z, scal,
                                               myscal, e.bar_cg, ep_cg, a.err, a.spin, a.eps_sub,
                                               a.max_inner)
                    : cg_solve_team<double, DP>((const double*)e.H, e.ldh, d, rank, Tc, R, Z,
                                                scal, myscal, e.bar_cg, ep_cg, a.err, a.spin,
                                                a.eps_sub, a.max_inner);
      else
        k = a.h_f32 ? cg_solve<float, DP>((const float*)e.H, e.ldh, d, c_lo, c_hi, R, Z, Q, scal,
                                          myscal, Tc, e.bar_cg, ep_cg, a.err, a.spin, a.eps_sub,
                                          a.max_inner)
                    : cg_solve<double, DP>((const double*)e.H, e.ldh, d, c_lo, c_hi, R, Z, Q,
                                           scal, myscal, Tc, e.bar_cg, ep_cg, a.err, a.spin,
                                           a.eps_sub, a.max_inner);
      alive = k >= 0;
      if (alive && Tc > 1 && !exact) ep_cg += 2u * (unsigned)k + (team_cg ? 1u : 0u);
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
        const double xc = co_load(xp);
        const double zv =
            !exact ? co_load(Z + o) : (sh.active[j] ? co_load(Q + (int64_t)j * e.dp + c) : 0.0);
        const double xn = xc + sh.alpha[j] * zv + sh.beta[j] * (xc - XP[o]);
        XP[o] = xc;
        co_store(xp, xn);
        s0 += (xn - xc) * (xn - xc);
        s1 += xn * xn;
      }
      column_partials(s0, myscal + 2 * KR, sh.red);
      column_partials(s1, myscal + 3 * KR, sh.red);
    }
    // members outside the CG sub-team wait here through the whole inner solve
    if (!(alive = group_sync(e.bar, T, ep_all, a.err, s_flag, cg ? a.spin : a.spin_idle))) break;
    team_slot_sums(scal, Tc, 2 * KR, sh.ufin, sh.red);
    team_slot_sums(scal, Tc, 3 * KR, sh.acg, sh.red);
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
    int all_done = 1;
    for (int j = 0; j < KR; ++j) all_done &= sh.done[j];
    if (all_done) {
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
    const long long ticks = wall_clock64() - t_start;
    const long long us = a.wall_khz > 0 ? ticks * 1000 / a.wall_khz : 0;
    inf->elapsed_us = (int32_t)(us < 0x7fffffffLL ? us : 0x7fffffffLL);
  }
  __syncthreads();
}

template <int DPMAX>
__global__ __launch_bounds__(kBlock) void batched_kernel(BatchArgs a) {
  extern __shared__ uint4 lds_raw[];
  Shared& sh = g_sh;
  void* lds = (void*)lds_raw;
  const int* items = a.wg_items + (int64_t)blockIdx.x * a.items_stride;
  for (int i = 0; i < a.items_stride; ++i) {
    const int ei = items[i];
    if (ei < 0) break;
    const BatchEntry e = a.entries[ei];
    const int rank = (int)blockIdx.x - e.team0;
    // each entry runs at its own padded width (<= DPMAX)
    if (e.dp <= 64) run_entry<64>(a, e, rank, lds, sh);
    else if (DPMAX >= 128 && e.dp <= 128) run_entry<(DPMAX >= 128 ? 128 : 64)>(a, e, rank, lds, sh);
    else if (DPMAX >= 256 && e.dp <= 256) run_entry<(DPMAX >= 256 ? 256 : 64)>(a, e, rank, lds, sh);
    else if (DPMAX >= 512 && e.dp <= 512) run_entry<(DPMAX >= 512 ? 512 : 64)>(a, e, rank, lds, sh);
    else if (DPMAX >= 1024) run_entry<(DPMAX >= 1024 ? 1024 : 64)>(a, e, rank, lds, sh);
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


}  // namespace

int block_max_d() { return 1024; }

namespace {

// Distinct sketches (by group id) in order of first appearance.
std::vector<int64_t> group_leaders(const BlockEntryDesc* ents, int64_t count) {
  std::vector<int64_t> lead;
  for (int64_t i = 0; i < count; ++i) {
    bool seen = false;
    for (int64_t l : lead)
      if (ents[l].sa_group == ents[i].sa_group) {
        seen = true;
        break;
      }
    if (!seen) lead.push_back(i);
  }
  return lead;
}

struct BlockLayout {
  size_t ent_off, item_off, gram_off, bar_off, total;
  std::vector<size_t> work_off, h_off, fac_off;  // fac_off empty without exact sub-solves
  std::vector<int> ngram;  // gram jobs per group
  size_t njobs;
};

BlockLayout block_layout(const BlockEntryDesc* ents, int64_t count, const Schedule& S, int G,
                         bool exact) {
  BlockLayout L;
  size_t off = 0;
  L.ent_off = off;
  off = align_up(off + (size_t)count * sizeof(BatchEntry), 256);
  L.item_off = off;
  off = align_up(off + (size_t)G * S.stride * sizeof(int), 256);
  const std::vector<int64_t> lead = group_leaders(ents, count);
  L.njobs = 0;
  for (int64_t l : lead) {
    const int nb = dp_for(ents[l].d) / 64;
    L.ngram.push_back(nb * (nb + 1) / 2);
    L.njobs += (size_t)nb * (nb + 1) / 2;
  }
  L.gram_off = off;
  off = align_up(off + L.njobs * sizeof(GramJob), 256);
  L.work_off.resize(count);
  for (int64_t i = 0; i < count; ++i) {
    L.work_off[i] = off;
    off = align_up(off + entry_layout(dp_for(ents[i].d), S.tsize[i]).total * sizeof(double), 256);
  }
  for (int64_t l : lead) {
    const size_t dp = (size_t)dp_for(ents[l].d);
    L.h_off.push_back(off);
    off = align_up(off + dp * dp * sizeof(double), 256);
  }
  if (exact)
    for (int64_t i = 0; i < count; ++i) {
      const size_t dp = (size_t)dp_for(ents[i].d);
      L.fac_off.push_back(off);
      off = align_up(off + (size_t)ents[i].ncols * dp * dp * sizeof(double), 256);
    }
  // barrier words (two lines per entry, plus the error flag), then one
  // factorization flag per entry: all cleared by every launch
  L.bar_off = off;
  off = align_up(off + (size_t)(2 * count + 2) * 128 + (size_t)count * sizeof(int), 256);
  L.total = off;
  return L;
}

// One FP64 Cholesky factor per (entry, column) for the exact sub-solves:
// L L^T = H + lambda_j I, L in the lower triangle of F (dp x dp), L^T mirrored
// into the upper triangle, zero at indices >= d.  Right-looking by 16-column
// panels: the diagonal block is factored in registers of one wave (one
// lane broadcast per column pair), the rows below it are solved against it
// one row per thread and staged in LDS, and the trailing lower triangle is
// updated in global memory from the staged panel.  Each finished panel is
// also written transposed into the upper triangle.  A non-positive or non-finite pivot
// sets the entry's fac_bad word (the solve then uses the inner CG) and the
// factorization goes on with pivot 1 so that every value stays finite.
constexpr int kPanel = 16;
constexpr int kPanelLd = kPanel + 1;  // LDS row pitch (odd: no bank conflicts)
__host__ __device__ constexpr size_t chol_lds_bytes(int dp) {
  return ((size_t)dp + kPanel) * kPanelLd * sizeof(double);
}
template <typename TH>
__global__ __launch_bounds__(kBlock) void chol_kernel(const BatchEntry* __restrict__ ents) {
  extern __shared__ uint4 lds_raw[];
  const BatchEntry& e = ents[blockIdx.x / KR];
  const int col = (int)(blockIdx.x % KR);
  if (col >= e.ncols || !e.fac) return;
  const int d = e.d, dp = e.dp;
  const int64_t ld = dp;
  double* __restrict__ F = e.fac + (int64_t)col * ld * ld;
  const TH* __restrict__ H = (const TH*)e.H;
  const double lam = e.lam[col];
  const int tid = (int)threadIdx.x, lane = lane_id(), wave = wave_id();
  double* D = (double*)lds_raw;        // diagonal block, kPanel x kPanelLd
  double* P = D + kPanel * kPanelLd;   // panel rows below it, dp x kPanelLd
  // lower triangle of H + lambda I, zero elsewhere (the upper triangle is
  // written with L^T as the panels are produced); a wave per row, eight
  // independent copies per lane in flight
  for (int i = wave; i < dp; i += kWavesPerBlock) {
    const TH* Hi = H + (int64_t)i * e.ldh;
    double* Fi = F + (int64_t)i * ld;
    for (int k0 = 0; k0 < dp; k0 += 8 * kWave) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = k0 + u * kWave + lane;
        v[u] = (i < d && k <= i) ? (double)Hi[k] + (i == k ? lam : 0.0) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = k0 + u * kWave + lane;
        if (k < dp) Fi[k] = v[u];
      }
    }
  }
  __syncthreads();
  bool bad = false;
  for (int J = 0; J < d; J += kPanel) {
    const int w = min(kPanel, d - J);
    if (wave == 0) {
      // lanes r < 16 hold row J + r of the diagonal block (lanes >= 16 repeat them)
      const int r = lane & 15;
      double a[kPanel];
#pragma unroll
      for (int c = 0; c < kPanel; ++c)
        a[c] = (r < w && c <= r) ? F[(int64_t)(J + r) * ld + J + c] : 0.0;
#pragma unroll
      for (int c = 0; c < kPanel; ++c)
        if (c < w) {
          double piv = lane_value(a[c], c);
          if (!(piv > 0.0) || !isfinite(piv)) {
            bad = true;
            piv = 1.0;
          }
          const double sq = sqrt(piv);
          if (r == c) a[c] = sq;
          else if (r > c) a[c] /= sq;
#pragma unroll
          for (int cc = c + 1; cc < kPanel; ++cc) {
            const double lcc = lane_value(a[c], cc);
            if (r >= cc) a[cc] -= a[c] * lcc;
          }
        }
      if (lane < kPanel) {
#pragma unroll
        for (int c = 0; c < kPanel; ++c) {
          D[r * kPanelLd + c] = (r < w && c <= r) ? a[c] : 0.0;
          if (r < w && c <= r) {
            F[(int64_t)(J + r) * ld + J + c] = a[c];
            F[(int64_t)(J + c) * ld + J + r] = a[c];  // L^T
          }
        }
      }
    }
    __syncthreads();
    // panel: row i below the block solves x D^T = F[i][J .. J + w)
    const int i0 = J + w, nt = d - i0;
    for (int i = i0 + tid; i < d; i += kBlock) {
      double x[kPanel];
#pragma unroll
      for (int c = 0; c < kPanel; ++c) {
        if (c < w) {
          double v = F[(int64_t)i * ld + J + c];
#pragma unroll
          for (int t = 0; t < c; ++t) v -= x[t] * D[c * kPanelLd + t];
          x[c] = v / D[c * kPanelLd + c];
        } else {
          x[c] = 0.0;
        }
      }
#pragma unroll
      for (int c = 0; c < kPanel; ++c) {
        if (c < w) {
          F[(int64_t)i * ld + J + c] = x[c];
          F[(int64_t)(J + c) * ld + i] = x[c];  // L^T (consecutive i: coalesced)
        }
        P[(i - i0) * kPanelLd + c] = x[c];
      }
    }
    __syncthreads();
    // trailing lower triangle: F[i][k] -= P_i . P_k for i0 <= k <= i < d, four
    // consecutive rows per wave step (four independent updates per column k,
    // one LDS read of P_k for all four)
    constexpr int RW = 4;
    for (int q0 = RW * wave; q0 < nt; q0 += RW * kWavesPerBlock) {
      double pi[RW][kPanel];
#pragma unroll
      for (int q = 0; q < RW; ++q)
#pragma unroll
        for (int c = 0; c < kPanel; ++c)
          pi[q][c] = q0 + q < nt ? P[(q0 + q) * kPanelLd + c] : 0.0;
      const int klast = min(q0 + RW, nt) - 1;
      for (int kk = lane; kk <= klast; kk += kWave) {
        double pk[kPanel];
#pragma unroll
        for (int c = 0; c < kPanel; ++c) pk[c] = P[kk * kPanelLd + c];
#pragma unroll
        for (int q = 0; q < RW; ++q)
          if (kk <= q0 + q && q0 + q < nt) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < kPanel; ++c) s += pi[q][c] * pk[c];
            F[(int64_t)(i0 + q0 + q) * ld + i0 + kk] -= s;
          }
      }
    }
    __syncthreads();
  }
  if (bad && lane == 0) *e.fac_bad = 1;
}

__global__ void clear_words(unsigned* p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

}  // namespace

struct BlockPlan {
  BatchKernel kern;
  size_t shmem;
  int G;
  BatchArgs args;
  const GramJob* d_jobs;
  int64_t njobs;
  int sa_f32;
  unsigned* bar;       // barrier words, the error flag and the factorization flags
  int64_t bar_words;
  int exact;           // launch the Cholesky factors before the solve
  int64_t count;
  size_t chol_shmem;
};

size_t block_workspace_bytes(const mihs_handle* h, const BlockEntryDesc* ents, int64_t count) {
  if (count <= 0) return 0;
  // Every schedule has at most G team members in all and at most G items per
  // workgroup list: size for teams of one plus G extra members of the widest
  // entry, and the longest item list.
  const int G = h->num_cu;
  Schedule S;
  S.team0.assign(count, 0);
  S.tsize.assign(count, 1);
  S.tcg.assign(count, 1);
  S.stride = (size_t)std::max<int64_t>(count, G) + 1;
  int dpmax = 64;
  for (int64_t i = 0; i < count; ++i) dpmax = std::max(dpmax, dp_for(ents[i].d));
  const size_t base = block_layout(ents, count, S, G, true).total;
  const size_t extra = (size_t)G * ((size_t)dpmax * KR + kNScal) * sizeof(double) + 256 * (size_t)count;
  return base + extra;
}

int plan_block(const mihs_handle* h, const BlockEntryDesc* ents, int64_t count, int a_f32,
               int sa_f32, double eps_sub, double tol, int64_t max_outer, int64_t max_inner,
               const mihs_batched_tuning_t& tuning, const std::vector<double>* cost, void* ws,
               size_t ws_bytes, hipStream_t st, BlockPlan** out) {
  *out = nullptr;
  if (count <= 0) return MIHS_ERR_INVALID;
  if (!block_tuning_valid(tuning)) return MIHS_ERR_INVALID;
  int dpmax = 64;
  for (int64_t i = 0; i < count; ++i) {
    if (ents[i].d < 1 || ents[i].d > block_max_d() || ents[i].ncols < 1 || ents[i].ncols > KR)
      return MIHS_ERR_INVALID;
    dpmax = std::max(dpmax, dp_for(ents[i].d));
  }
  BatchKernel kern = pick(dpmax);
  if (!kern) return MIHS_ERR_UNSUPPORTED;
  const size_t shmem = lds_bytes(dpmax);
  if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)shmem) != hipSuccess)
    return MIHS_ERR_HIP;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kBlock, shmem) != hipSuccess)
    return MIHS_ERR_HIP;
  if (occ < 1) return MIHS_ERR_UNSUPPORTED;
  const int G = h->num_cu;  // one workgroup per compute unit

  Schedule S;
  int rc = make_schedule(ents, count, G, tuning, cost, &S);
  if (rc) return rc;
  const BlockLayout L = block_layout(ents, count, S, G, tuning.exact != 0);
  if (!ws || L.total > ws_bytes) return MIHS_ERR_WORKSPACE;
  char* base = (char*)ws;

  // ---- Gram matrices of the distinct sketches
  const std::vector<int64_t> lead = group_leaders(ents, count);
  std::vector<GramJob> jobs;
  jobs.reserve(L.njobs);
  for (size_t g = 0; g < lead.size(); ++g) {
    const BlockEntryDesc& s = ents[lead[g]];
    const int dp = dp_for(s.d);
    const int nb = dp / 64;
    for (int bi = 0; bi < nb; ++bi)
      for (int bj = bi; bj < nb; ++bj) {
        GramJob j;
        j.M = s.SA;
        j.m = s.m;
        j.ld = s.ldsa;
        j.H = (void*)(base + L.h_off[g]);
        j.h_f32 = sa_f32;
        j.ldh = dp;
        j.d = (int)s.d;
        j.bi = bi;
        j.bj = bj;
        jobs.push_back(j);
      }
  }

  std::vector<BatchEntry> host(count);
  for (int64_t i = 0; i < count; ++i) {
    const BlockEntryDesc& s = ents[i];
    BatchEntry& e = host[i];
    size_t g = 0;
    while (ents[lead[g]].sa_group != s.sa_group) ++g;
    e.A = s.A;
    e.n = s.n;
    e.lda = s.lda;
    e.B = s.B;
    e.ldb = s.ldb;
    e.ldbc = s.ldbc;
    e.RHS = s.RHS;
    e.ldr = s.ldr;
    e.H = (const void*)(base + L.h_off[g]);
    e.ldh = dp_for(s.d);
    e.X = s.X;
    e.ldx = s.ldx;
    e.lam = s.lam;
    e.alpha = s.alpha;
    e.beta = s.beta;
    e.info = s.info;
    e.work = (double*)(base + L.work_off[i]);
    e.fac = L.fac_off.empty() ? nullptr : (double*)(base + L.fac_off[i]);
    e.fac_bad = (int*)(base + L.bar_off + (size_t)(2 * count + 2) * 128) + i;
    e.bar = (unsigned*)(base + L.bar_off + (size_t)(2 * i + 1) * 128);
    e.bar_cg = (unsigned*)(base + L.bar_off + (size_t)(2 * i + 2) * 128);
    e.d = (int)s.d;
    e.dp = dp_for(s.d);
    e.ncols = s.ncols;
    e.team0 = S.team0[i];
    e.tsize = S.tsize[i];
    e.tcg = S.tcg[i];
  }
  std::vector<int> hitems((size_t)G * S.stride, -1);
  for (int g = 0; g < G; ++g)
    for (size_t k = 0; k < S.items[g].size(); ++k) hitems[(size_t)g * S.stride + k] = S.items[g][k];

  if (hipMemcpyAsync(base + L.ent_off, host.data(), (size_t)count * sizeof(BatchEntry),
                     hipMemcpyHostToDevice, st) != hipSuccess)
    return MIHS_ERR_HIP;
  if (hipMemcpyAsync(base + L.item_off, hitems.data(), hitems.size() * sizeof(int),
                     hipMemcpyHostToDevice, st) != hipSuccess)
    return MIHS_ERR_HIP;
  if (hipMemcpyAsync(base + L.gram_off, jobs.data(), jobs.size() * sizeof(GramJob),
                     hipMemcpyHostToDevice, st) != hipSuccess)
    return MIHS_ERR_HIP;
  // the host tables above are freed when this function returns
  if (hipStreamSynchronize(st) != hipSuccess) return MIHS_ERR_HIP;

  BlockPlan* P = new BlockPlan();
  P->kern = kern;
  P->shmem = shmem;
  P->G = G;
  P->d_jobs = (const GramJob*)(base + L.gram_off);
  P->njobs = (int64_t)jobs.size();
  P->sa_f32 = sa_f32;
  P->bar = (unsigned*)(base + L.bar_off);
  P->bar_words = (int64_t)(2 * count + 2) * 32 + count;
  P->exact = tuning.exact;
  P->count = count;
  P->chol_shmem = chol_lds_bytes(dpmax);
  if (tuning.exact) {
    const void* ck = sa_f32 ? (const void*)chol_kernel<float> : (const void*)chol_kernel<double>;
    if (hipFuncSetAttribute(ck, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)P->chol_shmem) != hipSuccess) {
      delete P;
      return MIHS_ERR_HIP;
    }
  }
  BatchArgs& a = P->args;
  a.entries = (const BatchEntry*)(base + L.ent_off);
  a.wg_items = (const int*)(base + L.item_off);
  a.items_stride = (int)S.stride;
  a.err = (int*)(base + L.bar_off);
  a.a_f32 = a_f32;
  a.h_f32 = sa_f32;
  a.a_dma = tuning.a_dma;
  a.exact = tuning.exact;
  a.wall_khz = h->wall_khz;
  a.eps_sub = eps_sub;
  a.tol = tol;
  a.max_outer = max_outer;
  a.max_inner = max_inner;
  a.spin.limit = 1L << 26;
  a.spin.sleep = 1;
  a.spin_idle.limit = 1L << 24;
  a.spin_idle.sleep = 16;
  *out = P;
  return MIHS_OK;
}

int run_block(const BlockPlan* P, hipStream_t st) {
  // barrier words and the error flag start at zero (a fill kernel, not a
  // memset, so that the sequence can be captured)
  hipLaunchKernelGGL(clear_words, dim3(1), dim3(256), 0, st, P->bar, P->bar_words);
  if (hipGetLastError() != hipSuccess) return MIHS_ERR_HIP;
  if (P->njobs > 0) {
    const int rc = launch_gram_jobs(P->d_jobs, P->njobs, P->sa_f32, st);
    if (rc) return rc;
  }
  if (P->exact) {
    const dim3 grid((unsigned)(P->count * KR));
    if (P->sa_f32)
      hipLaunchKernelGGL(chol_kernel<float>, grid, dim3(kBlock), P->chol_shmem, st,
                         P->args.entries);
    else
      hipLaunchKernelGGL(chol_kernel<double>, grid, dim3(kBlock), P->chol_shmem, st,
                         P->args.entries);
    if (hipGetLastError() != hipSuccess) return MIHS_ERR_HIP;
  }
  BatchArgs a = P->args;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess) return MIHS_ERR_HIP;
  if (cap == hipStreamCaptureStatusActive) {
    // one workgroup per compute unit fits (checked by the plan); the graph
    // node is an ordinary launch
    void* args[] = {&a};
    if (hipLaunchKernel((const void*)P->kern, dim3(P->G), dim3(kBlock), args, P->shmem, st) !=
        hipSuccess)
      return MIHS_ERR_HIP;
    return MIHS_OK;
  }
  void* args[] = {&a};
  if (hipLaunchCooperativeKernel((const void*)P->kern, dim3(P->G), dim3(kBlock), args, P->shmem,
                                 st) != hipSuccess)
    return MIHS_ERR_HIP;
  return MIHS_OK;
}

void free_block_plan(BlockPlan* P) { delete P; }

int launch_block(mihs_handle* h, const BlockEntryDesc* ents, int64_t count, int a_f32,
                 int sa_f32, double eps_sub, double tol, int64_t max_outer, int64_t max_inner,
                 void* ws, size_t ws_bytes, hipStream_t st) {
  if (count <= 0) return MIHS_OK;
  std::vector<double> cost;
  const mihs_batched_tuning_t tn = block_tuning_for(h, ents, count, &cost);
  BlockPlan* P = nullptr;
  int rc = plan_block(h, ents, count, a_f32, sa_f32, eps_sub, tol, max_outer, max_inner, tn,
                      &cost, ws, ws_bytes, st, &P);
  if (rc) return rc;
  rc = run_block(P, st);
  free_block_plan(P);
  return rc;
}

}  // namespace mihs

