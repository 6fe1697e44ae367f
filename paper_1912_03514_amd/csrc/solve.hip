// Persistent M-IHS solve kernel (Algorithm 1 with a CG inner solver).
//
// One cooperative launch runs the whole outer loop.  Every workgroup stays
// resident; phases are separated by a device-wide barrier:
//
//   A1  stage x in LDS; stream this workgroup's contiguous row block of A once:
//       each wave holds whole rows in registers, forms r_i = b_i - A_i x by a
//       wave reduction and accumulates A_i^T r_i into per-lane partial
//       gradients; the four waves combine in LDS and write one partial d-vector.
//   A2  column owners add the partials (fixed order), form
//       g = sum + rhs - lambda x and start CG (z = 0, r = p = g).
//   CG  per iteration two barriers:
//       C1  every workgroup forms p = r + beta_cg p_prev in LDS (owners also
//           store their slice), and the first Gcg workgroups stream their rows
//           of SA: u_j = SA_j p, partial -SA^T u, sum u_j^2.
//       C2  p^T q = ||u||^2 + lambda ||p||^2 (scalar partials, fixed order),
//           owners form q = -sum + lambda p and update z, r.
//       The stop test ||r|| <= eps_sub ||g|| uses sums that every workgroup
//       computes identically, so all leave the loop together.
//   U   owners apply the heavy-ball step x+ = x + alpha z + beta (x - x_prev)
//       and the relative-step stop test.
//
// Every reduction runs in a fixed order, so a solve is bit-reproducible.
#include <math.h>

#include "device_util.hpp"
#include "internal.hpp"

namespace mihs {

namespace {

constexpr int kScal = 8;           // scalar partial slots per workgroup
constexpr int kMaxBlocksPerCU = 2;

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
  double* partA;
  void* partS;
  double* scal;
  void* r;
  void* z;
  void* p0;
  void* p1;
  unsigned* bar;
  int* err;
  int d, dpad, G, Gcg, cpw;
  long spin_limit;
};

template <int EPT>
struct RowsInFlight {
  static constexpr int value = EPT >= 64 ? 1 : (EPT >= 8 ? 2 : 4);
};

// One pass over rows [r0, r1) of M: for each row, u = c_row - M_row . v and
// acc += u * M_row (acc in this lane's columns), ssq += u^2.
template <typename TM, typename TV, int EPT, bool NT>
__device__ __forceinline__ void rowpass(const TM* __restrict__ M, int64_t ld, int64_t r0,
                                        int64_t r1, int d, const TV* __restrict__ v,
                                        const double* __restrict__ c, TV (&acc)[EPT], TV& ssq) {
  using L = RowLayout<TM, EPT>;
  constexpr int R = RowsInFlight<EPT>::value;
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
      if (row + t < r1) u = (c ? (TV)c[row + t] : TV(0)) - dot[t];
      ssq += u * u;
#pragma unroll
      for (int e = 0; e < EPT; ++e) acc[e] += u * (TV)rv[t][e];
    }
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
  for (int col = threadIdx.x; col < d; col += kBlock) out[col] = red[col];
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

template <typename TA, typename TS, typename TV, int EPT>
__global__ __launch_bounds__(kBlock) void solve_kernel(SolveArgs a) {
  extern __shared__ double smem[];
  double* vbuf = smem;           // x (A pass) or p (CG, as TV)
  double* rbuf = smem + a.dpad;  // workgroup reduction buffer
  __shared__ double s_red[kWavesPerBlock];
  __shared__ int s_flag;

  const int w = blockIdx.x;
  const int G = a.G;
  const int d = a.d;
  unsigned epoch = 0;
  const int c_lo = min(d, w * a.cpw);
  const int c_hi = min(d, c_lo + a.cpw);
  double* scal_w = a.scal + (int64_t)w * kScal;
  TV* r = (TV*)a.r;
  TV* z = (TV*)a.z;
  TV* P[2] = {(TV*)a.p0, (TV*)a.p1};
  TV* partS = (TV*)a.partS;
  const TA* A = (const TA*)a.A;
  const TS* SA = (const TS*)a.SA;

  if (a.xp_from_x)
    for (int c = c_lo + threadIdx.x; c < c_hi; c += kBlock) a.xp[c] = a.x[c];

  const int64_t a_r0 = a.n * w / G, a_r1 = a.n * (w + 1) / G;
  const int64_t s_r0 = (w < a.Gcg) ? a.m * w / a.Gcg : 0;
  const int64_t s_r1 = (w < a.Gcg) ? a.m * (w + 1) / a.Gcg : 0;

  int64_t outer = 0, inner_total = 0, inner_max = 0;
  double last_step = 0.0, last_gnorm = 0.0;
  int status = MIHS_MAX_ITER;
  bool alive = true;

  while (outer < a.max_outer) {
    // ---- A1: partial A^T (b - A x) over this workgroup's rows
    for (int c = threadIdx.x; c < a.dpad; c += kBlock) vbuf[c] = (c < d) ? a.x[c] : 0.0;
    __syncthreads();
    {
      double acc[EPT];
#pragma unroll
      for (int e = 0; e < EPT; ++e) acc[e] = 0.0;
      double ssq = 0.0;
      rowpass<TA, double, EPT, true>(A, a.lda, a_r0, a_r1, d, vbuf, a.b, acc, ssq);
      wg_store_partial<TA, double, EPT>(acc, rbuf, a.partA + (int64_t)w * a.dpad, d);
    }
    if (!(alive = grid_barrier(a.bar, epoch, G, a.err, &s_flag, a.spin_limit))) break;

    // ---- A2: owners form g and start CG
    double rr_part = 0.0;
    for (int c = c_lo; c < c_hi; ++c) {
      const double s = block_sum_strided(a.partA + c, G, a.dpad, s_red);
      if (threadIdx.x == 0) {
        const double g = s + (a.rhs ? a.rhs[c] : 0.0) - a.lam * a.x[c];
        const TV gt = (TV)g;
        r[c] = gt;
        z[c] = TV(0);
        P[0][c] = gt;
        rr_part += (double)gt * (double)gt;
      }
    }
    if (threadIdx.x == 0) scal_w[0] = rr_part;
    if (!(alive = grid_barrier(a.bar, epoch, G, a.err, &s_flag, a.spin_limit))) break;

    const double rr0 = block_sum_strided(a.scal + 0, G, kScal, s_red);
    last_gnorm = sqrt(rr0);
    if (!(rr0 > 0.0)) {  // stationary point (or NaN)
      status = (rr0 == 0.0) ? MIHS_CONVERGED : MIHS_BREAKDOWN;
      break;
    }
    const double stop = a.eps_sub * a.eps_sub * rr0;
    double rr = rr0, bcg = 0.0;
    int64_t k = 0;
    bool breakdown = false;
    while (true) {
      // ---- C1: p = r + beta_cg p_prev (k > 0), staged in LDS; pass over SA
      TV* vp = (TV*)vbuf;
      TV* pcur = P[k & 1];
      const TV* pprev = P[(k + 1) & 1];
      const TV bc = (TV)bcg;
      for (int c = threadIdx.x; c < a.dpad; c += kBlock) {
        TV pv = TV(0);
        if (c < d) {
          pv = (k == 0) ? pcur[c] : (TV)(r[c] + bc * pprev[c]);
          if (k > 0 && c >= c_lo && c < c_hi) pcur[c] = pv;
        }
        vp[c] = pv;
      }
      __syncthreads();
      double pp = 0.0;
      if (threadIdx.x == 0)
        for (int c = c_lo; c < c_hi; ++c) pp += (double)vp[c] * (double)vp[c];
      TV ssq = TV(0);
      if (w < a.Gcg) {
        TV acc[EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e) acc[e] = TV(0);
        rowpass<TS, TV, EPT, false>(SA, a.ldsa, s_r0, s_r1, d, vp, nullptr, acc, ssq);
        wg_store_partial<TS, TV, EPT>(acc, (TV*)rbuf, partS + (int64_t)w * a.dpad, d);
        ssq = wg_sum_ssq(ssq, s_red);
      }
      if (threadIdx.x == 0) {
        scal_w[1] = pp;
        scal_w[2] = (double)ssq;
      }
      if (!(alive = grid_barrier(a.bar, epoch, G, a.err, &s_flag, a.spin_limit))) break;

      // ---- C2: step length and owner updates
      const double uu = block_sum_strided(a.scal + 2, G, kScal, s_red);
      const double ppn = block_sum_strided(a.scal + 1, G, kScal, s_red);
      const double pq = uu + a.lam * ppn;
      const double acg = rr / pq;
      if (!(pq > 0.0) || !isfinite(acg)) {
        breakdown = true;
        break;
      }
      double rpart = 0.0;
      const TV at = (TV)acg, lt = (TV)a.lam;
      for (int c = c_lo; c < c_hi; ++c) {
        const double qs = block_sum_strided(partS + c, a.Gcg, a.dpad, s_red);
        if (threadIdx.x == 0) {
          const TV pc = vp[c];
          const TV q = (TV)(-qs) + lt * pc;
          z[c] = z[c] + at * pc;
          const TV rn = r[c] - at * q;
          r[c] = rn;
          rpart += (double)rn * (double)rn;
        }
      }
      if (threadIdx.x == 0) scal_w[3] = rpart;
      if (!(alive = grid_barrier(a.bar, epoch, G, a.err, &s_flag, a.spin_limit))) break;
      const double rr_new = block_sum_strided(a.scal + 3, G, kScal, s_red);
      ++k;
      bcg = rr_new / rr;
      rr = rr_new;
      if (rr <= stop || k >= a.max_inner) break;
    }
    if (!alive) break;
    inner_total += k;
    if (k > inner_max) inner_max = k;
    if (breakdown) {
      status = MIHS_BREAKDOWN;
      break;
    }

    // ---- U: heavy-ball update on owned columns, relative-step test
    double s0 = 0.0, s1 = 0.0;
    if (threadIdx.x == 0) {
      for (int c = c_lo; c < c_hi; ++c) {
        const double xc = a.x[c];
        const double xn = xc + a.alpha * (double)z[c] + a.beta * (xc - a.xp[c]);
        a.xp[c] = xc;
        a.x[c] = xn;
        s0 += (xn - xc) * (xn - xc);
        s1 += xn * xn;
      }
      scal_w[4] = s0;
      scal_w[5] = s1;
    }
    if (!(alive = grid_barrier(a.bar, epoch, G, a.err, &s_flag, a.spin_limit))) break;
    const double S0 = block_sum_strided(a.scal + 4, G, kScal, s_red);
    const double S1 = block_sum_strided(a.scal + 5, G, kScal, s_red);
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
  }
  if (!alive) status = MIHS_BARRIER_TIMEOUT;
  if (w == 0 && threadIdx.x == 0) {
    a.info->outer_iters = outer;
    a.info->inner_iters_total = inner_total;
    a.info->inner_iters_max = inner_max;
    a.info->rel_step = last_step;
    a.info->grad_norm = last_gnorm;
    a.info->status = status;
    a.info->reserved = 0;
  }
}

__global__ void zero_words(unsigned* p, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0u;
}

typedef void (*SolveKernel)(SolveArgs);

template <typename TA, typename TS, typename TV>
SolveKernel pick_by_ept(int ept) {
  switch (ept) {
    case 1: return solve_kernel<TA, TS, TV, 1>;
    case 2: return solve_kernel<TA, TS, TV, 2>;
    case 4: return solve_kernel<TA, TS, TV, 4>;
    case 8: return solve_kernel<TA, TS, TV, 8>;
    case 16: return solve_kernel<TA, TS, TV, 16>;
    case 32: return solve_kernel<TA, TS, TV, 32>;
    case 64: return solve_kernel<TA, TS, TV, 64>;
    default: return nullptr;
  }
}

SolveKernel pick_kernel(int a_f32, int mixed, int ept) {
  if (!a_f32 && !mixed) return pick_by_ept<double, double, double>(ept);
  if (!a_f32 && mixed) return pick_by_ept<double, float, float>(ept);
  if (a_f32 && !mixed) return pick_by_ept<float, double, double>(ept);
  return pick_by_ept<float, float, float>(ept);
}

struct SolveLayout {
  size_t partA, partS, scal, vecs, xp, bar, total;
};

SolveLayout layout(int G, int Gcg, int64_t dpad) {
  SolveLayout L;
  size_t off = 0;
  L.partA = off; off = align_up(off + (size_t)G * dpad * 8, 256);
  L.partS = off; off = align_up(off + (size_t)Gcg * dpad * 8, 256);
  L.scal = off;  off = align_up(off + (size_t)G * kScal * 8, 256);
  L.vecs = off;  off = align_up(off + 4 * (size_t)dpad * 8, 256);
  L.xp = off;    off = align_up(off + (size_t)dpad * 8, 256);
  L.bar = off;   off = align_up(off + 256, 256);
  L.total = off;
  return L;
}

int max_grid(const mihs_handle* h) { return h->num_cu * kMaxBlocksPerCU; }

}  // namespace

int ept_for(int64_t d) {
  int e = 1;
  while (64 * (int64_t)e < d) e *= 2;
  return e;
}

size_t solve_workspace_bytes(const mihs_handle* h, int64_t n, int64_t d, int64_t m, int mixed) {
  (void)n;
  (void)m;
  (void)mixed;
  const int G = max_grid(h);
  return layout(G, G, dpad_for(d)).total;
}

int launch_solve(const mihs_handle* h, const SolveDesc& s, void* ws, size_t ws_bytes,
                 hipStream_t stream) {
  const int ept = ept_for(s.d);
  if (ept > 64) return MIHS_ERR_UNSUPPORTED;
  SolveKernel kern = pick_kernel(s.a_f32, s.mixed, ept);
  if (!kern) return MIHS_ERR_UNSUPPORTED;
  const int64_t dpad = dpad_for(s.d);
  const size_t shmem = 2 * (size_t)dpad * sizeof(double);
  if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)shmem) != hipSuccess)
    return MIHS_ERR_HIP;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kBlock, shmem) != hipSuccess)
    return MIHS_ERR_HIP;
  if (occ < 1) return MIHS_ERR_UNSUPPORTED;
  occ = occ > kMaxBlocksPerCU ? kMaxBlocksPerCU : occ;
  int G = h->num_cu * occ;
  // small problems: keep at least ~64 rows of A per workgroup
  const int64_t g_rows = (s.n + 63) / 64;
  if ((int64_t)G > g_rows) G = (int)(g_rows < 1 ? 1 : g_rows);
  constexpr int kRowsPerWaveCG = 2;
  int64_t gcg = (s.m + kWavesPerBlock * kRowsPerWaveCG - 1) / (kWavesPerBlock * kRowsPerWaveCG);
  if (gcg > G) gcg = G;
  if (gcg < 1) gcg = 1;
  const SolveLayout L = layout(G, (int)gcg, dpad);
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
  a.bar = (unsigned*)(base + L.bar);
  a.err = (int*)(base + L.bar + 64);
  a.d = (int)s.d;
  a.dpad = (int)dpad;
  a.G = G;
  a.Gcg = (int)gcg;
  a.cpw = (int)((s.d + G - 1) / G);
  a.spin_limit = 1L << 25;

  hipLaunchKernelGGL(zero_words, dim3(1), dim3(64), 0, stream, a.bar, 64);
  if (hipGetLastError() != hipSuccess) return MIHS_ERR_HIP;
  void* args[] = {&a};
  if (hipLaunchCooperativeKernel((const void*)kern, dim3(G), dim3(kBlock), args, shmem, stream) !=
      hipSuccess)
    return MIHS_ERR_HIP;
  return MIHS_OK;
}

}  // namespace mihs
