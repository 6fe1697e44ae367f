// Device helpers shared by the libmihs kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mihs {

constexpr int kWave = 64;
constexpr int kBlock = 256;            // 4 waves per workgroup everywhere
constexpr int kWavesPerBlock = kBlock / kWave;

typedef double dbl2 __attribute__((ext_vector_type(2)));
typedef float flt2 __attribute__((ext_vector_type(2)));
typedef float flt4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// Lane moves inside rows of 16 lanes (DPP): CTRL is a permutation of each
// row's lanes, so every lane reads a lane of its own row.
template <int CTRL>
__device__ __forceinline__ int dpp_row_move(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_row_move(double x) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)dpp_row_move<CTRL>((int)(unsigned)b);
  const unsigned hi = (unsigned)dpp_row_move<CTRL>((int)(unsigned)(b >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_row_move(float x) {
  return __builtin_bit_cast(float, dpp_row_move<CTRL>(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ double read_lane(double x, int l) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ float read_lane(float x, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
}

// Sum over the 64 lanes of a wave whose lanes are all active; every lane
// receives the total.  Each row of 16 lanes is summed by DPP moves (lane ^ 1,
// lane ^ 2, the mirrored half-row, the mirrored row), then the four row sums
// are read as scalars and added in order.  The order is fixed, so the result
// is deterministic.  (The butterfly over __shfl_xor, an LDS permute per stage
// and two per double, made the CG step's row products 0.55 us slower.)
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  v += dpp_row_move<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_row_move<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_row_move<0x141>(v);  // row_half_mirror
  v += dpp_row_move<0x140>(v);  // row_mirror
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Deterministic workgroup sum (256 threads); every thread receives the total.
// `scratch` is __shared__ storage of at least kWavesPerBlock elements.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* scratch) {
  v = wave_sum(v);
  __syncthreads();
  if (lane_id() == 0) scratch[wave_id()] = v;
  __syncthreads();
  T t = scratch[0];
#pragma unroll
  for (int w = 1; w < kWavesPerBlock; ++w) t += scratch[w];
  return t;
}

// Sum of `count` doubles at base[0], base[stride], ... in a fixed order.
template <typename T>
__device__ __forceinline__ double block_sum_strided(const T* base, int count, int64_t stride,
                                                    double* scratch) {
  double v = 0.0;
  for (int k = threadIdx.x; k < count; k += kBlock) v += (double)base[(int64_t)k * stride];
  return block_sum(v, scratch);
}

// Loads of one row chunk.  Streaming matrices (read once per pass) use
// non-temporal loads so they do not evict the reused sketch from the caches.
template <typename T, int V, bool NT>
struct VecLoad;

template <bool NT>
struct VecLoad<double, 2, NT> {
  static __device__ __forceinline__ void run(const double* p, double* out) {
    dbl2 v = NT ? __builtin_nontemporal_load((const dbl2*)p) : *(const dbl2*)p;
    out[0] = v.x;
    out[1] = v.y;
  }
};
template <bool NT>
struct VecLoad<double, 4, NT> {
  static __device__ __forceinline__ void run(const double* p, double* out) {
    VecLoad<double, 2, NT>::run(p, out);
    VecLoad<double, 2, NT>::run(p + 2, out + 2);
  }
};
template <bool NT>
struct VecLoad<float, 4, NT> {
  static __device__ __forceinline__ void run(const float* p, float* out) {
    flt4 v = NT ? __builtin_nontemporal_load((const flt4*)p) : *(const flt4*)p;
    out[0] = v.x;
    out[1] = v.y;
    out[2] = v.z;
    out[3] = v.w;
  }
};
template <bool NT>
struct VecLoad<float, 2, NT> {
  static __device__ __forceinline__ void run(const float* p, float* out) {
    flt2 v = NT ? __builtin_nontemporal_load((const flt2*)p) : *(const flt2*)p;
    out[0] = v.x;
    out[1] = v.y;
  }
};
template <typename T, bool NT>
struct VecLoad<T, 1, NT> {
  static __device__ __forceinline__ void run(const T* p, T* out) {
    out[0] = NT ? __builtin_nontemporal_load(p) : *p;
  }
};

// Vector width (elements per 16-byte load) used for a row of T split into EPT
// elements per lane.
template <typename T, int EPT>
struct RowLayout {
  static constexpr int kVecFull = 16 / (int)sizeof(T);
  static constexpr int V = EPT < kVecFull ? EPT : kVecFull;
  static constexpr int J = EPT / V;  // 16-byte chunks per lane
  // column of element (j, v) held by `lane`
  static __device__ __forceinline__ int col(int j, int lane, int v) { return (j * kWave + lane) * V + v; }
};

// Load one row (EPT elements per lane); columns >= d read as zero.
template <typename T, int EPT, bool NT>
__device__ __forceinline__ void load_row(const T* __restrict__ row, int d, int lane, T (&out)[EPT]) {
  using L = RowLayout<T, EPT>;
#pragma unroll
  for (int j = 0; j < L::J; ++j) {
    const int c0 = L::col(j, lane, 0);
    if (c0 + L::V <= d) {
      VecLoad<T, L::V, NT>::run(row + c0, &out[j * L::V]);
    } else {
#pragma unroll
      for (int v = 0; v < L::V; ++v) out[j * L::V + v] = (c0 + v < d) ? row[c0 + v] : T(0);
    }
  }
}

// ---- Device-wide barriers and the data they hand over ----------------------
// The persistent kernels (one cooperative launch per solve) meet at counting
// barriers: counters only grow, and barrier number e of a group of `nblocks`
// workgroups waits for e * nblocks arrivals.  Each XCD has its own L2, and the
// L2s are not kept coherent with each other, so data one workgroup writes for
// another during the launch must not sit in an L2:
//
//  * every such value is stored with co_store (an agent-scope store, sc1:
//    written through to memory) and read with co_load (an agent-scope load,
//    sc1: served coherently, never from a stale L2 line) -- how the compiler
//    implements relaxed agent-scope atomics; no plain store ever writes an
//    address another workgroup reads or writes during the launch (a plain
//    store's dirty L2 line could be written back later over a newer value);
//  * at a barrier every wave first waits until its own stores have completed
//    (vmcnt(0); on gfx950 the counter covers stores, and __syncthreads, a bare
//    s_barrier, does not wait for other waves' stores), then the workgroup
//    meets, and thread 0 arrives with a relaxed fetch-add and polls with
//    relaxed loads; loads issued after the wait observe every store made before
//    any arrival.
//
// Data only read during the launch (A, b, SA, the Gram matrix) keeps plain
// cached loads and stays in the L2s across barriers.  (Checked on the
// hardware: 128 and 256 workgroups exchanging slots across all XCDs, 1.3e10
// reads, no stale value; the same exchange through plain accesses read stale
// values almost everywhere.  The alternative -- plain accesses, with the L2
// written back before each arrival and invalidated after each wait -- is also
// correct, but the write-backs and invalidations walk the whole L2 of the XCD
// and queue up when 16-32 workgroups per XCD arrive together: 6.5 us per
// barrier at 128 workgroups against 3.2 us, 11.3 against 5.8 us at 256, and
// every line the workgroups were reusing, a Gram matrix re-read by every CG
// step, had to come back from memory after each barrier.)
//
// The waits are bounded: after `spin.limit` polls a barrier records a timeout
// in *err and returns false, so no wave can hang; callers then leave the
// kernel.
struct BarrierSpin {
  long limit;
  int sleep;  // s_sleep argument between polls (x64 clocks)
};

template <typename T>
__device__ __forceinline__ T co_load(const T* p) {
  typedef const T __attribute__((address_space(1))) gT;
  return __hip_atomic_load((gT*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void co_store(T* p, T v) {
  typedef T __attribute__((address_space(1))) gT;
  __hip_atomic_store((gT*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool wait_counter(const unsigned* counter, unsigned target, int* err,
                                             BarrierSpin spin) {
  long spins = 0;
  while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (spin.sleep >= 16)
      __builtin_amdgcn_s_sleep(16);
    else
      __builtin_amdgcn_s_sleep(1);
    if (++spins > spin.limit) {
      atomicOr(err, 1);
      return false;
    }
  }
  return true;
}

__device__ __forceinline__ void publish_wave_stores() {
  asm volatile("" ::: "memory");       // no memory access moves across the wait
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt and lgkmcnt unconstrained
  asm volatile("" ::: "memory");
}

// One counter shared by all `nblocks` workgroups (cheap up to ~128 of them).
__device__ __forceinline__ bool barrier_flat(unsigned* counter, unsigned& epoch, unsigned nblocks,
                                             int* err, int* s_flag, BarrierSpin spin) {
  publish_wave_stores();
  __syncthreads();
  epoch += 1u;
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = wait_counter(counter, epoch * nblocks, err, spin) ? 1 : 0;
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) ok = 0;
    *s_flag = ok;
  }
  __syncthreads();
  asm volatile("" ::: "memory");
  return *s_flag != 0;
}

// Two-level barrier for large groups: workgroups arrive on one of 8 group
// counters (blockIdx % 8, one 128-byte line each: the workgroups of one XCD);
// the last arrival of a group arrives on the top counter, which everybody waits
// on.  `words` points at 9 lines: top counter first, then the group counters.
// The group's workgroups are blockIdx 0 .. nblocks - 1.
__device__ __forceinline__ bool barrier_hier(unsigned* words, unsigned& epoch, unsigned nblocks,
                                             int* err, int* s_flag, BarrierSpin spin) {
  publish_wave_stores();
  __syncthreads();
  epoch += 1u;
  if (threadIdx.x == 0) {
    const unsigned g = blockIdx.x & 7u;
    const unsigned ngroups = nblocks < 8u ? nblocks : 8u;
    const unsigned gsize = (nblocks - g + 7u) / 8u;
    unsigned* top = words;
    unsigned* gc = words + 32u * (1u + g);
    const unsigned old = __hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old == epoch * gsize - 1u)
      __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = wait_counter(top, epoch * ngroups, err, spin) ? 1 : 0;
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) ok = 0;
    *s_flag = ok;
  }
  __syncthreads();
  asm volatile("" ::: "memory");
  return *s_flag != 0;
}

}  // namespace mihs
