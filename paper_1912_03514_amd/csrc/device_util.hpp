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

// Butterfly sum over the 64 lanes; every lane receives the total.  The pairing
// order is fixed, so the result is deterministic.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
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

// Device-wide barrier for a cooperative launch of `nblocks` workgroups.  The
// counter only grows; barrier number e waits for e * nblocks arrivals.  The
// wait is bounded: after `spin_limit` polls the barrier records a timeout in
// *err and every workgroup leaves, so no wave can hang.  Returns false once an
// error is recorded (callers then exit).
__device__ __forceinline__ bool grid_barrier(unsigned* counter, unsigned& epoch, unsigned nblocks,
                                             int* err, int* s_flag, long spin_limit) {
  __syncthreads();
  epoch += 1u;
  if (threadIdx.x == 0) {
    const unsigned target = epoch * nblocks;
    __threadfence();
    atomicAdd(counter, 1u);
    long spins = 0;
    int ok = 1;
    while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > spin_limit) {
        atomicOr(err, 1);
        ok = 0;
        break;
      }
    }
    __threadfence();
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) ok = 0;
    *s_flag = ok;
  }
  __syncthreads();
  return *s_flag != 0;
}

}  // namespace mihs
