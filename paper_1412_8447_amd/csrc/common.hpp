// Shared device helpers and launch-argument structures of libidcur (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace idcur {

// Device status bits (written by kernels, read by idcur_sync_status).
enum : int {
  ST_RANKCAP = 1,
  ST_NONFINITE = 2,
  ST_TIMEOUT = 4,
  ST_BADINDEX = 8,   // an index array held a value out of range (clamped)
};

// Spin limit of every grid-wide wait (polls, each followed by s_sleep 1).
// About one second of waiting before a wave gives up and reports ST_TIMEOUT.
constexpr long kSpinLimit = 1L << 24;

// ---------------------------------------------------------------------------
// Coherent (device-scope) loads and stores used to exchange data between
// workgroups on different XCDs inside one kernel. Each XCD has its own L2, so
// ordinary accesses may hit stale lines; agent-scope atomic accesses are
// performed coherently. Ordering between a writer's data and its ready flag is
// enforced by waiting for all outstanding memory operations (s_waitcnt 0)
// before the flag store; readers issue their data loads only after the flag
// load has returned the expected value.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void cstore(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T cload(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void wait_all_mem() { __builtin_amdgcn_s_waitcnt(0); }

__device__ __forceinline__ void set_status(int* status, int bit) {
  if (status) atomicOr(status, bit);
}

// ---------------------------------------------------------------------------
// Reductions.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// Sum within aligned groups of G consecutive lanes (G a power of two <= 64).
template <typename T>
__device__ __forceinline__ T group_sum(T v, int G) {
  for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Argmax key: larger value wins; equal values go to the smaller index.
struct ArgMax {
  double v;
  int i;
};
__device__ __forceinline__ bool better(double va, int ia, double vb, int ib) {
  return (va > vb) || (va == vb && ia < ib);
}
__device__ __forceinline__ ArgMax wave_argmax(ArgMax a) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    double ov = __shfl_xor(a.v, o, 64);
    int oi = __shfl_xor(a.i, o, 64);
    if (better(ov, oi, a.v, a.i)) { a.v = ov; a.i = oi; }
  }
  return a;
}

template <typename T>
__device__ __forceinline__ T ldg(const T* p) { return *p; }

__host__ __device__ constexpr inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ constexpr inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

}  // namespace idcur
