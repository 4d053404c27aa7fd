// Streaming kernels with no arithmetic: the measured HBM ceiling that the
// step kernels are compared against.
//
// k_copy_lines   a plain copy, one contiguous tile of 256 * UNROLL elements of
//                W bytes per block, all loads issued before the stores
//                (W = 4, 8 or 16; cached or non-temporal)
// k_copy_soa     the step's access pattern without its arithmetic: one thread
//                per cell reads Q structure-of-arrays rows at its own index
//                (4- or 8-byte accesses, all Q loads in flight; cached or
//                non-temporal) and writes them to Q other rows
//                (non-temporal), plus one extra row read and one written (the
//                phase field's two streams)
#pragma once
#include <hip/hip_runtime.h>

namespace pflbm {

// 8- and 16-byte lanes as clang vector types (the nontemporal builtins take them)
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

template <typename T, int UNROLL, bool NT>
__global__ __launch_bounds__(256) void k_copy_lines(const T* __restrict__ src, T* __restrict__ dst,
                                                    long long n) {
  const long long base = (long long)blockIdx.x * (256 * UNROLL) + threadIdx.x;
  T v[UNROLL];
#pragma unroll
  for (int j = 0; j < UNROLL; ++j) {
    const long long i = base + 256ll * j;
    if (i < n) v[j] = NT ? __builtin_nontemporal_load(src + i) : src[i];
  }
#pragma unroll
  for (int j = 0; j < UNROLL; ++j) {
    const long long i = base + 256ll * j;
    if (i < n) {
      if (NT) __builtin_nontemporal_store(v[j], dst + i); else dst[i] = v[j];
    }
  }
}

template <int Q, bool NT_LOAD, typename T = float>
__global__ __launch_bounds__(256) void k_copy_soa(const T* __restrict__ src, T* __restrict__ dst,
                                                  long long N) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= N) return;
  T v[Q + 1];
#pragma unroll
  for (int q = 0; q <= Q; ++q) v[q] = NT_LOAD ? __builtin_nontemporal_load(src + q * N + idx) : src[q * N + idx];
#pragma unroll
  for (int q = 0; q <= Q; ++q) __builtin_nontemporal_store(v[q], dst + q * N + idx);
}

}  // namespace pflbm
