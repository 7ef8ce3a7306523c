// fic_search_common.h -- helpers shared by the matrix-core search kernels.
#pragma once

#include "fic_device.h"

namespace fic {

// Device memory seen through a global (address space 1) pointer.  Kernels
// that read their buffer pointers from memory (the batch tables) would
// otherwise issue generic "flat" accesses, which also count against the LDS
// wait counter, so every LDS wait would wait for the operand prefetch too.
template <typename T>
using global_ptr = __attribute__((address_space(1))) T *;

// T a scalar or a clang vector type: HIP's uint2/uint4/float4 are classes
// whose copy constructor takes a generic reference, which brings the flat
// access back.
template <typename T>
__device__ __forceinline__ T gld(const T *p) {
  return *(global_ptr<const T>)p;
}

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned long long load_best(
    const unsigned long long *p) {
  // bypass the non-coherent L1 so other workgroups' improvements are seen
  return __hip_atomic_load((global_ptr<unsigned long long>)p, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Non-returning atomic min of a best key (agent scope).
__device__ __forceinline__ void publish_best(unsigned long long *p,
                                             unsigned long long v) {
  __hip_atomic_fetch_min((global_ptr<unsigned long long>)p, v,
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Prune weight W' = (V - K best)/K^2 of a range from its packed key, rounded
// down (relative 2^-20) so that float rounding in the test can only let more
// candidates through; 0 when the bound is useless, +inf for a range without
// variance (every candidate ties with the seeded candidate 0 there).
__device__ __forceinline__ float weight_from_key(unsigned long long key,
                                                 double V, const Geo &g) {
  const double K = (double)g.K;
  const double Wd = fma(-K * g.invEscale, (double)(key >> g.cbits), V);
  const float w = (float)(fmax(Wd, 0.0) * (g.invK * g.invK)) * (1.0f - 0x1p-20f);
  return V == 0.0 ? __builtin_inff() : w;
}

}  // namespace fic
