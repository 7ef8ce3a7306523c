// fic_search_common.h -- helpers shared by the matrix-core search kernels.
#pragma once

#include "fic_device.h"

namespace fic {

__device__ __forceinline__ unsigned long long load_best(
    const unsigned long long *p) {
  // bypass the non-coherent L1 so other workgroups' improvements are seen
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
