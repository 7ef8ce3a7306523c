// fic_block.h -- block access helpers shared by the preparation and code
// extraction kernels: lane-group sums and image row loads.
#pragma once

#include "fic_device.h"

namespace fic {

template <typename Pix>
__device__ __forceinline__ int cell_sum(const Pix *img, int W, int y, int x) {
  const Pix *p = img + (size_t)y * W + x;
  return (int)p[0] + (int)p[1] + (int)p[W] + (int)p[W + 1];
}

// The value of a partner lane inside the lane's row of 16 (DPP, no LDS
// traffic): CTRL 0xB1 = lane ^ 1, 0x4E = lane ^ 2, 0x141 = mirror within 8,
// 0x140 = mirror within 16.  Every lane of the row must be active.
template <int CTRL, typename T>
__device__ __forceinline__ T dpp_partner(T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
  if constexpr (sizeof(T) == 4) {
    const int x = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(
        T, __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false));
  } else {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF,
                                               0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32),
                                               CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(
        T, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
  }
}

// Sum over aligned groups of W lanes (W a power of two <= 64), the result in
// every lane of the group.  Butterfly: after each step every lane holds the
// sum of its aligned group of twice the size.  Every lane of a group must be
// active (integer or exactly representable sums, so the order is free).
template <int W, typename T>
__device__ __forceinline__ T group_sum(T v) {
  static_assert(W >= 1 && W <= 64 && (W & (W - 1)) == 0, "power of two");
  if constexpr (W >= 2) v += dpp_partner<0xB1>(v);
  if constexpr (W >= 4) v += dpp_partner<0x4E>(v);
  if constexpr (W >= 8) v += dpp_partner<0x141>(v);
  if constexpr (W >= 16) v += dpp_partner<0x140>(v);
  if constexpr (W >= 32) v += __shfl_xor(v, 16);
  if constexpr (W >= 64) v += __shfl_xor(v, 32);
  return v;
}

// The C pixels p[0 .. C) of an image row (C sizeof(Pix) a multiple of 4).
// wide: p is 4-byte aligned, so the run is read as 32-bit words (four 8-bit
// or two 16-bit pixels each).
template <typename Pix, int C>
__device__ __forceinline__ void load_run(const Pix *p, bool wide, int (&v)[C]) {
  constexpr int PW = 4 / sizeof(Pix);  // pixels per word
  static_assert(C % PW == 0, "whole words");
  if (wide) {
    const unsigned *w = (const unsigned *)p;
#pragma unroll
    for (int q = 0; q < C / PW; ++q) {
      const unsigned u = w[q];
#pragma unroll
      for (int e = 0; e < PW; ++e)
        v[q * PW + e] = (int)((u >> (8 * sizeof(Pix) * e)) &
                              ((1u << (8 * sizeof(Pix))) - 1u));
    }
  } else {
#pragma unroll
    for (int k = 0; k < C; ++k) v[k] = (int)p[k];
  }
}

// The 2N pixels of one domain row.
template <typename Pix, int N>
__device__ __forceinline__ void load_row(const Pix *p, bool wide,
                                         int (&v)[2 * N]) {
  load_run<Pix, 2 * N>(p, wide, v);
}

// Whether every domain row starts on a 4-byte boundary: the image, its width
// and the domain step allow it.
template <typename Pix>
__device__ __forceinline__ bool domain_rows_aligned(const Geo &g,
                                                    const Pix *img) {
  return ((uintptr_t)img & 3) == 0 &&
         ((g.W | g.step) & (sizeof(Pix) == 1 ? 3 : 1)) == 0;
}

}  // namespace fic
