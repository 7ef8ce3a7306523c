// fic_device.h -- device helpers shared by the libfic kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fic_internal.h"

namespace fic {

// Source cell of output pixel (i, j) under transform k (the eight symmetries
// of the square, Section V): block[i][j] = T[sigma_k(i, j)], m = n - 1.
__host__ __device__ inline void sigma(int k, int i, int j, int m, int &si,
                                      int &sj) {
  switch (k & 7) {
    case 0: si = i;     sj = j;     break;  // identity
    case 1: si = j;     sj = m - i; break;  // quarter turn ccw
    case 2: si = m - i; sj = m - j; break;  // half turn
    case 3: si = m - j; sj = i;     break;  // three quarter turns ccw
    case 4: si = i;     sj = m - j; break;  // mirror left-right
    case 5: si = j;     sj = i;     break;  // transpose
    case 6: si = m - i; sj = j;     break;  // mirror top-bottom
    default: si = m - j; sj = m - i; break; // anti-transpose
  }
}

// Inverse of sigma_k: the output pixel (i, j) that reads cell (ci, cj).
__host__ __device__ inline void sigma_inv(int k, int ci, int cj, int m, int &i,
                                          int &j) {
  switch (k & 7) {
    case 0: i = ci;     j = cj;     break;
    case 1: i = m - cj; j = ci;     break;
    case 2: i = m - ci; j = m - cj; break;
    case 3: i = cj;     j = m - ci; break;
    case 4: i = ci;     j = m - cj; break;
    case 5: i = cj;     j = ci;     break;
    case 6: i = m - ci; j = cj;     break;
    default: i = m - cj; j = m - ci; break;
  }
}

// Rounded mean of a non-negative block sum: the integer nearest sum / K
// (halves up).  8-bit matrix-core operands are centred on it.
__host__ __device__ inline int centre_of(long long sum, int K) {
  return (int)((sum + K / 2) / K);
}

// The same rounded mean of a sum below 2^24 held in FP32, with invK = 1/K:
// the scaling, the added half and the floor are all exact.
__device__ __forceinline__ float centre_f(float sum, float invK) {
  return floorf(fmaf(sum, invK, 0.5f));
}

// Exact G = sum A b of a candidate from the product h of its centred
// operands (A - m_d and b - m_r, m_d and m_r the rounded means of SA and Sb):
// G = h + m_r SA + m_d Sb - K m_d m_r, every term an integer held exactly.
__device__ __forceinline__ double g_from_centred(double h, double sa,
                                                 double sb, const Geo &g) {
  const double md = floor(fma(sa, g.invK, 0.5)), mr = floor(fma(sb, g.invK, 0.5));
  return h + mr * sa + md * sb - (double)g.K * md * mr;
}

// Position of k-element p of sweep column c in (a plane of) the FP16 domain
// operand.  The matrix-core searches that sweep columns in (nearly) index
// order (a full 8-bit centred search, whose column list is the identity,
// the 16x16 and the 12-bit searches) store the operand in MFMA fragment
// order: block c / 32, k-step p / 16, lane (p / 8 mod 2) 32 + c mod 32,
// element p mod 8, so that the 64 lanes of a wave read one contiguous run
// per k-step.
// Otherwise each column holds its K elements in order.
__host__ __device__ inline size_t bop_index(const Geo &g, long long c, int p) {
  if (g.frag)
    return (size_t)(c >> 5) * 32 * g.K + (size_t)(p >> 4) * 512 +
           (size_t)((((p >> 3) & 1) << 5) | (int)(c & 31)) * 8 + (p & 7);
  return (size_t)c * g.K + p;
}

// The same for a plane of the int8 operand (k-steps of 32 one-byte elements,
// 16 per lane): block c / 32, k-step p / 32, lane (p / 16 mod 2) 32 +
// c mod 32, element p mod 16.
__host__ __device__ inline size_t bop8_index(const Geo &g, long long c, int p) {
  if (g.frag)
    return (size_t)(c >> 5) * 32 * g.K + (size_t)(p >> 5) * 1024 +
           (size_t)((((p >> 4) & 1) << 5) | (int)(c & 31)) * 16 + (p & 15);
  return (size_t)c * g.K + p;
}

// Result of the exact fit of one candidate.
struct Fit {
  double err;  // eq. (8) with quantised s, o
  int j, m;    // contrast / offset indices
};

// Exact least-squares fit and quantisation of one candidate from its integer
// sums (eqs. 9-12).  All inputs are integers held exactly in double:
//   G   = sum_q A[sigma_k(q)] b[q]  (A: 2x2 cell sums, i.e. 4 x the
//                                    contracted value a)
//   SA  = sum A,  SAA = sum A^2,  Sb = sum b,  Sbb = sum b^2.
// With a = A/4 the slope of eq. (9) is 4 N'/D', N' = K G - SA Sb,
// D' = K SAA - SA^2; every other quantity below is a dyadic rational with at
// most 46 significant bits, so the only rounding is that one division.
__device__ __forceinline__ Fit fit_exact(double G, double SA, double SAA,
                                         double Sb, double Sbb, const Geo &g) {
  const double K = (double)g.K;
  const double Dp = K * SAA - SA * SA;
  const double Np = K * G - SA * Sb;
  const double s = (Dp == 0.0) ? 0.0 : (4.0 * Np) / Dp;  // eq. (11) / (9)
  double j = floor((s + 1.0) * g.S + 0.5);
  j = fmin(fmax(j, 0.0), 2.0 * g.S - 1.0);
  // K, S and dlt are powers of two: scaling by the reciprocal is exact
  const double sq = j * g.invS - 1.0;
  const double o = (Sb - sq * SA * 0.25) * g.invK;        // eq. (10) / (12)
  double m = floor((o + g.P) * g.invDlt + 0.5);
  m = fmin(fmax(m, 0.0), ldexp(1.0, g.ob) - 1.0);
  const double oq = m * g.dlt - g.P;
  // eq. (8) expanded over the sums: sum (sq a + oq - b)^2 with a = A/4
  const double E = sq * sq * SAA * 0.0625 + sq * oq * SA * 0.5 -
                   sq * G * 0.5 + K * oq * oq - 2.0 * oq * Sb + Sbb;
  Fit f;
  f.err = E;
  f.j = (int)j;
  f.m = (int)m;
  return f;
}

// 64-bit search key: residual (scaled to an integer) above, candidate below.
// Ordering keys orders (residual, candidate) lexicographically, so a plain
// unsigned min keeps the smallest residual and, among equal residuals, the
// smallest candidate index (the first one met in Alg. 2's loop order).
__device__ __forceinline__ unsigned long long make_key(double err, long long c,
                                                       const Geo &g) {
  const unsigned long long e = (unsigned long long)(err * g.escale);
  return (e << g.cbits) | (unsigned long long)c;
}

__device__ __forceinline__ double key_err(unsigned long long key,
                                          const Geo &g) {
  return (double)(key >> g.cbits) * g.invEscale;
}

// Prune weight of a range from its best residual so far.  A candidate can
// still reach residual <= best only if its unquantised least-squares residual
// (V - N'^2/D')/K does, i.e. only if (G - SA*Sb/K)^2 >= W' D' with
// W' = (V - K best)/K^2, V = K Sbb - Sb^2.  W' is rounded down (relative
// 2^-20) so that float rounding in the test can only let extra candidates
// through.  A range without variance returns +inf: every candidate ties
// with candidate 0 there, which is seeded, so nothing else is examined.
__device__ __forceinline__ float prune_weight(double best_err, double Sb,
                                              double Sbb, const Geo &g) {
  const double K = (double)g.K;
  const double V = K * Sbb - Sb * Sb;
  if (V == 0.0) return __builtin_inff();
  const double Wd = V - K * best_err;
  if (!(Wd > 0.0)) return 0.0f;
  const float w = (float)(Wd / (K * K));
  return w * (1.0f - 0x1p-20f);
}

// Image range held by range slot i (a permutation of [0, R_pad); values
// >= R mark padding slots).
__device__ __forceinline__ int range_of_slot(const Geo &g, int i) {
  // 32-bit arithmetic whenever i * stride < R_pad^2 fits in 32 bits
  if (g.R_pad <= 65535)
    return (int)(((unsigned)i * (unsigned)g.rng_stride) % (unsigned)g.R_pad);
  return (int)(((unsigned long long)i * (unsigned)g.rng_stride) %
               (unsigned)g.R_pad);
}

// Round a positive double down to float (D' can exceed 2^24).
__device__ __forceinline__ float round_down_f(double v) {
  float f = (float)v;
  if ((double)f > v) f = nextafterf(f, 0.0f);
  return f;
}

// Load a workgroup-uniform struct (a slice descriptor, a work item) into
// scalar registers: each 32-bit word is read and broadcast from the first
// active lane.  The caller guarantees that every lane reads the same address.
template <typename T>
__device__ __forceinline__ T load_uniform(const T *p) {
  static_assert(sizeof(T) % 4 == 0, "whole 32-bit words");
  T v;
  const int *src = (const int *)p;
  int *dst = (int *)&v;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i)
    dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
  return v;
}

}  // namespace fic
