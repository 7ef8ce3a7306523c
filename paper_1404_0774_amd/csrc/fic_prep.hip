// fic_prep.hip -- operand packing, statistics, seeding and the final code
// extraction of the range-domain search.
#include <math.h>

#include "fic_device.h"

namespace fic {

namespace {

template <typename Pix>
__device__ __forceinline__ int cell_sum(const Pix *img, int W, int y, int x) {
  const Pix *p = img + (size_t)y * W + x;
  return (int)p[0] + (int)p[1] + (int)p[W] + (int)p[W + 1];
}

// One thread per (column, group of 8 cells).  Column c of the sweep holds
// domain d = (c * dom_stride) mod ND; its 2x2 cell sums A (4x the contracted
// value of Alg. 1) are written as exact FP16 integers.  12-bit images store
// A = 128 A_hi + A_lo as two planes.
template <typename Pix, int K>
__global__ void k_prep_domains(Geo g, const Pix *img, EncBufs b) {
  constexpr int GRP = K / 8;  // threads per column
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long col = t / GRP;
  const int part = (int)(t % GRP);
  if (col >= g.NC_pad) return;
  const int n = g.n;
  long long SA = 0, SAA = 0;
  int d = -1;
  _Float16 hi[8], lo[8];
  if (col < g.ND) {
    d = (int)((col * (long long)g.dom_stride) % g.ND);
    const int Y = (d / g.NX) * g.step, X = (d % g.NX) * g.step;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int q = part * 8 + e, i = q / n, j = q % n;
      const int A = cell_sum(img, g.W, Y + 2 * i, X + 2 * j);
      SA += A;
      SAA += (long long)A * A;
      if (g.bits == 12) {
        hi[e] = (_Float16)(float)(A >> 7);
        lo[e] = (_Float16)(float)(A & 127);
      } else {
        hi[e] = (_Float16)(float)A;
        lo[e] = (_Float16)0.0f;
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) hi[e] = lo[e] = (_Float16)0.0f;
  }
  _Float16 *dst = b.bop + (size_t)col * K + part * 8;
#pragma unroll
  for (int e = 0; e < 8; ++e) dst[e] = hi[e];
  if (g.bits == 12) {
    _Float16 *dl = b.bop + (size_t)g.NC_pad * K + (size_t)col * K + part * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e) dl[e] = lo[e];
  }
  // reduce the column statistics over its GRP threads (adjacent lanes)
#pragma unroll
  for (int o = 1; o < GRP; o <<= 1) {
    SA += __shfl_xor(SA, o, GRP);
    SAA += __shfl_xor(SAA, o, GRP);
  }
  if (part == 0) {
    b.col_dom[col] = d;
    b.col_sa[col] = (float)SA;
    b.col_saa[col] = (double)SAA;
    if (d < 0) {
      b.col_dp[col] = __builtin_inff();
    } else {
      const double Dp = (double)K * (double)SAA - (double)SA * (double)SA;
      b.col_dp[col] = round_down_f(Dp);  // exact D' for later, flags below
      if (Dp == 0.0) atomicMin(b.flat_first, d);
    }
  }
}

// Flat domains (no variance) all fit any range with s = 0 and the same o
// (eq. 11-12), so they tie; only the first one (smallest d) can be kept.
__global__ void k_prep_flat(Geo g, EncBufs b) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= g.ND) return;
  if (b.col_dp[col] == 0.0f && b.col_dom[col] != *b.flat_first)
    b.col_dp[col] = __builtin_inff();
}

// One thread per (range, transform).  Row 8 r + k of the range operand holds
// the range pixels b placed so that sum_p T[p] row[p] = sum_q T[sigma_k(q)]
// b[q], i.e. row[sigma_k(q)] = b[q].  12-bit: b = 64 b_hi + b_lo, two planes.
// The k = 0 thread also writes the range statistics and seeds the range's
// best key with candidate c = 0 (domain 0, identity), evaluated exactly.
template <typename Pix, int K>
__global__ void k_prep_ranges(Geo g, const Pix *img, EncBufs b) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = t >> 3, k = t & 7;
  if (r >= g.R_pad) return;
  const int n = g.n, m = n - 1;
  _Float16 *row_hi = b.aop + ((size_t)r * 8 + k) * K;
  _Float16 *row_lo = b.aop + (size_t)g.R_pad * 8 * K + ((size_t)r * 8 + k) * K;
  if (r >= g.R) {
    for (int p = 0; p < K; ++p) row_hi[p] = (_Float16)0.0f;
    if (g.bits == 12)
      for (int p = 0; p < K; ++p) row_lo[p] = (_Float16)0.0f;
    if (k == 0) {
      b.rng_sb[r] = 0.0;
      b.rng_sbb[r] = 0.0;
      b.best[r] = ~0ull;
    }
    return;
  }
  const int ry = r / g.RW, rx = r % g.RW;
  long long Sb = 0, Sbb = 0, G0 = 0, SA0 = 0, SAA0 = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const int v = (int)img[(size_t)(ry * n + i) * g.W + rx * n + j];
      int si, sj;
      sigma(k, i, j, m, si, sj);
      const int p = si * n + sj;
      if (g.bits == 12) {
        row_hi[p] = (_Float16)(float)(v >> 6);
        row_lo[p] = (_Float16)(float)(v & 63);
      } else {
        row_hi[p] = (_Float16)(float)v;
      }
      if (k == 0) {
        Sb += v;
        Sbb += (long long)v * v;
        const int A = cell_sum(img, g.W, 2 * i, 2 * j);  // domain 0 at (0, 0)
        G0 += (long long)A * v;
        SA0 += A;
        SAA0 += (long long)A * A;
      }
    }
  if (k == 0) {
    b.rng_sb[r] = (double)Sb;
    b.rng_sbb[r] = (double)Sbb;
    const Fit f = fit_exact((double)G0, (double)SA0, (double)SAA0, (double)Sb,
                            (double)Sbb, g);
    b.best[r] = make_key(f.err, 0, g);
  }
}

// One thread per range: unpack the winning key and recompute its fit from
// the image to produce the code (domain, transform, s index, o index, error).
template <typename Pix>
__global__ void k_finalize(Geo g, const Pix *img, EncBufs b, fic_codes out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= g.R) return;
  const unsigned long long key = b.best[r];
  const long long c = (long long)(key & ((1ull << g.cbits) - 1));
  const int d = (int)(c >> 3), k = (int)(c & 7);
  const int n = g.n, m = n - 1;
  const int ry = r / g.RW, rx = r % g.RW;
  const int Y = (d / g.NX) * g.step, X = (d % g.NX) * g.step;
  long long G = 0, SA = 0, SAA = 0, Sb = 0, Sbb = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const long long v = (long long)img[(size_t)(ry * n + i) * g.W + rx * n + j];
      int si, sj;
      sigma(k, i, j, m, si, sj);
      const long long A = cell_sum(img, g.W, Y + 2 * si, X + 2 * sj);
      G += A * v;
      SA += A;
      SAA += A * A;
      Sb += v;
      Sbb += v * v;
    }
  const Fit f = fit_exact((double)G, (double)SA, (double)SAA, (double)Sb,
                          (double)Sbb, g);
  out.domain[r] = d;
  out.iso[r] = (uint8_t)k;
  out.s_idx[r] = (uint8_t)f.j;
  out.o_idx[r] = (uint8_t)f.m;
  out.err[r] = f.err;
}

__global__ void k_fill_i32(int32_t *p, int v) { *p = v; }

template <typename Pix>
hipError_t prep_impl(const Geo &g, const Pix *img, const EncBufs &b,
                     hipStream_t st) {
  // flat_first := ND (a fill kernel rather than a memset node keeps the
  // sequence safe to capture into a graph)
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(1), 0, st, b.flat_first, g.ND);
  const long long dthreads = (long long)g.NC_pad * (g.K / 8);
  const int bs = 256;
  if (g.K == 64)
    hipLaunchKernelGGL((k_prep_domains<Pix, 64>), dim3((dthreads + bs - 1) / bs),
                       dim3(bs), 0, st, g, img, b);
  else
    hipLaunchKernelGGL((k_prep_domains<Pix, 16>), dim3((dthreads + bs - 1) / bs),
                       dim3(bs), 0, st, g, img, b);
  hipLaunchKernelGGL(k_prep_flat, dim3((g.ND + bs - 1) / bs), dim3(bs), 0, st,
                     g, b);
  const long long rthreads = (long long)g.R_pad * 8;
  if (g.K == 64)
    hipLaunchKernelGGL((k_prep_ranges<Pix, 64>), dim3((rthreads + bs - 1) / bs),
                       dim3(bs), 0, st, g, img, b);
  else
    hipLaunchKernelGGL((k_prep_ranges<Pix, 16>), dim3((rthreads + bs - 1) / bs),
                       dim3(bs), 0, st, g, img, b);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_prep(const Geo &g, const void *image, const EncBufs &b,
                       hipStream_t st) {
  if (g.bits == 12) return prep_impl(g, (const uint16_t *)image, b, st);
  return prep_impl(g, (const uint8_t *)image, b, st);
}

hipError_t launch_finalize(const Geo &g, const void *image, const EncBufs &b,
                           fic_codes out, hipStream_t st) {
  const int bs = 256;
  if (g.bits == 12)
    hipLaunchKernelGGL(k_finalize<uint16_t>, dim3((g.R + bs - 1) / bs), dim3(bs),
                       0, st, g, (const uint16_t *)image, b, out);
  else
    hipLaunchKernelGGL(k_finalize<uint8_t>, dim3((g.R + bs - 1) / bs), dim3(bs),
                       0, st, g, (const uint8_t *)image, b, out);
  return hipGetLastError();
}

}  // namespace fic
