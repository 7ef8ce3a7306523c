// fic_prep.hip -- operand packing, statistics, seeding and the final code
// extraction of the range-domain search.
#include <limits.h>
#include <math.h>

#include "fic_device.h"

namespace fic {

namespace {

template <typename Pix>
__device__ __forceinline__ int cell_sum(const Pix *img, int W, int y, int x) {
  const Pix *p = img + (size_t)y * W + x;
  return (int)p[0] + (int)p[1] + (int)p[W] + (int)p[W + 1];
}

// Sum over aligned groups of `width` lanes (width a power of two <= 64).
template <typename T>
__device__ __forceinline__ T group_sum(T v, int width) {
  for (int o = 1; o < width; o <<= 1) v += __shfl_xor(v, o, width);
  return v;
}

// One thread per (column, cell row): N threads per column.  Column c of the
// sweep holds domain d = (c * dom_stride) mod ND; its 2x2 cell sums A (4x the
// contracted value of Alg. 1) are written as exact FP16 integers.  12-bit
// images store A = 128 A_hi + A_lo as two planes.  Flat domains (no
// variance) get +inf as their prune denominator: they all fit any range with
// s = 0 and the same offset (eqs. 11-12), so only the first of them, seeded
// per range, can be kept.  Each workgroup records the smallest flat domain
// index it saw.
template <typename Pix, int N>
__device__ __forceinline__ void prep_domains_body(const Geo &g, const Pix *img,
                                                  const EncBufs &b, int bid) {
  constexpr int K = N * N;
  typedef _Float16 halfN __attribute__((ext_vector_type(N)));
  __shared__ int s_flat;
  if (threadIdx.x == 0) s_flat = INT_MAX;
  __syncthreads();
  const long long t = (long long)bid * blockDim.x + threadIdx.x;
  const long long col = t / N;
  const int i = (int)(t % N);
  const bool live = col < g.NC_pad;
  long long SA = 0, SAA = 0;
  int d = -1;
  halfN vh, vl;
#pragma unroll
  for (int j = 0; j < N; ++j) vh[j] = vl[j] = (_Float16)0.0f;
  if (live && col < g.ND) {
    d = (int)((col * (long long)g.dom_stride) % g.ND);
    const int Y = (d / g.NX) * g.step, X = (d % g.NX) * g.step;
    const Pix *r0 = img + (size_t)(Y + 2 * i) * g.W + X;
    const Pix *r1 = r0 + g.W;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int A = (int)r0[2 * j] + (int)r0[2 * j + 1] + (int)r1[2 * j] +
                    (int)r1[2 * j + 1];
      SA += A;
      SAA += (long long)A * A;
      if (g.bits == 12) {
        vh[j] = (_Float16)(float)(A >> 7);
        vl[j] = (_Float16)(float)(A & 127);
      } else {
        vh[j] = (_Float16)(float)A;
      }
    }
  }
  if (live) {
    *(halfN *)(b.bop + (size_t)col * K + i * N) = vh;
    if (g.bits == 12)
      *(halfN *)(b.bop + (size_t)g.NC_pad * K + (size_t)col * K + i * N) = vl;
  }
  // the column's statistics over its N adjacent threads
  SA = group_sum(SA, N);
  SAA = group_sum(SAA, N);
  if (live && i == 0) {
    b.col_dom[col] = d;
    b.col_saa[col] = (double)SAA;
    float dp = __builtin_inff();
    if (d >= 0) {
      const double Dp = (double)K * (double)SAA - (double)SA * (double)SA;
      if (Dp == 0.0)
        atomicMin(&s_flat, d);
      else
        dp = round_down_f(Dp);
    }
    b.col_sadp[col] = float2{(float)SA, dp};
    ColRec rec;
    rec.sa = (float)SA;
    rec.dp = dp;
    rec.dom = d;
    rec.saa = g.bits == 8 ? (unsigned)SAA : 0u;
    b.col_rec[col] = rec;
  }
  __syncthreads();
  if (threadIdx.x == 0) b.flat_min[bid] = s_flat;
}

template <typename Pix, int N>
__global__ __launch_bounds__(256) void k_prep_domains(Geo g, const Pix *img,
                                                      EncBufs b) {
  prep_domains_body<Pix, N>(g, img, b, blockIdx.x);
}

// One thread per range pixel (K threads per range, one wave for n = 8).
// Every thread writes its pixel into the 8 rows of its range, row 8 r + k at
// position sigma_k(q), so that sum_p T[p] row[p] = sum_q T[sigma_k(q)] b[q].
// 12-bit: b = 64 b_hi + b_lo, two planes.  The range statistics are reduced
// over the K lanes, and the range's best key is seeded with the better of
// candidate c = 0 (domain 0, identity) and the first flat domain, both
// fitted exactly.
template <typename Pix, int N>
__device__ __forceinline__ void prep_ranges_body(const Geo &g, const Pix *img,
                                                 const EncBufs &b, int bid) {
  constexpr int K = N * N;
  // smallest flat domain over the domain-preparation workgroups
  __shared__ int s_ff;
  if (threadIdx.x == 0) s_ff = INT_MAX;
  __syncthreads();
  {
    int m = INT_MAX;
    for (int i = threadIdx.x; i < g.n_dwg; i += blockDim.x)
      m = min(m, b.flat_min[i]);
    atomicMin(&s_ff, m);
  }
  __syncthreads();
  const int ff = s_ff;
  const long long t = (long long)bid * blockDim.x + threadIdx.x;
  const int r = (int)(t / K), q = (int)(t % K);
  if (r >= g.R_pad) return;  // whole groups of K lanes leave together
  const int i = q / N, j = q % N, m = N - 1;
  _Float16 *row_hi = b.aop + (size_t)r * 8 * K;
  _Float16 *row_lo = b.aop + (size_t)g.R_pad * 8 * K + (size_t)r * 8 * K;
  int v = 0;
  long long A0 = 0;
  if (r < g.R) {
    const int ry = r / g.RW, rx = r % g.RW;
    v = (int)img[(size_t)(ry * N + i) * g.W + rx * N + j];
    A0 = cell_sum(img, g.W, 2 * i, 2 * j);  // domain 0 sits at (0, 0)
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    int si, sj;
    sigma(k, i, j, m, si, sj);
    const int p = si * N + sj;
    if (g.bits == 12) {
      row_hi[k * K + p] = (_Float16)(float)(v >> 6);
      row_lo[k * K + p] = (_Float16)(float)(v & 63);
    } else {
      row_hi[k * K + p] = (_Float16)(float)v;
    }
  }
  const long long Sb = group_sum((long long)v, K);
  const long long Sbb = group_sum((long long)v * v, K);
  const long long G0 = group_sum(A0 * v, K);
  const long long SA0 = group_sum(A0, K);
  const long long SAA0 = group_sum(A0 * A0, K);
  if (q != 0) return;
  b.rng_sb[r] = (double)Sb;
  b.rng_sbb[r] = (double)Sbb;
  if (r >= g.R) {
    b.best[r] = ~0ull;
    return;
  }
  const Fit f0 = fit_exact((double)G0, (double)SA0, (double)SAA0, (double)Sb,
                           (double)Sbb, g);
  unsigned long long key = make_key(f0.err, 0, g);
  if (ff < g.ND) {
    // a flat domain has A = const, so G = SA * Sb / K, N' = 0, s = 0
    const double SAf = 0.0;  // any constant domain gives the same fit
    const Fit f1 = fit_exact(0.0, SAf, 0.0, (double)Sb, (double)Sbb, g);
    const unsigned long long k1 = make_key(f1.err, 8ll * ff, g);
    if (k1 < key) key = k1;
  }
  b.best[r] = key;
}

template <typename Pix, int N>
__global__ __launch_bounds__(256) void k_prep_ranges(Geo g, const Pix *img,
                                                     EncBufs b) {
  prep_ranges_body<Pix, N>(g, img, b, blockIdx.x);
}

// One group of K lanes per range: unpack the winning key and recompute its
// fit from the image to produce the code (domain, transform, s index,
// o index, residual).
template <typename Pix, int N>
__device__ __forceinline__ void finalize_body(const Geo &g, const Pix *img,
                                              const EncBufs &b,
                                              const fic_codes &out, int bid) {
  constexpr int K = N * N;
  const long long t = (long long)bid * blockDim.x + threadIdx.x;
  const int r = (int)(t / K), q = (int)(t % K);
  if (r >= g.R) return;  // whole groups leave together (R_pad >= R)
  const unsigned long long key = b.best[r];
  const long long c = (long long)(key & ((1ull << g.cbits) - 1));
  const int d = (int)(c >> 3), k = (int)(c & 7);
  const int i = q / N, j = q % N, m = N - 1;
  const int ry = r / g.RW, rx = r % g.RW;
  const int Y = (d / g.NX) * g.step, X = (d % g.NX) * g.step;
  int si, sj;
  sigma(k, i, j, m, si, sj);
  const double v = (double)img[(size_t)(ry * N + i) * g.W + rx * N + j];
  const double A = (double)cell_sum(img, g.W, Y + 2 * si, X + 2 * sj);
  // integer sums below 2^53: exact in double in any order
  const double G = group_sum(A * v, K);
  const double SA = group_sum(A, K);
  const double SAA = group_sum(A * A, K);
  const double Sb = group_sum(v, K);
  const double Sbb = group_sum(v * v, K);
  if (q != 0) return;
  const Fit f = fit_exact(G, SA, SAA, Sb, Sbb, g);
  out.domain[r] = d;
  out.iso[r] = (uint8_t)k;
  out.s_idx[r] = (uint8_t)f.j;
  out.o_idx[r] = (uint8_t)f.m;
  out.err[r] = f.err;
}

template <typename Pix, int N>
__global__ __launch_bounds__(256) void k_finalize(Geo g, const Pix *img,
                                                  EncBufs b, fic_codes out) {
  finalize_body<Pix, N>(g, img, b, out, blockIdx.x);
}

template <typename Pix>
hipError_t prep_impl(const Geo &g, const Pix *img, const EncBufs &b,
                     hipStream_t st) {
  const int bs = 256;
  if (g.n == 8)
    hipLaunchKernelGGL((k_prep_domains<Pix, 8>), dim3(g.n_dwg), dim3(bs), 0, st,
                       g, img, b);
  else
    hipLaunchKernelGGL((k_prep_domains<Pix, 4>), dim3(g.n_dwg), dim3(bs), 0, st,
                       g, img, b);
  const dim3 rgrid((unsigned)(((long long)g.R_pad * g.K + bs - 1) / bs));
  if (g.n == 8)
    hipLaunchKernelGGL((k_prep_ranges<Pix, 8>), rgrid, dim3(bs), 0, st, g, img,
                       b);
  else
    hipLaunchKernelGGL((k_prep_ranges<Pix, 4>), rgrid, dim3(bs), 0, st, g, img,
                       b);
  return hipGetLastError();
}

// Slice of workgroup `bid` in a phase with offsets off[0..n] (off[n] is the
// total): the s with off[s] <= bid < off[s + 1].
__device__ __forceinline__ int slice_of(const int *off, int n, int bid) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= bid)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__global__ void k_batch_init(BatchDev bd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    *bd.counter = 0;
    bd.ticks[0] = ~0ull;
  }
  if (i < bd.n) {
    bd.remaining[i] = bd.items_per_slice[i];
    bd.ticks[1 + i] = 0;
  }
}

template <typename Pix, int N>
__global__ __launch_bounds__(256) void k_prep_domains_batch(BatchDev bd) {
  const int s = slice_of(bd.phase_off, bd.n, blockIdx.x);
  const Geo g = load_uniform(&bd.tab[s].g);
  const EncBufs b = load_uniform(&bd.tab[s].b);
  prep_domains_body<Pix, N>(g, (const Pix *)bd.tab[s].image, b,
                            blockIdx.x - bd.phase_off[s]);
}

template <typename Pix, int N>
__global__ __launch_bounds__(256) void k_prep_ranges_batch(BatchDev bd) {
  const int *off = bd.phase_off + (bd.n + 1);
  const int s = slice_of(off, bd.n, blockIdx.x);
  const Geo g = load_uniform(&bd.tab[s].g);
  const EncBufs b = load_uniform(&bd.tab[s].b);
  prep_ranges_body<Pix, N>(g, (const Pix *)bd.tab[s].image, b,
                           blockIdx.x - off[s]);
}

template <typename Pix, int N>
__global__ __launch_bounds__(256) void k_finalize_batch(BatchDev bd) {
  const int *off = bd.phase_off + 3 * (bd.n + 1);
  const int s = slice_of(off, bd.n, blockIdx.x);
  const Geo g = load_uniform(&bd.tab[s].g);
  const EncBufs b = load_uniform(&bd.tab[s].b);
  const fic_codes out = load_uniform(&bd.tab[s].out);
  finalize_body<Pix, N>(g, (const Pix *)bd.tab[s].image, b, out,
                        blockIdx.x - off[s]);
}

}  // namespace

hipError_t launch_prep_batch(const BatchDev &bd, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_init, dim3((bd.n + 255) / 256), dim3(256), 0, st,
                     bd);
  if (bd.bits == 12) {
    if (bd.rsize == 8) {
      hipLaunchKernelGGL((k_prep_domains_batch<uint16_t, 8>), dim3(bd.phase_total[0]), dim3(256), 0, st, bd);
      hipLaunchKernelGGL((k_prep_ranges_batch<uint16_t, 8>), dim3(bd.phase_total[1]), dim3(256), 0, st, bd);
    } else {
      hipLaunchKernelGGL((k_prep_domains_batch<uint16_t, 4>), dim3(bd.phase_total[0]), dim3(256), 0, st, bd);
      hipLaunchKernelGGL((k_prep_ranges_batch<uint16_t, 4>), dim3(bd.phase_total[1]), dim3(256), 0, st, bd);
    }
  } else {
    if (bd.rsize == 8) {
      hipLaunchKernelGGL((k_prep_domains_batch<uint8_t, 8>), dim3(bd.phase_total[0]), dim3(256), 0, st, bd);
      hipLaunchKernelGGL((k_prep_ranges_batch<uint8_t, 8>), dim3(bd.phase_total[1]), dim3(256), 0, st, bd);
    } else {
      hipLaunchKernelGGL((k_prep_domains_batch<uint8_t, 4>), dim3(bd.phase_total[0]), dim3(256), 0, st, bd);
      hipLaunchKernelGGL((k_prep_ranges_batch<uint8_t, 4>), dim3(bd.phase_total[1]), dim3(256), 0, st, bd);
    }
  }
  return hipGetLastError();
}

hipError_t launch_finalize_batch(const BatchDev &bd, hipStream_t st) {
  const dim3 grid(bd.phase_total[3]);
  if (bd.bits == 12) {
    if (bd.rsize == 8)
      hipLaunchKernelGGL((k_finalize_batch<uint16_t, 8>), grid, dim3(256), 0, st, bd);
    else
      hipLaunchKernelGGL((k_finalize_batch<uint16_t, 4>), grid, dim3(256), 0, st, bd);
  } else {
    if (bd.rsize == 8)
      hipLaunchKernelGGL((k_finalize_batch<uint8_t, 8>), grid, dim3(256), 0, st, bd);
    else
      hipLaunchKernelGGL((k_finalize_batch<uint8_t, 4>), grid, dim3(256), 0, st, bd);
  }
  return hipGetLastError();
}

hipError_t launch_prep(const Geo &g, const void *image, const EncBufs &b,
                       hipStream_t st) {
  if (g.bits == 12) return prep_impl(g, (const uint16_t *)image, b, st);
  return prep_impl(g, (const uint8_t *)image, b, st);
}

hipError_t launch_finalize(const Geo &g, const void *image, const EncBufs &b,
                           fic_codes out, hipStream_t st) {
  const int bs = 256;
  const dim3 grid((unsigned)(((long long)g.R * g.K + bs - 1) / bs));
  if (g.bits == 12) {
    if (g.n == 8)
      hipLaunchKernelGGL((k_finalize<uint16_t, 8>), grid, dim3(bs), 0, st, g,
                         (const uint16_t *)image, b, out);
    else
      hipLaunchKernelGGL((k_finalize<uint16_t, 4>), grid, dim3(bs), 0, st, g,
                         (const uint16_t *)image, b, out);
  } else {
    if (g.n == 8)
      hipLaunchKernelGGL((k_finalize<uint8_t, 8>), grid, dim3(bs), 0, st, g,
                         (const uint8_t *)image, b, out);
    else
      hipLaunchKernelGGL((k_finalize<uint8_t, 4>), grid, dim3(bs), 0, st, g,
                         (const uint8_t *)image, b, out);
  }
  return hipGetLastError();
}

}  // namespace fic
