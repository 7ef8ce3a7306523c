// fic_prep.hip -- operand packing, statistics, seeding and the final code
// extraction of the range-domain search.
#include <limits.h>
#include <math.h>

#include <type_traits>

#include "fic_device.h"

namespace fic {

namespace {

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
    // 32-bit arithmetic whenever col * stride < (ND + 32) * ND fits
    d = g.ND <= 65000
            ? (int)(((unsigned)col * (unsigned)g.dom_stride) % (unsigned)g.ND)
            : (int)((col * (long long)g.dom_stride) % g.ND);
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
  SA = group_sum<N>(SA);
  SAA = group_sum<N>(SAA);
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
    b.col_flag[col] = dp != __builtin_inff() ? 1 : 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) b.flat_min[bid] = s_flat;
}

// One thread per range pixel (K threads per range slot r, one wave for
// n = 8); the slot holds image range range_of_slot(r).
// Every thread writes its pixel into the 8 rows of its range, row 8 r + k at
// position sigma_k(q), so that sum_p T[p] row[p] = sum_q T[sigma_k(q)] b[q].
// 12-bit: b = 64 b_hi + b_lo, two planes.  The range statistics are reduced
// over the K lanes (32-bit sums for 8-bit images, where every sum is below
// 2^31), and the range's best key is seeded with candidate c = 0 (domain 0,
// identity), fitted exactly.
template <typename Pix, int N>
__device__ __forceinline__ void prep_ranges_body(const Geo &g, const Pix *img,
                                                 const EncBufs &b, int bid) {
  constexpr int K = N * N;
  typedef typename std::conditional<sizeof(Pix) == 1, int, long long>::type Acc;
  const long long t = (long long)bid * blockDim.x + threadIdx.x;
  const int r = (int)(t / K), q = (int)(t % K);
  if (r >= g.R_pad) return;  // whole groups of K lanes leave together
  const int i = q / N, j = q % N, m = N - 1;
  _Float16 *row_hi = b.aop + (size_t)r * 8 * K;
  _Float16 *row_lo = b.aop + (size_t)g.R_pad * 8 * K + (size_t)r * 8 * K;
  int v = 0, A0 = 0;
  const int ri = range_of_slot(g, r);  // image range of slot r
  if (ri < g.R) {
    const int ry = ri / g.RW, rx = ri % g.RW;
    v = (int)img[(size_t)(ry * N + i) * g.W + rx * N + j];
    A0 = cell_sum(img, g.W, 2 * i, 2 * j);  // domain 0 sits at (0, 0)
  }
#pragma unroll
  for (int k = 0; k < 8 && !g.pix_a; ++k) {
    int si, sj;
    sigma(k, i, j, m, si, sj);
    const int p = si * N + sj;
    if (sizeof(Pix) == 2) {
      row_hi[k * K + p] = (_Float16)(float)(v >> 6);
      row_lo[k * K + p] = (_Float16)(float)(v & 63);
    } else {
      row_hi[k * K + p] = (_Float16)(float)v;
    }
  }
  const Acc Sb = group_sum<K>((Acc)v);
  const Acc Sbb = group_sum<K>((Acc)v * v);
  const Acc G0 = group_sum<K>((Acc)A0 * v);
  const Acc SA0 = group_sum<K>((Acc)A0);
  const Acc SAA0 = group_sum<K>((Acc)A0 * A0);
  if (q != 0) return;
  b.rng_sb[r] = (double)Sb;
  b.rng_sbb[r] = (double)Sbb;
  // searched iff a real range with variance (K Sbb - Sb^2 != 0, exact)
  b.rng_flag[r] = ri < g.R && (Acc)K * Sbb - Sb * Sb != 0 ? 1 : 0;
  if (ri >= g.R) {
    b.best[r] = ~0ull;
    return;
  }
  const Fit f0 = fit_exact((double)G0, (double)SA0, (double)SAA0, (double)Sb,
                           (double)Sbb, g);
  b.best[r] = make_key(f0.err, 0, g);
}

// One launch for both operands: workgroups [0, n_dwg) prepare domains, the
// rest prepare ranges (the two parts are independent).
template <typename Pix, int N>
__global__ __launch_bounds__(256) void k_prep(Geo g, const Pix *img,
                                              EncBufs b) {
  if ((int)blockIdx.x < g.n_dwg)
    prep_domains_body<Pix, N>(g, img, b, blockIdx.x);
  else
    prep_ranges_body<Pix, N>(g, img, b, blockIdx.x - g.n_dwg);
}

// One group of K lanes per range: unpack the winning key and recompute its
// fit from the image to produce the code (domain, transform, s index,
// o index, residual).  Flat domains (no variance) all fit a range with s = 0
// and the range mean (eqs. 11-12), so they tie and only the first of them
// can win; the search skips them and the first one is compared here.
template <typename Pix, int N>
__device__ __forceinline__ void finalize_body(const Geo &g, const Pix *img,
                                              const EncBufs &b,
                                              const fic_codes &out, int bid) {
  constexpr int K = N * N;
  __shared__ int s_wmin[8];  // per-wave minima of the flat-domain table
  const long long t = (long long)bid * blockDim.x + threadIdx.x;
  const int slot = (int)(t / K), q = (int)(t % K);
  const bool live = slot < g.R_pad;
  const int r = live ? range_of_slot(g, slot) : g.R;  // image range
  // independent loads first: the key, the range sums, the flat-domain table
  const int i = q / N, j = q % N, m = N - 1;
  unsigned long long key = ~0ull;
  double Sb0 = 0.0, Sbb0 = 0.0, v = 0.0;
  if (live && r < g.R) {
    key = b.best[slot];
    Sb0 = b.rng_sb[slot];
    Sbb0 = b.rng_sbb[slot];
    v = (double)img[(size_t)((r / g.RW) * N + i) * g.W + (r % g.RW) * N + j];
  }
  int mf = INT_MAX;
  for (int i = threadIdx.x; i < g.n_dwg; i += blockDim.x)
    mf = min(mf, b.flat_min[i]);
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) mf = min(mf, __shfl_xor(mf, o));
  if ((threadIdx.x & 63) == 0) s_wmin[threadIdx.x >> 6] = mf;
  __syncthreads();
  int ff = s_wmin[0];
  for (int wv = 1; wv < (int)(blockDim.x >> 6); ++wv) ff = min(ff, s_wmin[wv]);
  if (!live || r >= g.R) return;  // padding: whole groups of K lanes leave
  if (ff < g.ND) {
    const Fit f0 = fit_exact(0.0, 0.0, 0.0, Sb0, Sbb0, g);
    const unsigned long long kf = make_key(f0.err, 8ll * ff, g);
    key = kf < key ? kf : key;
  }
  const long long c = (long long)(key & ((1ull << g.cbits) - 1));
  const int d = (int)(c >> 3), k = (int)(c & 7);
  const int Y = (d / g.NX) * g.step, X = (d % g.NX) * g.step;
  int si, sj;
  sigma(k, i, j, m, si, sj);
  const double A = (double)cell_sum(img, g.W, Y + 2 * si, X + 2 * sj);
  // integer sums below 2^53: exact in double in any order
  const double G = group_sum<K>(A * v);
  const double SA = group_sum<K>(A);
  const double SAA = group_sum<K>(A * A);
  const double Sb = group_sum<K>(v);
  const double Sbb = group_sum<K>(v * v);
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
  const long long rwg = ((long long)g.R_pad * g.K + 255) / 256;
  const dim3 grid((unsigned)(g.n_dwg + rwg));
  if (g.n == 8)
    hipLaunchKernelGGL((k_prep<Pix, 8>), grid, dim3(256), 0, st, g, img, b);
  else
    hipLaunchKernelGGL((k_prep<Pix, 4>), grid, dim3(256), 0, st, g, img, b);
  return hipGetLastError();
}

// Ordered compaction of the indices i < n whose flag byte is 1, by one
// workgroup of 1024 threads (n a multiple of 16).  Thread t owns the
// contiguous 16-byte words [t P, (t + 1) P) of the flags and counts them
// with one popcount per word; the counts are scanned in LDS and each thread
// writes its selected indices in order.
__device__ __forceinline__ void block_compact(int n, const uint8_t *flag,
                                              int32_t *out, int32_t *count) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int words = n / 16;
  const int per = (words + 1023) / 1024;
  const int w0 = min(t * per, words), w1 = min(w0 + per, words);
  const uint4 *fw = (const uint4 *)flag;
  int c = 0;
  for (int i = w0; i < w1; ++i) {
    const uint4 v = fw[i];  // 16 flags of 0 or 1
    c += __builtin_popcount(v.x) + __builtin_popcount(v.y) +
         __builtin_popcount(v.z) + __builtin_popcount(v.w);
  }
  part[t] = c;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int pos = part[t] - c;
  for (int i = w0; i < w1; ++i) {
    const uint4 v = fw[i];
    const unsigned u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if ((u[q] >> (8 * e)) & 1u) out[pos++] = 16 * i + 4 * q + e;
  }
  if (t == 1023) *count = part[1023];
  __syncthreads();  // part is reused by the next call
}

// The search's work lists: range slots holding a range with variance and
// domain columns holding a domain with variance (flags written by the
// preparation), both in slot / sweep order.
__device__ __forceinline__ void compact_body(const Geo &g, const EncBufs &b) {
  block_compact(g.R_pad, b.rng_flag, b.act_slot, &b.n_act[0]);
  block_compact(g.NC_pad, b.col_flag, b.act_col, &b.n_act[1]);
}

__global__ __launch_bounds__(1024) void k_compact(Geo g, EncBufs b) {
  compact_body(g, b);
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

// Workgroups [0, phase_total[0]) prepare domains, the rest ranges, each
// phase laid out slice after slice.
template <typename Pix, int N>
__global__ __launch_bounds__(256) void k_prep_batch(BatchDev bd) {
  const int bid = blockIdx.x;
  const bool dom = bid < bd.phase_total[0];
  const int *off = bd.phase_off + (dom ? 0 : bd.n + 1);
  const int pb = dom ? bid : bid - bd.phase_total[0];
  const int s = slice_of(off, bd.n, pb);
  const Geo g = load_uniform(&bd.tab[s].g);
  const EncBufs b = load_uniform(&bd.tab[s].b);
  const Pix *img = (const Pix *)load_uniform(&bd.tab[s].image);
  if (dom)
    prep_domains_body<Pix, N>(g, img, b, pb - off[s]);
  else
    prep_ranges_body<Pix, N>(g, img, b, pb - off[s]);
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

// One workgroup per slice.
__global__ __launch_bounds__(1024) void k_compact_batch(BatchDev bd) {
  const Geo g = load_uniform(&bd.tab[blockIdx.x].g);
  const EncBufs b = load_uniform(&bd.tab[blockIdx.x].b);
  compact_body(g, b);
}

}  // namespace

hipError_t launch_compact(const Geo &g, const EncBufs &b, hipStream_t st) {
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, st, g, b);
  return hipGetLastError();
}

hipError_t launch_compact_batch(const BatchDev &bd, hipStream_t st) {
  hipLaunchKernelGGL(k_compact_batch, dim3(bd.n), dim3(1024), 0, st, bd);
  return hipGetLastError();
}

hipError_t launch_prep_batch(const BatchDev &bd, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_init, dim3((bd.n + 255) / 256), dim3(256), 0, st,
                     bd);
  const dim3 grid(bd.phase_total[0] + bd.phase_total[1]);
  if (bd.bits == 12) {
    if (bd.rsize == 8)
      hipLaunchKernelGGL((k_prep_batch<uint16_t, 8>), grid, dim3(256), 0, st, bd);
    else
      hipLaunchKernelGGL((k_prep_batch<uint16_t, 4>), grid, dim3(256), 0, st, bd);
  } else {
    if (bd.rsize == 8)
      hipLaunchKernelGGL((k_prep_batch<uint8_t, 8>), grid, dim3(256), 0, st, bd);
    else
      hipLaunchKernelGGL((k_prep_batch<uint8_t, 4>), grid, dim3(256), 0, st, bd);
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
  const dim3 grid((unsigned)(((long long)g.R_pad * g.K + bs - 1) / bs));
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
