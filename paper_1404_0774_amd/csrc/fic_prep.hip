// fic_prep.hip -- operand packing, statistics, seeding and the final code
// extraction of the range-domain search.
#include <limits.h>
#include <math.h>

#include <type_traits>

#include "fic_finalize.h"

namespace fic {

namespace {

// One thread per (sweep column, cell row): N threads per column, columns in
// order, so that the threads of a wave write neighbouring operand runs and
// records (the domains they read are scattered over the image, which stays
// in the L2).  Column c holds domain (c * dom_stride) mod ND; threads past
// ND fill the padding columns.  Its 2x2 cell sums A (4x the contracted value of Alg. 1)
// are written as exact FP16 integers.  12-bit images store A = 128 A_hi +
// A_lo as two planes.  Flat domains (no variance) get +inf as their prune
// denominator: they all fit any range with s = 0 and the same offset (eqs.
// 11-12), so only the first of them, seeded per range, can be kept.  Each
// workgroup records the smallest flat domain index it saw.
template <typename Pix, int N>
__device__ __forceinline__ void prep_domains_body(const Geo &g, const Pix *img,
                                                  const EncBufs &b, int bid) {
  constexpr int K = N * N;
  typedef _Float16 halfN __attribute__((ext_vector_type(N)));
  __shared__ int s_flat;
  if (threadIdx.x == 0) s_flat = INT_MAX;
  __syncthreads();
  const long long t = (long long)bid * blockDim.x + threadIdx.x;
  const long long e = t / N;  // column (sweep order), or padding e >= ND
  const int i = (int)(t % N);
  const bool live = e < g.NC_pad;
  long long col = e;
  long long SA = 0, SAA = 0;
  int d = -1;
  halfN vh, vl;
  int Av[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    vh[j] = vl[j] = (_Float16)0.0f;
    Av[j] = 0;
  }
  if (live && e < g.ND) {
    // column e holds domain (e * dom_stride) mod ND; 32-bit arithmetic
    // whenever e * dom_stride < ND^2 fits
    d = g.ND <= 65000
            ? (int)(((unsigned)e * (unsigned)g.dom_stride) % (unsigned)g.ND)
            : (int)((e * g.dom_stride) % g.ND);
    const int Y = (d / g.NX) * g.step, X = (d % g.NX) * g.step;
    const Pix *r0 = img + (size_t)(Y + 2 * i) * g.W + X;
    const bool wide = domain_rows_aligned(g, img);
    int p0[2 * N], p1[2 * N];
    load_row<Pix, N>(r0, wide, p0);
    load_row<Pix, N>(r0 + g.W, wide, p1);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int A = p0[2 * j] + p0[2 * j + 1] + p1[2 * j] + p1[2 * j + 1];
      Av[j] = A;
      SA += A;
      SAA += (long long)A * A;
      if (g.bits == 12) {
        vh[j] = (_Float16)(float)(A >> 7);
        vl[j] = (_Float16)(float)(A & 127);
      } else if (N == 16) {
        vh[j] = (_Float16)(float)(A - 510);  // centred: |A - 510| <= 510
      } else {
        vh[j] = (_Float16)(float)A;
      }
    }
  }
  // the column's statistics over its N adjacent threads
  SA = group_sum<N>(SA);
  SAA = group_sum<N>(SAA);
  if (g.ctr && N != 16) {
    // centred on the rounded mean: |A - m| <= 1020, exact in FP16
    const int m = d >= 0 ? centre_of(SA, K) : 0;
#pragma unroll
    for (int j = 0; j < N; ++j) vh[j] = (_Float16)(float)(Av[j] - m);
  }
  if (live) {
    if constexpr (N == 16) {
      // fragment order keeps runs of 8 elements together, not 16
      typedef _Float16 half8v __attribute__((ext_vector_type(8)));
      *(half8v *)(b.bop + bop_index(g, col, i * N)) =
          __builtin_shufflevector(vh, vh, 0, 1, 2, 3, 4, 5, 6, 7);
      *(half8v *)(b.bop + bop_index(g, col, i * N + 8)) =
          __builtin_shufflevector(vh, vh, 8, 9, 10, 11, 12, 13, 14, 15);
    } else {
      *(halfN *)(b.bop + bop_index(g, col, i * N)) = vh;
    }
    if (g.bits == 12)
      *(halfN *)(b.bop + (size_t)g.NC_pad * K + bop_index(g, col, i * N)) = vl;
    if (g.i8) {
      // the same pieces as int8 (both <= 127) for the int8 search
      int8_t *dh = b.bop8 + bop8_index(g, col, i * N);
      int8_t *dl = dh + (size_t)g.NC_pad * K;
#pragma unroll
      for (int j = 0; j < N; ++j) {
        dh[j] = (int8_t)(float)vh[j];
        dl[j] = (int8_t)(float)vl[j];
      }
    }
  }
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
    rec.sc = dp == __builtin_inff()
                 ? dp
                 : round_down_f(sqrt((double)K * (double)SAA -
                                     (double)SA * (double)SA));
    rec.dom = d;
    rec.saa = g.bits == 8 ? (unsigned)SAA : 0u;
    b.col_rec[col] = rec;
    // searched: a domain with variance, or any domain in a full search
    b.col_flag[col] = d >= 0 && (g.full || dp != __builtin_inff()) ? 1 : 0;
    if (g.ident) b.act_col[col] = (int)col;  // columns 0 .. ND - 1 are real
  }
  __syncthreads();
  if (threadIdx.x == 0) b.flat_min[bid] = s_flat;
}

// L lanes per range slot r (L = K = N^2: one pixel each, one wave for
// n = 8; L = N: one row each), the slot holding image range
// range_of_slot(r).  Every pixel is written into the 8 rows of its range,
// row 8 r + k at position sigma_k(q), so that sum_p T[p] row[p] =
// sum_q T[sigma_k(q)] b[q] (unless the search builds those rows from the
// pixels itself).  12-bit: b = 64 b_hi + b_lo, two planes.  The range
// statistics are reduced over the L lanes (32-bit sums for 8-bit images,
// where every sum is below 2^31), and the range's best key is seeded with
// candidate c = 0 (domain 0, identity), fitted exactly.
template <typename Pix, int N, int L>
__device__ __forceinline__ void prep_ranges_body(const Geo &g, const Pix *img,
                                                 const EncBufs &b, int bid) {
  constexpr int K = N * N, P = K / L;  // pixels per lane
  static_assert(L == N || L == K, "a row or a pixel per lane");
  typedef typename std::conditional<sizeof(Pix) == 1, int, long long>::type Acc;
  const long long t = (long long)bid * blockDim.x + threadIdx.x;
  const int r = (int)(t / L), q0 = (int)(t % L) * P, m = N - 1;
  if (r >= g.R_pad) return;  // whole groups of L lanes leave together
  const int i = q0 / N, j0 = q0 % N;  // the lane's pixels: row i, j0 ..
  _Float16 *row_hi = b.aop + (size_t)r * 8 * K;
  _Float16 *row_lo = b.aop + (size_t)g.R_pad * 8 * K + (size_t)r * 8 * K;
  int v[P], A0[P];
#pragma unroll
  for (int e = 0; e < P; ++e) v[e] = A0[e] = 0;
  const int ri = range_of_slot(g, r);  // image range of slot r
  if (ri < g.R) {
    const int ry = ri / g.RW, rx = ri % g.RW;
    const Pix *p = img + (size_t)(ry * N + i) * g.W + rx * N + j0;
    if constexpr (P == N) {
      // a range row and a cell row of domain 0 (at (0, 0)), as words when
      // the rows are aligned
      const bool wide = domain_rows_aligned(g, img);
      int p0[2 * N], p1[2 * N];
      load_run<Pix, N>(p, wide, v);
      load_row<Pix, N>(img + (size_t)(2 * i) * g.W, wide, p0);
      load_row<Pix, N>(img + (size_t)(2 * i + 1) * g.W, wide, p1);
#pragma unroll
      for (int e = 0; e < P; ++e)
        A0[e] = p0[2 * e] + p0[2 * e + 1] + p1[2 * e] + p1[2 * e + 1];
    } else {
#pragma unroll
      for (int e = 0; e < P; ++e) {
        v[e] = (int)p[e];
        A0[e] = cell_sum(img, g.W, 2 * i, 2 * (j0 + e));  // domain 0: (0, 0)
      }
    }
  }
  Acc Sb = 0, Sbb = 0, G0 = 0, SA0 = 0, SAA0 = 0;
#pragma unroll
  for (int e = 0; e < P; ++e) {
    Sb += v[e];
    Sbb += (Acc)v[e] * v[e];
    G0 += (Acc)A0[e] * v[e];
    SA0 += A0[e];
    SAA0 += (Acc)A0[e] * A0[e];
  }
  Sb = group_sum<L>(Sb);
  Sbb = group_sum<L>(Sbb);
  G0 = group_sum<L>(G0);
  SA0 = group_sum<L>(SA0);
  SAA0 = group_sum<L>(SAA0);
  if (!g.pix_a) {
    // 8-bit matrix-core operands are centred on the range's rounded mean
    const int mr = g.ctr ? centre_of((long long)Sb, K) : 0;
#pragma unroll
    for (int e = 0; e < P; ++e) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        int si, sj;
        sigma(k, i, j0 + e, m, si, sj);
        const int pp = si * N + sj;
        if (sizeof(Pix) == 2) {
          row_hi[k * K + pp] = (_Float16)(float)(v[e] >> 6);
          row_lo[k * K + pp] = (_Float16)(float)(v[e] & 63);
          if (g.i8) {
            int8_t *r8 = b.aop8 + (size_t)r * 8 * K;
            r8[k * K + pp] = (int8_t)(v[e] >> 6);
            r8[(size_t)g.R_pad * 8 * K + k * K + pp] = (int8_t)(v[e] & 63);
          }
        } else if (N == 16) {
          row_hi[k * K + pp] = (_Float16)(float)(v[e] - 128);  // centred
        } else {
          row_hi[k * K + pp] = (_Float16)(float)(v[e] - mr);
        }
      }
    }
  }
  if (q0 != 0) return;
  b.rng_sb[r] = (double)Sb;
  b.rng_sbb[r] = (double)Sbb;
  // searched: a real range with variance (K Sbb - Sb^2 != 0, exact), or
  // any real range in a full search; never one the range mask leaves out
  b.rng_flag[r] = ri < g.R && (!b.rmask || b.rmask[ri]) &&
                         (g.full || (Acc)K * Sbb - Sb * Sb != 0)
                     ? 1
                     : 0;
  if (g.ident) b.act_slot[r] = r;  // every slot holds a real range
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
  if (g.ident && blockIdx.x == 0 && threadIdx.x == 0) {
    b.n_act[0] = g.R_pad;
    b.n_act[1] = g.ND;
  }
  if ((int)blockIdx.x < g.n_dwg) {
    prep_domains_body<Pix, N>(g, img, b, blockIdx.x);
  } else if (g.pix_a || N == 16) {
    // (16x16 ranges: a row of 16 pixels per lane, 16 lanes per range)
    // a row per lane when only statistics are needed, a pixel per lane when
    // the range operand is written as well (its scattered stores spread)
    prep_ranges_body<Pix, N, N>(g, img, b, blockIdx.x - g.n_dwg);
  } else {
    if constexpr (N != 16)
      prep_ranges_body<Pix, N, N * N>(g, img, b, blockIdx.x - g.n_dwg);
  }
}

template <typename Pix, int N>
__global__ __launch_bounds__(256) void k_finalize(Geo g, const Pix *img,
                                                  EncBufs b, fic_codes out) {
  // a pixel per lane; 16x16 ranges a row per lane (a range spans 16 lanes)
  finalize_body<Pix, N, (N == 16 ? N : N * N)>(g, img, b, out, blockIdx.x);
}

template <typename Pix>
hipError_t prep_impl(const Geo &g, const Pix *img, const EncBufs &b,
                     hipStream_t st) {
  const long long lanes = (g.pix_a || g.n == 16) ? g.n : g.K;  // as k_prep
  const long long rwg = ((long long)g.R_pad * lanes + 255) / 256;
  const dim3 grid((unsigned)(g.n_dwg + rwg));
  if (g.n == 16)
    hipLaunchKernelGGL((k_prep<Pix, 16>), grid, dim3(256), 0, st, g, img, b);
  else if (g.n == 8)
    hipLaunchKernelGGL((k_prep<Pix, 8>), grid, dim3(256), 0, st, g, img, b);
  else
    hipLaunchKernelGGL((k_prep<Pix, 4>), grid, dim3(256), 0, st, g, img, b);
  return hipGetLastError();
}

// Ordered compaction of the indices whose flag byte is 1, for two flag
// arrays at once (lengths multiples of 16), by one workgroup of 1024
// threads.  Wave w owns a contiguous stretch of each array, a multiple of
// 256 flags long.  In rounds of 256 flags, lane l reads flags 4l .. 4l + 3
// as one 32-bit word; one ballot per byte position gives every set flag its
// rank (set flags in lower lanes: the sum of the four ballots' mbcnt; in the
// lane itself: the set bytes below it), so each round's stores land next to
// each other.  A first pass counts each wave's flags, the 16 totals are
// exchanged in LDS, and a second pass writes; up to 16 rounds a wave (65,536
// flags an array) the words stay in registers between the passes.
__device__ __forceinline__ unsigned flag_bits(const uint8_t *flag, int i,
                                              int end) {
  // bit e: flag i + e (i a multiple of 4, end a multiple of 16)
  const unsigned u = i < end ? *(const unsigned *)(flag + i) : 0u;
  return (u & 1u) | ((u >> 7) & 2u) | ((u >> 14) & 4u) | ((u >> 21) & 8u);
}

__device__ __forceinline__ int wave_count(const uint8_t *flag, int beg,
                                          int end, int lane) {
  int c = 0;
  for (int b = beg; b < end; b += 256)
    c += __builtin_popcount(flag_bits(flag, b + 4 * lane, end));
  // lanes hold partial counts: sum over the wave
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  return c;
}

__device__ __forceinline__ void wave_write(const uint8_t *flag, int beg,
                                           int end, int lane, int pos,
                                           int32_t *out) {
  for (int b = beg; b < end; b += 256) {
    const int i = b + 4 * lane;
    const unsigned bits = flag_bits(flag, i, end);
    int below = 0, total = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const unsigned long long m = __builtin_amdgcn_ballot_w64((bits >> e) & 1u);
      below += __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                         __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
      total += __popcll(m);
    }
    int at = pos + below;
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if ((bits >> e) & 1u) out[at++] = i + e;
    pos += total;
  }
}

// Up to R rounds a wave: every round's word is loaded at once and kept in
// registers for both passes (one trip to memory instead of two chains of
// dependent loads).
template <int R>
__device__ __forceinline__ int regs_count(const uint8_t *flag, int beg,
                                          int end, int lane,
                                          unsigned (&bits)[R]) {
  int c = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    bits[r] = flag_bits(flag, beg + 256 * r + 4 * lane, end);
    c += __builtin_popcount(bits[r]);
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  return c;
}

template <int R>
__device__ __forceinline__ void regs_write(int beg, int end, int lane,
                                           int pos, const unsigned (&bits)[R],
                                           int32_t *out) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = beg + 256 * r + 4 * lane;
    if (beg + 256 * r >= end) break;  // wave-uniform
    int below = 0, total = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const unsigned long long m =
          __builtin_amdgcn_ballot_w64((bits[r] >> e) & 1u);
      below += __builtin_amdgcn_mbcnt_hi(
          (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
      total += __popcll(m);
    }
    int at = pos + below;
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if ((bits[r] >> e) & 1u) out[at++] = i + e;
    pos += total;
  }
}

// Exclusive prefix of the 16 waves' counts (x, y) and their totals.
__device__ __forceinline__ void wave_prefix(const int2 *wtot, int wave,
                                            int &q0, int &q1, int &t0,
                                            int &t1) {
  q0 = q1 = t0 = t1 = 0;
  for (int w = 0; w < 16; ++w) {
    const int2 v = wtot[w];
    if (w < wave) {
      q0 += v.x;
      q1 += v.y;
    }
    t0 += v.x;
    t1 += v.y;
  }
}

__device__ __forceinline__ void block_compact2(int n0, const uint8_t *f0,
                                               int32_t *o0, int n1,
                                               const uint8_t *f1, int32_t *o1,
                                               int32_t *count) {
  __shared__ int2 wtot[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // each wave's stretch: whole rounds of 256 flags
  const int s0 = (n0 + 16 * 256 - 1) / (16 * 256) * 256;
  const int s1 = (n1 + 16 * 256 - 1) / (16 * 256) * 256;
  const int a0 = min(wave * s0, n0), a1 = min(a0 + s0, n0);
  const int b0 = min(wave * s1, n1), b1 = min(b0 + s1, n1);
  int q0, q1, t0, t1;
  if (s0 <= 256 * 8 && s1 <= 256 * 8) {
    // both arrays' words in registers, one exchange
    unsigned r0[8], r1[8];
    const int c0 = regs_count<8>(f0, a0, a1, lane, r0);
    const int c1 = regs_count<8>(f1, b0, b1, lane, r1);
    if (lane == 0) wtot[wave] = int2{c0, c1};
    __syncthreads();
    wave_prefix(wtot, wave, q0, q1, t0, t1);
    regs_write<8>(a0, a1, lane, q0, r0, o0);
    regs_write<8>(b0, b1, lane, q1, r1, o1);
  } else if (s0 <= 256 * 16 && s1 <= 256 * 16) {
    // one array at a time; the second exchange uses the other half of each
    // entry, so it never overwrites counts another wave may still read
    unsigned r[16];
    const int c0 = regs_count<16>(f0, a0, a1, lane, r);
    if (lane == 0) wtot[wave].x = c0;
    __syncthreads();
    wave_prefix(wtot, wave, q0, q1, t0, t1);
    regs_write<16>(a0, a1, lane, q0, r, o0);
    const int c1 = regs_count<16>(f1, b0, b1, lane, r);
    if (lane == 0) wtot[wave].y = c1;
    __syncthreads();
    wave_prefix(wtot, wave, q0, q1, t0, t1);
    regs_write<16>(b0, b1, lane, q1, r, o1);
  } else {
    const int c0 = wave_count(f0, a0, a1, lane);
    const int c1 = wave_count(f1, b0, b1, lane);
    if (lane == 0) wtot[wave] = int2{c0, c1};
    __syncthreads();
    wave_prefix(wtot, wave, q0, q1, t0, t1);
    wave_write(f0, a0, a1, lane, q0, o0);
    wave_write(f1, b0, b1, lane, q1, o1);
  }
  if (threadIdx.x == 0) {
    count[0] = t0;
    count[1] = t1;
  }
}

// The search's work lists: range slots and domain columns it visits (those
// with variance, or every real one in a full search; flags written by the
// preparation), both in slot / sweep order.
__device__ __forceinline__ void compact_body(const Geo &g, const EncBufs &b) {
  block_compact2(g.R_pad, b.rng_flag, b.act_slot, g.NC_pad, b.col_flag,
                 b.act_col, b.n_act);
}

__global__ __launch_bounds__(1024) void k_compact(Geo g, EncBufs b) {
  compact_body(g, b);
}

// Slice of workgroup `bid` in a phase with offsets off[0..n] (off[n] is the
// total): the s with off[s] <= bid < off[s + 1].
__global__ void k_batch_init(BatchDev bd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    *bd.counter = 0;
    bd.ticks[0] = ~0ull;
  }
  if (i < bd.n) {
    bd.remaining[i] = bd.items_per_slice[i];
    bd.fin_remaining[i] = bd.fin_per_slice[i];
    bd.ticks[1 + i] = 0;
  }
}

// Workgroups [0, phase_total[0]) prepare domains, the rest ranges, each
// phase laid out slice after slice.
template <typename Pix, int N>
__global__ __launch_bounds__(256) void k_prep_batch(BatchDev bd) {
  // the two phases are consecutive in the map: (slice, workgroup in slice)
  const bool dom = (int)blockIdx.x < bd.phase_total[0];
  const int2 m = load_uniform(&bd.wg_map[bd.phase_base[0] + blockIdx.x]);
  const Geo g = load_uniform(&bd.tab[m.x].g);
  const EncBufs b = load_uniform(&bd.tab[m.x].b);
  const Pix *img = (const Pix *)load_uniform(&bd.tab[m.x].image);
  if (dom)
    prep_domains_body<Pix, N>(g, img, b, m.y);
  else
    prep_ranges_body<Pix, N, N>(g, img, b, m.y);
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

hipError_t launch_prep(const Geo &g, const void *image, const EncBufs &b,
                       hipStream_t st) {
  if (g.bits == 12) return prep_impl(g, (const uint16_t *)image, b, st);
  return prep_impl(g, (const uint8_t *)image, b, st);
}

hipError_t launch_finalize(const Geo &g, const void *image, const EncBufs &b,
                           fic_codes out, hipStream_t st) {
  const int bs = 256;
  const long long lanes = g.n == 16 ? g.n : g.K;  // per range, as k_finalize
  const dim3 grid((unsigned)(((long long)g.R_pad * lanes + bs - 1) / bs));
  if (g.n == 16) {
    if (g.bits != 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_finalize<uint8_t, 16>), grid, dim3(bs), 0, st, g,
                       (const uint8_t *)image, b, out);
    return hipGetLastError();
  }
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
