// fic_finalize.h -- code extraction: the winning key of every range turned
// into its code, shared by the single-image launch and the batched search.
#pragma once

#include <limits.h>

#include "fic_block.h"
#include "fic_search_common.h"

namespace fic {

// One group of L lanes per range (L = N or K = N^2), each lane holding K / L
// consecutive pixels of the range: unpack the winning key and recompute its
// fit from the image to produce the code (domain, transform, s index, o
// index, residual).  K lanes suit one image (many short waves), N lanes a
// batch (a quarter or an eighth of the waves).  Flat domains (no variance)
// all fit a range with s = 0 and the range mean (eqs. 11-12), so they tie and
// only the first of them can win; the search never keeps one (it skips them,
// or its test rejects them) and the first one is compared here.
template <typename Pix, int N, int L>
__device__ __forceinline__ void finalize_body(const Geo &g, const Pix *img,
                                              const EncBufs &b,
                                              const fic_codes &out, int bid) {
  constexpr int P = N * N / L;  // pixels per lane
  static_assert(L == N || L == N * N, "a row or a pixel per lane");
  __shared__ int s_wmin[8];  // per-wave minima of the flat-domain table
  const long long t = (long long)bid * blockDim.x + threadIdx.x;
  const int slot = (int)(t / L), q0 = (int)(t % L) * P, m = N - 1;
  const bool live = slot < g.R_pad;
  const int r = live ? range_of_slot(g, slot) : g.R;  // image range
  // independent loads first: the key, the range sums, the flat-domain table
  unsigned long long key = ~0ull;
  double Sb0 = 0.0, Sbb0 = 0.0;
  if (live && r < g.R) {
    // an agent-scope load: the keys may have been lowered by atomics of
    // other workgroups of the same launch (the batched search)
    key = load_best(&b.best[slot]);
    Sb0 = b.rng_sb[slot];
    Sbb0 = b.rng_sbb[slot];
  }
  int mf = INT_MAX;
  for (int w = threadIdx.x; w < g.n_dwg; w += blockDim.x)
    mf = min(mf, b.flat_min[w]);
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) mf = min(mf, __shfl_xor(mf, o));
  if ((threadIdx.x & 63) == 0) s_wmin[threadIdx.x >> 6] = mf;
  __syncthreads();
  int ff = s_wmin[0];
  for (int wv = 1; wv < (int)(blockDim.x >> 6); ++wv) ff = min(ff, s_wmin[wv]);
  if (!live || r >= g.R) return;  // padding: whole groups of L lanes leave
  if (ff < g.ND) {
    const Fit f0 = fit_exact(0.0, 0.0, 0.0, Sb0, Sbb0, g);
    const unsigned long long kf = make_key(f0.err, 8ll * ff, g);
    key = kf < key ? kf : key;
  }
  const long long c = (long long)(key & ((1ull << g.cbits) - 1));
  const int d = (int)(c >> 3), k = (int)(c & 7);
  const int Y = (d / g.NX) * g.step, X = (d % g.NX) * g.step;
  // The lane takes cells (ci, cj0 ..) of the domain in natural order and
  // the range pixels they meet, sigma_k^-1 of each cell: G = sum_q
  // A[sigma_k(q)] b[q] = sum_p A[p] b[sigma_k^-1(p)].  Integer sums (below
  // 2^63 per lane and 2^53 in total): exact.
  const int ci = q0 / N, cj0 = q0 % N;
  int A[P];
  if constexpr (P == N) {
    // one cell row: two image rows, as words when they are aligned
    int p0[2 * N], p1[2 * N];
    const Pix *c0 = img + (size_t)(Y + 2 * ci) * g.W + X;
    const bool wide = domain_rows_aligned(g, img);
    load_row<Pix, N>(c0, wide, p0);
    load_row<Pix, N>(c0 + g.W, wide, p1);
#pragma unroll
    for (int e = 0; e < P; ++e)
      A[e] = p0[2 * e] + p0[2 * e + 1] + p1[2 * e] + p1[2 * e + 1];
  } else {
#pragma unroll
    for (int e = 0; e < P; ++e)
      A[e] = cell_sum(img, g.W, Y + 2 * ci, X + 2 * (cj0 + e));
  }
  const Pix *rb = img + (size_t)((r / g.RW) * N) * g.W + (r % g.RW) * N;
  long long G = 0, SA = 0, SAA = 0, Sb = 0, Sbb = 0;
#pragma unroll
  for (int e = 0; e < P; ++e) {
    int bi, bj;
    sigma_inv(k, ci, cj0 + e, m, bi, bj);
    const long long bv = (long long)rb[(size_t)bi * g.W + bj];
    G += (long long)A[e] * bv;
    SA += A[e];
    SAA += (long long)A[e] * A[e];
    Sb += bv;
    Sbb += bv * bv;
  }
  G = group_sum<L>(G);
  SA = group_sum<L>(SA);
  SAA = group_sum<L>(SAA);
  Sb = group_sum<L>(Sb);
  Sbb = group_sum<L>(Sbb);
  if (q0 != 0) return;
  const Fit f = fit_exact((double)G, (double)SA, (double)SAA, (double)Sb,
                          (double)Sbb, g);
  out.domain[r] = d;
  out.iso[r] = (uint8_t)k;
  out.s_idx[r] = (uint8_t)f.j;
  out.o_idx[r] = (uint8_t)f.m;
  out.err[r] = f.err;
}

}  // namespace fic
