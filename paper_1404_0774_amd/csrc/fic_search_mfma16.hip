// fic_search_mfma16.hip -- the matrix-core search for 8-bit images with
// 16x16 ranges (the largest level of the quadtree partition).
//
// With K = 256 pixels the plain products no longer fit: G = sum A b reaches
// 256 * 1020 * 255 > 2^24.  Centring both operands fixes that without a
// split: with A' = A - 510 (|A'| <= 510) and b' = b - 128 (|b'| <= 128),
// every partial sum of G' = sum A' b' stays within 256 * 510 * 128 =
// 16,711,680 < 2^24, so one FP16 chain with FP32 accumulation is exact in
// any order, and
//     G = G' + 128 SA + 510 Sb - 65280 K        (K = 256)
// exactly.  The least-squares test needs G - SA Sb / K = G' - SA' Sb' / K
// (SA' = SA - 510 K, Sb' = Sb - 128 K), so the prune runs on G' directly;
// the queue carries G rebuilt exactly in FP64.  Otherwise this is the 12-bit
// kernel's organisation: one row block (4 ranges x 8 transforms) per wave,
// a per-wave LDS queue drained 64 pairs at a time, FP64 fits, packed-key
// minima in LDS and, every few blocks, in the global table.
#include <math.h>

#include "fic_search_common.h"

namespace fic {

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kWR = 4;      // ranges per wave (one row block)
constexpr int kSync = 4;    // column blocks between global syncs
constexpr int kQueue = 128; // pairs; >= 63 + 64 lanes

struct __attribute__((aligned(16))) QEntry16 {
  double g[8];  // exact G of the 8 transforms
  double saa;
  float sa, dp;
  int dom, lr;
  int pad[2];
};


// Exact-safe test of one candidate in FP64: G - SA Sb/K is exact in double,
// t = W' D' is rounded down.
__device__ __forceinline__ bool passes_exact(double G, double sa, double Sb,
                                             double invK, float t) {
  const double a = G - sa * Sb * invK;  // K is a power of two
  return a * a >= (double)t;
}

// Surviving transforms are listed as pair index << 3 | transform.
__device__ __forceinline__ void drain16(QEntry16 *queue, unsigned *cands,
                                        int &qn, int n,
                                        unsigned long long *best,
                                        const double2 *rstat, const Geo &g) {
  const int lane = threadIdx.x & 63;
  const double K = (double)g.K;
  for (int base = 0; base < n; base += 64) {
    const int i = base + lane;
    int nc = 0;
    {
      double gv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      unsigned pass = 0;
      if (i < n) {
        const QEntry16 &q = queue[i];
#pragma unroll
        for (int k = 0; k < 8; ++k) gv[k] = q.g[k];
        const double2 rs = rstat[q.lr];
        const float t =
            weight_from_key(best[q.lr], K * rs.y - rs.x * rs.x, g) * q.dp;
#pragma unroll
        for (int k = 0; k < 8; ++k)
          pass |= passes_exact(gv[k], (double)q.sa, rs.x, g.invK, t) ? (1u << k) : 0u;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const bool f = (pass >> k) & 1u;
        const unsigned long long m = __builtin_amdgcn_ballot_w64(f);
        if (f) {
          const int off = __builtin_amdgcn_mbcnt_hi(
              (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
          cands[nc + off] = ((unsigned)i << 3) | k;
        }
        nc += __popcll(m);
      }
    }
    __builtin_amdgcn_wave_barrier();
    for (int c = lane; c < nc; c += 64) {
      const unsigned pk = cands[c];
      const QEntry16 &q = queue[pk >> 3];
      const double2 rs = rstat[q.lr];
      const Fit f = fit_exact(q.g[pk & 7], (double)q.sa, q.saa, rs.x, rs.y, g);
      atomicMin(&best[q.lr], make_key(f.err, 8ll * q.dom + (pk & 7), g));
    }
    __builtin_amdgcn_wave_barrier();
  }
  const int rem = qn - n;
  static_assert(sizeof(QEntry16) == 96, "entry is six 16-byte words");
  uint4 t[6];
#pragma unroll
  for (int w = 0; w < 6; ++w) t[w] = uint4{0, 0, 0, 0};
  if (lane < rem) {
    const uint4 *src = (const uint4 *)&queue[n + lane];
#pragma unroll
    for (int w = 0; w < 6; ++w) t[w] = src[w];
  }
  __builtin_amdgcn_wave_barrier();
  if (lane < rem) {
    uint4 *dst = (uint4 *)&queue[lane];
#pragma unroll
    for (int w = 0; w < 6; ++w) dst[w] = t[w];
  }
  qn = rem;
}

// Column ci of the searched list for block cb and lane column cl (-1 past
// the list); with identity lists (ident) the entry is its own index and
// is not read.
__device__ __forceinline__ int column16(const EncBufs &b, int nD, int cb,
                                        int cl, int ident) {
  const int j = cb * 32 + cl;
  if (ident) return j < nD ? j : -1;
  return j < nD ? b.act_col[j] : -1;
}

// A 1-D grid of G workgroups over the searched lists (ranges and domains
// with variance, built by the compaction; the lengths are read on the
// device): rows of 16 searched ranges, each split into G / rows chunks of
// 32-column blocks (at least one).  Block: 4 waves of 4 ranges each.  Same
// lane layout as the 8-bit kernel: accumulator v of lane l holds transform
// v mod 8 of range 2 (l / 32) + v / 8 of the wave, for domain column
// l mod 32.
template <int K>
__global__ __launch_bounds__(256, 2) void k_search_mfma_16(Geo g, EncBufs b) {
  constexpr int KS = K / 16;
  __shared__ unsigned long long s_best[4][kWR];
  __shared__ double2 s_rstat[4][kWR];
  __shared__ int s_slot[4][kWR];
  __shared__ QEntry16 s_queue[4][kQueue];
  __shared__ unsigned s_cands[4][8 * 64];
  const int nA = __builtin_amdgcn_readfirstlane(b.n_act[0]);
  const int nD = __builtin_amdgcn_readfirstlane(b.n_act[1]);
  const int rows = (nA + 4 * kWR - 1) / (4 * kWR);
  const int ncb = (nD + 31) / 32;
  if (rows == 0 || ncb == 0) return;
  const int chunks = max(1, min((int)gridDim.x / rows, ncb));
  const int rg = blockIdx.x / chunks, chunk = blockIdx.x % chunks;
  if (rg >= rows) return;
  const int cbpc = (ncb + chunks - 1) / chunks;
  const int c0 = chunk * cbpc, c1 = min(c0 + cbpc, ncb);
  if (c0 >= c1) return;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int h = lane >> 5;
  const int cl = lane & 31;
  const int wr0 = rg * (4 * kWR) + wave * kWR;  // entries of the range list
  unsigned long long *my_best = s_best[wave];
  double2 *rstat = s_rstat[wave];
  int *slots = s_slot[wave];
  QEntry16 *queue = s_queue[wave];
  unsigned *cands = s_cands[wave];
  int qn = 0;
  const double Kd = (double)g.K;

  // the wave's range slots (-1: none), their keys and sums
  unsigned long long gsnap = ~0ull;
  int my_slot = -1;
  if (lane < kWR) {
    my_slot = wr0 + lane < nA ? b.act_slot[wr0 + lane] : -1;
    slots[lane] = my_slot;
    double sb = 0.0, sbb = 0.0;
    if (my_slot >= 0) {
      gsnap = load_best(&b.best[my_slot]);
      sb = b.rng_sb[my_slot];
      sbb = b.rng_sbb[my_slot];
    }
    my_best[lane] = gsnap;
    rstat[lane] = double2{sb, sbb};
  }
  __builtin_amdgcn_wave_barrier();

  // the range operand holds b' = b - 128 (a padding slot holds zeros)
  half8 ah[KS];
  {
    const int rho = lane & 31;
    const int gg = rho >> 3, hh = (rho >> 2) & 1, q = rho & 3;
    const int rl = 2 * hh + (gg >> 1), iso = 4 * (gg & 1) + q;
    const int sl = slots[rl];
    const _Float16 *src =
        b.aop + ((size_t)(sl >= 0 ? sl : 0) * 8 + iso) * K + 8 * h;
#pragma unroll
    for (int kk = 0; kk < KS; ++kk)
      ah[kk] = sl >= 0 ? *(const half8 *)(src + 16 * kk) : half8{};
  }

  // centred range means Sb' / K and the prune weights
  float wp[2], bbar[2];
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const double2 rs = rstat[2 * h + e];
    bbar[e] = (float)(rs.x * g.invK - 128.0);
    wp[e] = weight_from_key(my_best[2 * h + e], Kd * rs.y - rs.x * rs.x, g);
  }
  const float sa_off = 510.0f * (float)K;  // SA' = SA - 510 K

  // a column past the searched list reads column 0 and is marked flat
  // (D' = +inf), so it never passes the prune
  // the domain operand holds A' = A - 510
  half8 bh[KS];
  float csa, cdp;
  int cdom;
  double csaa;
  {
    const int ci = column16(b, nD, c0, cl, g.ident);
    const int col = ci >= 0 ? ci : 0;
    const _Float16 *bsrc =
        b.bop + (size_t)(col >> 5) * 32 * K + ((h << 5) | (col & 31)) * 8;
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) bh[kk] = *(const half8 *)(bsrc + 512 * kk);
    const float2 sadp = b.col_sadp[col];
    csa = sadp.x;
    cdp = ci >= 0 ? sadp.y : __builtin_inff();
    cdom = b.col_dom[col];
    csaa = b.col_saa[col];
  }
  // column index of the next block, read a block ahead
  int ci_next = c0 + 1 < c1 ? column16(b, nD, c0 + 1, cl, g.ident) : -1;

  for (int cb = c0; cb < c1; ++cb) {
    const int slot = (cb - c0) % kSync;
    half8 bhn[KS];
    const int ncol = ci_next >= 0 ? ci_next : 0;
    const bool nlive = ci_next >= 0;
    {
      // fragment order (bop_index): lane (h, c mod 32) of k-step kk reads
      // 16 bytes at block offset kk 1024 + 16 lane, one run per wave
      const _Float16 *bsrc =
          b.bop + (size_t)(ncol >> 5) * 32 * K + ((h << 5) | (ncol & 31)) * 8;
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) bhn[kk] = *(const half8 *)(bsrc + 512 * kk);
    }
    const float2 nsadp = b.col_sadp[ncol];
    const float nsa = nsadp.x, ndp = nlive ? nsadp.y : __builtin_inff();
    const int ndom = b.col_dom[ncol];
    const double nsaa = b.col_saa[ncol];
    // the column of the block after next, read after this block's loads so
    // that waiting for them never waits for it
    ci_next = cb + 2 < c1 ? column16(b, nD, cb + 2, cl, g.ident) : -1;

    f32x16 gp = f32x16{};
#pragma unroll
    for (int kk = 0; kk < KS; ++kk)
      gp = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[kk], bh[kk], gp, 0, 0, 0);

    // G' (exact, signed) per transform: max and min over the 8 transforms
    float gmx[2], gmn[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      float x = gp[8 * e], n = x;
#pragma unroll
      for (int k = 1; k < 8; ++k) {
        x = fmaxf(x, gp[8 * e + k]);
        n = fminf(n, gp[8 * e + k]);
      }
      gmx[e] = x;
      gmn[e] = n;
    }
    const float csac = csa - sa_off;  // SA' of the column
    bool ps[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const float a0 = fmaf(-csac, bbar[e], gmx[e]);
      const float a1 = fmaf(-csac, bbar[e], gmn[e]);
      // margin for the rounding of a (as the 12-bit kernel's)
      const float mm = fmaf(fmaxf(fabsf(a0), fabsf(a1)), 1.0f + 0x1p-20f,
                            fmaxf(fabsf(gmx[e]), fabsf(gmn[e])) * 0x1p-20f);
      ps[e] = mm * mm >= wp[e] * cdp;
    }

    if (__any(ps[0] || ps[1])) {
      bool drained = false;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const unsigned long long m = __builtin_amdgcn_ballot_w64(ps[e]);
        if (m == 0) continue;
        if (ps[e]) {
          const int off = __builtin_amdgcn_mbcnt_hi(
              (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
          QEntry16 *q = &queue[qn + off];
          // G = G' + 128 SA + 510 Sb - 65280 K, exact in FP64
          const double corr = 128.0 * (double)csa +
                              510.0 * rstat[2 * h + e].x - 65280.0 * Kd;
#pragma unroll
          for (int k = 0; k < 8; ++k) q->g[k] = (double)gp[8 * e + k] + corr;
          q->saa = csaa;
          q->sa = csa;
          q->dp = cdp;
          q->dom = cdom;
          q->lr = 2 * h + e;
        }
        qn += __popcll(m);
        if (qn >= 64) {
          drain16(queue, cands, qn, qn & ~63, my_best, rstat, g);
          drained = true;
        }
      }
      if (drained) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const double2 rs = rstat[2 * h + e];
          wp[e] = weight_from_key(my_best[2 * h + e], Kd * rs.y - rs.x * rs.x, g);
        }
      }
    }

    const int jn = cb - c0 + 1;
    if (jn == 1 || jn == 2 || slot == kSync - 1 || cb + 1 == c1) {
      if (cb + 1 == c1 && qn > 0)
        drain16(queue, cands, qn, qn, my_best, rstat, g);
      // publish, then read the global keys and use them at once
      if (lane < kWR && my_slot >= 0) {
        const unsigned long long m = my_best[lane];
        if (m < gsnap) atomicMin(&b.best[my_slot], m);
        gsnap = load_best(&b.best[my_slot]);
        my_best[lane] = min(m, gsnap);
      }
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const double2 rs = rstat[2 * h + e];
        wp[e] = weight_from_key(my_best[2 * h + e], Kd * rs.y - rs.x * rs.x, g);
      }
    }

#pragma unroll
    for (int kk = 0; kk < KS; ++kk) bh[kk] = bhn[kk];
    csa = nsa;
    cdp = ndp;
    cdom = ndom;
    csaa = nsaa;
  }
}

}  // namespace

hipError_t launch_search_mfma16(const Geo &g, const EncBufs &b,
                                int workgroups, hipStream_t st) {
  if (g.bits != 8 || g.K != 256) return hipErrorInvalidValue;
  static_assert(4 * kWR == kMfma12RangesPerWG, "row group size");
  if (workgroups < 1) workgroups = 1;
  // the kernel reads the domain operand in fragment order only
  if (!g.frag) return hipErrorInvalidValue;
  auto kern = k_search_mfma_16<256>;
  hipLaunchKernelGGL(kern, dim3(workgroups), dim3(256), 0, st, g, b);
  return hipGetLastError();
}

}  // namespace fic
