// fic_search_mfma12.hip -- the matrix-core search for 12-bit images.
//
// 12-bit pixels (<= 4095) and their 2x2 cell sums (<= 16380) are not exact in
// FP16, so both operands are split: b = 64 b_hi + b_lo (6 + 6 bits) and
// A = 128 A_hi + A_lo (7 + 7 bits).  Then
//     G = sum A b = 8192 G_hh + 64 M + G_ll,
//     G_hh = sum A_hi b_hi,  G_ll = sum A_lo b_lo,
//     M    = sum (A_hi * 2 b_lo + A_lo * b_hi),
// where every partial sum is an integer below 64 * 127 * 189 < 2^24, so three
// FP16 MFMA chains with FP32 accumulation give the three partials exactly
// (M runs over K' = 2K products).  The factor 2 is applied once to the
// resident b_lo fragment (exact: values <= 126), not to the streamed operand.
//
// The prune uses G rebuilt in FP32 (rounding error below 2^-22 G) with a
// matching margin; queued pairs carry G exactly (an integer below 2^32), and
// drains test and fit in FP64.  One row block (4 ranges x 8 transforms) per
// wave; the domain operand's two planes are read in fragment order
// (bop_index), into two register buffers in turn.
#include <math.h>

#include "fic_search_common.h"

namespace fic {

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kWR = 4;      // ranges per wave (one row block)
constexpr int kSync = 4;    // column blocks between global syncs
constexpr int kQueue = 128; // pairs; >= 63 + 64 lanes

struct __attribute__((aligned(16))) QEntry12 {
  unsigned g[8];  // exact G of the 8 transforms (G <= 64 16380 4095 < 2^32)
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
__device__ __forceinline__ void drain12(QEntry12 *queue, unsigned *cands,
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
        const QEntry12 &q = queue[i];
#pragma unroll
        for (int k = 0; k < 8; ++k) gv[k] = (double)q.g[k];
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
      const QEntry12 &q = queue[pk >> 3];
      const double2 rs = rstat[q.lr];
      const Fit f = fit_exact((double)q.g[pk & 7], (double)q.sa, q.saa, rs.x, rs.y, g);
      atomicMin(&best[q.lr], make_key(f.err, 8ll * q.dom + (pk & 7), g));
    }
    __builtin_amdgcn_wave_barrier();
  }
  const int rem = qn - n;
  static_assert(sizeof(QEntry12) == 64, "entry is four 16-byte words");
  uint4 t[4];
#pragma unroll
  for (int w = 0; w < 4; ++w) t[w] = uint4{0, 0, 0, 0};
  if (lane < rem) {
    const uint4 *src = (const uint4 *)&queue[n + lane];
#pragma unroll
    for (int w = 0; w < 4; ++w) t[w] = src[w];
  }
  __builtin_amdgcn_wave_barrier();
  if (lane < rem) {
    uint4 *dst = (uint4 *)&queue[lane];
#pragma unroll
    for (int w = 0; w < 4; ++w) dst[w] = t[w];
  }
  qn = rem;
}

// Column ci of the searched list for block cb and lane column cl (-1 past
// the list); with identity lists (ident) the entry is its own index and
// is not read.
__device__ __forceinline__ int column12(const EncBufs &b, int nD, int cb,
                                        int cl, int ident) {
  const int j = cb * 32 + cl;
  if (ident) return j < nD ? j : -1;
  return j < nD ? b.act_col[j] : -1;
}

// A 1-D grid of G workgroups over the searched lists (ranges and domains
// with variance, built by the compaction; the lengths are read on the
// device): rows of 16 searched ranges, each split into G / (R_pad / 16)
// chunks of 32-column blocks (between one and the number of blocks); with
// fewer searched rows than R_pad / 16 the workgroups left over return.  Block: 4 waves of 4 ranges each.  Same
// lane layout as the 8-bit kernel: accumulator v of lane l holds transform
// v mod 8 of range 2 (l / 32) + v / 8 of the wave, for domain column
// l mod 32.
template <int K, bool FRAG>
__global__ __launch_bounds__(256, 2) void k_search_mfma_12(Geo g, EncBufs b) {
  constexpr int KS = K / 16;
  __shared__ unsigned long long s_best[4][kWR];
  __shared__ double2 s_rstat[4][kWR];
  __shared__ int s_slot[4][kWR];
  __shared__ QEntry12 s_queue[4][kQueue];
  __shared__ unsigned s_cands[4][8 * 64];
  const int nA = __builtin_amdgcn_readfirstlane(b.n_act[0]);
  const int nD = __builtin_amdgcn_readfirstlane(b.n_act[1]);
  const int rows = (nA + 4 * kWR - 1) / (4 * kWR);
  const int ncb = (nD + 31) / 32;
  if (rows == 0 || ncb == 0) return;
  // G / (R_pad / 16) chunks per row (the launch's col_chunks): rows of
  // searched ranges do not take more, the workgroups left over return
  const int cmax = max(1, (int)gridDim.x / max(1, g.R_pad / (4 * kWR)));
  const int chunks = max(1, min(min((int)gridDim.x / rows, cmax), ncb));
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
  QEntry12 *queue = s_queue[wave];
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

  const size_t aplane = (size_t)g.R_pad * 8 * K;
  const size_t bplane = (size_t)g.NC_pad * K;
  half8 ah[KS], al[KS], al2[KS];  // al2 = 2 b_lo
  {
    const int rho = lane & 31;
    const int gg = rho >> 3, hh = (rho >> 2) & 1, q = rho & 3;
    const int rl = 2 * hh + (gg >> 1), iso = 4 * (gg & 1) + q;
    const int sl = slots[rl];
    const _Float16 *src =
        b.aop + ((size_t)(sl >= 0 ? sl : 0) * 8 + iso) * K + 8 * h;
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      ah[kk] = sl >= 0 ? *(const half8 *)(src + 16 * kk) : half8{};
      al[kk] = sl >= 0 ? *(const half8 *)(src + aplane + 16 * kk) : half8{};
      al2[kk] = al[kk] + al[kk];
    }
  }

  float wp[2], bbar[2];
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const double2 rs = rstat[2 * h + e];
    bbar[e] = (float)(rs.x * g.invK);
    wp[e] = weight_from_key(my_best[2 * h + e], Kd * rs.y - rs.x * rs.x, g);
  }

  // A column past the searched list reads column 0 and is marked flat
  // (D' = +inf), so it never passes the prune.
  struct Col12 {
    float sa, dp;
    int dom;
    double saa;
  };
  // FRAG: the operand planes are in fragment order (a full search), where
  // lane (h, c mod 32) of k-step kk reads 16 bytes at block offset
  // kk 1024 + 16 lane, one contiguous run per wave and k-step
  auto load_col = [&](int ci, half8 (&hh)[KS], half8 (&ll)[KS], Col12 &c) {
    const int col = ci >= 0 ? ci : 0;
    const _Float16 *bsrc =
        FRAG ? b.bop + (size_t)(col >> 5) * 32 * K + ((h << 5) | (col & 31)) * 8
             : b.bop + (size_t)col * K + 8 * h;
    constexpr int kstep = FRAG ? 512 : 16;
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      hh[kk] = *(const half8 *)(bsrc + kstep * kk);
      ll[kk] = *(const half8 *)(bsrc + bplane + kstep * kk);
    }
    const float2 sadp = b.col_sadp[col];
    c.sa = sadp.x;
    c.dp = ci >= 0 ? sadp.y : __builtin_inff();
    c.dom = b.col_dom[col];
    c.saa = b.col_saa[col];
  };
  // two operand buffers: a block reads one while the next block's column
  // streams into the other (no register copies, so no wait for the loads
  // within the block that issued them)
  half8 bhA[KS], blA[KS], bhB[KS], blB[KS];
  Col12 colA, colB;
  load_col(column12(b, nD, c0, cl, g.ident), bhA, blA, colA);
  // column index of the next block, read a block ahead
  int ci_next = c0 + 1 < c1 ? column12(b, nD, c0 + 1, cl, g.ident) : -1;

  auto block = [&](int cb, const half8 (&bh)[KS], const half8 (&bl)[KS],
                   const Col12 &cc, half8 (&bhn)[KS], half8 (&bln)[KS],
                   Col12 &nc) {
    const int slot = (cb - c0) % kSync;
    load_col(ci_next, bhn, bln, nc);
    // the column of the block after next, read after this block's loads so
    // that waiting for them never waits for it
    ci_next = cb + 2 < c1 ? column12(b, nD, cb + 2, cl, g.ident) : -1;
    const float csa = cc.sa, cdp = cc.dp;
    const int cdom = cc.dom;
    const double csaa = cc.saa;

    f32x16 ghh = f32x16{}, gmid = f32x16{}, gll = f32x16{};
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      ghh = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[kk], bh[kk], ghh, 0, 0, 0);
      gll = __builtin_amdgcn_mfma_f32_32x32x16_f16(al[kk], bl[kk], gll, 0, 0, 0);
      gmid = __builtin_amdgcn_mfma_f32_32x32x16_f16(al2[kk], bh[kk], gmid, 0, 0, 0);
      gmid = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[kk], bl[kk], gmid, 0, 0, 0);
    }

    // G in FP32 (non-negative), max/min over the 8 transforms on bit patterns
    f32x16 gap;
#pragma unroll
    for (int v = 0; v < 16; ++v)
      gap[v] = fmaf(8192.0f, ghh[v], fmaf(64.0f, gmid[v], gll[v]));
    float gmx[2], gmn[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      unsigned ux = __float_as_uint(gap[8 * e]), un = ux;
#pragma unroll
      for (int k = 1; k < 8; ++k) {
        const unsigned u = __float_as_uint(gap[8 * e + k]);
        ux = max(ux, u);
        un = min(un, u);
      }
      gmx[e] = __uint_as_float(ux);
      gmn[e] = __uint_as_float(un);
    }
    bool ps[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const float a0 = fmaf(-csa, bbar[e], gmx[e]);
      const float a1 = fmaf(-csa, bbar[e], gmn[e]);
      // margin for the FP32 rebuild of G and the rounding of a
      const float mm = fmaf(fmaxf(fabsf(a0), fabsf(a1)), 1.0f + 0x1p-20f,
                            gmx[e] * 0x1p-20f);
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
          QEntry12 *q = &queue[qn + off];
#pragma unroll
          for (int k = 0; k < 8; ++k)
            q->g[k] = (unsigned)fma(8192.0, (double)ghh[8 * e + k],
                                    fma(64.0, (double)gmid[8 * e + k],
                                        (double)gll[8 * e + k]));
          q->saa = csaa;
          q->sa = csa;
          q->dp = cdp;
          q->dom = cdom;
          q->lr = 2 * h + e;
        }
        qn += __popcll(m);
        if (qn >= 64) {
          drain12(queue, cands, qn, qn & ~63, my_best, rstat, g);
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
        drain12(queue, cands, qn, qn, my_best, rstat, g);
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
  };
  for (int cb = c0; cb < c1; cb += 2) {
    block(cb, bhA, blA, colA, bhB, blB, colB);
    if (cb + 1 < c1) block(cb + 1, bhB, blB, colB, bhA, blA, colA);
  }
}

}  // namespace

hipError_t launch_search_mfma12(const Geo &g, const EncBufs &b,
                                int workgroups, hipStream_t st) {
  if (g.bits != 12) return hipErrorInvalidValue;
  static_assert(4 * kWR == kMfma12RangesPerWG, "row group size");
  if (workgroups < 1) workgroups = 1;
  auto kern = g.K == 64 ? (g.frag ? k_search_mfma_12<64, true>
                                  : k_search_mfma_12<64, false>)
                        : (g.frag ? k_search_mfma_12<16, true>
                                  : k_search_mfma_12<16, false>);
  hipLaunchKernelGGL(kern, dim3(workgroups), dim3(256), 0, st, g, b);
  return hipGetLastError();
}

}  // namespace fic
