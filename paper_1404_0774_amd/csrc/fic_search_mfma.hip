// fic_search_mfma.hip -- the range-domain search of Alg. 2/3 as a matrix-core
// contraction on CDNA4 (gfx950).
//
// For a range r, a domain d and a transform k the least-squares fit needs one
// range-specific inner product, G = sum_q A_d[sigma_k(q)] b_r[q] (the other
// sums of eqs. 9-10 are per-range or per-domain constants).  Putting the
// eight transforms on the range side (row 8 r + k of the range operand holds
// b_r scattered by sigma_k), all G form one product
//       G[(r, k), d] = sum_p Rop[(r, k), p] * Bop[d, p]
// of an (8 R) x K by K x ND pair of integer matrices.  Pixels (<= 255) and
// 2x2 cell sums (<= 1020) are exact in FP16 and every partial sum stays below
// 2^24, so v_mfma_f32_32x32x16_f16 with FP32 accumulation produces G exactly.
//
// The output is never stored.  Each 32x32 MFMA tile holds, per lane, one
// domain column and the 8 transforms of two ranges (the row order of the
// range operand is chosen for that), and the epilogue prunes with an
// exact-safe least-squares bound shared by the 8 transforms: a candidate can
// only tie or beat the range's best residual if
//       (G - SA Sb / K)^2 >= W' D'.
// Pairs that pass are appended, with their 8 G values and the column's
// statistics, to a per-wave LDS queue; 64 at a time they are re-tested per
// transform, the surviving transforms are compacted into a list and fitted
// exactly in FP64, one per lane.
// The resulting packed (residual, candidate) keys are folded into a per-wave
// LDS table (ds_min) and, every few column blocks, into the global table
// with a 64-bit atomic min.  Keys order (residual, candidate)
// lexicographically, so the result does not depend on the order of the work.
#include <math.h>

#include "fic_device.h"

namespace fic {

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kRB = 4;              // row blocks (4 ranges each) per wave
constexpr int kSlots = 2 * kRB;     // ranges per lane
constexpr int kWaveRanges = 4 * kRB;
constexpr int kSync = 4;            // column blocks between global syncs
constexpr int kQueue = 128;         // pairs; >= 63 + 64 lanes

// A queued (range, domain) pair: the 8 transforms' G, the column's
// statistics and the wave-local range index.
struct __attribute__((aligned(16))) QEntry {
  float4 g0, g1;
  double saa;
  float sa, dp;
  int dom, lr;
};

// A surviving transform of a queued pair: G, and pair index << 3 | k.
struct Cand {
  float g;
  unsigned pk;
};

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
  const double Wd = fma(-K / g.escale, (double)(key >> g.cbits), V);
  const float w = (float)(fmax(Wd, 0.0) * (1.0 / (K * K))) * (1.0f - 0x1p-20f);
  return V == 0.0 ? __builtin_inff() : w;
}

// The least-squares test shared by the 8 transforms of one (range, domain)
// pair: max_k |G_k - SA Sb/K| >= sqrt(W' D').
__device__ __forceinline__ bool pair_passes(float gmx, float gmn, float csa,
                                            float bbar, float wp, float cdp) {
  const float a0 = fmaf(-csa, bbar, gmx);
  const float a1 = fmaf(-csa, bbar, gmn);
  const float mm = fmaxf(fabsf(a0), fabsf(a1));
  return mm * mm >= wp * cdp;
}

__device__ __forceinline__ void refresh_weights(float *wp,
                                                const unsigned long long *best,
                                                const double2 *rstat, int h,
                                                const Geo &g) {
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    const int lr = 4 * (s >> 1) + 2 * h + (s & 1);
    const double2 rs = rstat[lr];
    wp[s] = weight_from_key(best[lr], (double)g.K * rs.y - rs.x * rs.x, g);
  }
}

// Process the first n queued pairs (64 per round, one per lane): re-test
// each transform with the range's current weight, compact the survivors into
// `cands` and fit them exactly, one per lane, folding their keys into the
// wave's best table.  The remaining qn - n pairs (fewer than 64) move to the
// front of the queue.
__device__ __forceinline__ void drain(QEntry *queue, Cand *cands, int &qn,
                                      int n, unsigned long long *best,
                                      const double2 *rstat, const Geo &g) {
  const int lane = threadIdx.x & 63;
  const double K = (double)g.K;
  for (int base = 0; base < n; base += 64) {
    const int i = base + lane;
    int nc = 0;
    {
      float gv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      unsigned pass = 0;
      if (i < n) {
        const QEntry &q = queue[i];
        const float4 g0 = q.g0, g1 = q.g1;
        gv[0] = g0.x; gv[1] = g0.y; gv[2] = g0.z; gv[3] = g0.w;
        gv[4] = g1.x; gv[5] = g1.y; gv[6] = g1.z; gv[7] = g1.w;
        const float sa = q.sa, dp = q.dp;
        const int lr = q.lr;
        const double2 rs = rstat[lr];
        const float bbar = (float)(rs.x / K);
        const float t = weight_from_key(best[lr], K * rs.y - rs.x * rs.x, g) * dp;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const float a = fmaf(-sa, bbar, gv[k]);
          pass |= (a * a >= t) ? (1u << k) : 0u;
        }
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const bool f = (pass >> k) & 1u;
        const unsigned long long m = __builtin_amdgcn_ballot_w64(f);
        if (f) {
          const int off = __builtin_amdgcn_mbcnt_hi(
              (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
          cands[nc + off] = Cand{gv[k], ((unsigned)i << 3) | k};
        }
        nc += __popcll(m);
      }
    }
    __builtin_amdgcn_wave_barrier();
    for (int c = lane; c < nc; c += 64) {
      const Cand cd = cands[c];
      const QEntry &q = queue[cd.pk >> 3];
      const int lr = q.lr;
      const double2 rs = rstat[lr];
      const Fit f = fit_exact((double)cd.g, (double)q.sa, q.saa, rs.x, rs.y, g);
      atomicMin(&best[lr], make_key(f.err, 8ll * q.dom + (cd.pk & 7), g));
    }
    __builtin_amdgcn_wave_barrier();
  }
  const int rem = qn - n;
  static_assert(sizeof(QEntry) == 64, "entry is four 16-byte words");
  uint4 t0 = uint4{0, 0, 0, 0}, t1 = t0, t2 = t0, t3 = t0;
  if (lane < rem) {
    const uint4 *src = (const uint4 *)&queue[n + lane];
    t0 = src[0];
    t1 = src[1];
    t2 = src[2];
    t3 = src[3];
  }
  __builtin_amdgcn_wave_barrier();
  if (lane < rem) {
    uint4 *dst = (uint4 *)&queue[lane];
    dst[0] = t0;
    dst[1] = t1;
    dst[2] = t2;
    dst[3] = t3;
  }
  qn = rem;
}

// grid: (chunks, R_pad / 64); block: 4 waves, each owning 16 ranges
// (4 row blocks of 32 rows = 4 ranges x 8 transforms).  The workgroup sweeps
// column blocks [cb_begin + x * cb_per_chunk, ...) of 32 domains each.
//
// Lane layout of v_mfma_f32_32x32x16_f16: lane l supplies row (l mod 32) of
// the A block and column (l mod 32) of the B block, k-slice 8 (l / 32) .. +7,
// and receives column (l mod 32), rows 8 (v / 4) + 4 (l / 32) + (v mod 4) of
// the result in accumulator v.  Row rho = 8 g + 4 h + q of a block is mapped
// to range 2 h + g / 2 and transform 4 (g mod 2) + q, so accumulators 0..7
// of lane l hold the 8 transforms of range 2 (l / 32) and accumulators 8..15
// those of range 2 (l / 32) + 1.
template <int K>
__global__ __launch_bounds__(256, 2) void k_search_mfma_u8(Geo g, EncBufs b,
                                                           int cb_begin,
                                                           int cb_end,
                                                           int cb_per_chunk) {
  constexpr int KS = K / 16;
  __shared__ unsigned long long s_best[4][kWaveRanges];
  __shared__ double2 s_rstat[4][kWaveRanges];   // (Sb, Sbb) of each range
  __shared__ QEntry s_queue[4][kQueue];
  __shared__ Cand s_cands[4][8 * 64];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int h = lane >> 5;
  const int cl = lane & 31;
  const int wr0 = blockIdx.y * (4 * kWaveRanges) + wave * kWaveRanges;
  unsigned long long *my_best = s_best[wave];
  double2 *rstat = s_rstat[wave];
  QEntry *queue = s_queue[wave];
  Cand *cands = s_cands[wave];
  int qn = 0;  // queued survivors (wave-uniform)

  unsigned long long gsnap = ~0ull;  // global keys as last seen
  if (lane < kWaveRanges) {
    gsnap = load_best(&b.best[wr0 + lane]);
    my_best[lane] = gsnap;
    rstat[lane] = double2{b.rng_sb[wr0 + lane], b.rng_sbb[wr0 + lane]};
  }

  half8 af[kRB][KS];
  {
    const int rho = lane & 31;
    const int gg = rho >> 3, hh = (rho >> 2) & 1, q = rho & 3;
    const int rl = 2 * hh + (gg >> 1), iso = 4 * (gg & 1) + q;
#pragma unroll
    for (int rb = 0; rb < kRB; ++rb) {
      const _Float16 *src =
          b.aop + ((size_t)(wr0 + 4 * rb + rl) * 8 + iso) * K + 8 * h;
#pragma unroll
      for (int kk = 0; kk < KS; ++kk)
        af[rb][kk] = *(const half8 *)(src + 16 * kk);
    }
  }

  // per lane: ranges wr0 + 4 rb + 2 h + e for slot s = 2 rb + e
  float wp[kSlots], bbar[kSlots];
#pragma unroll
  for (int s = 0; s < kSlots; ++s)
    bbar[s] = (float)(b.rng_sb[wr0 + 4 * (s >> 1) + 2 * h + (s & 1)] / K);
  __builtin_amdgcn_wave_barrier();
  refresh_weights(wp, my_best, rstat, h, g);

  const int c0 = cb_begin + blockIdx.x * cb_per_chunk;
  const int c1 = min(c0 + cb_per_chunk, cb_end);
  if (c0 >= c1) return;

  half8 bf[KS];
  float csa, cdp;
  int cdom;
  double csaa;
  {
    const int col = c0 * 32 + cl;
    const _Float16 *bsrc = b.bop + (size_t)col * K + 8 * h;
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) bf[kk] = *(const half8 *)(bsrc + 16 * kk);
    csa = b.col_sa[col];
    cdp = b.col_dp[col];
    cdom = b.col_dom[col];
    csaa = b.col_saa[col];
  }

  for (int cb = c0; cb < c1; ++cb) {
    const int slot = (cb - c0) % kSync;
    // prefetch the next column block
    half8 bn[KS];
    const int ncol = (cb + 1 < c1 ? cb + 1 : cb) * 32 + cl;
    {
      const _Float16 *bsrc = b.bop + (size_t)ncol * K + 8 * h;
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) bn[kk] = *(const half8 *)(bsrc + 16 * kk);
    }
    const float nsa = b.col_sa[ncol], ndp = b.col_dp[ncol];
    const int ndom = b.col_dom[ncol];
    const double nsaa = b.col_saa[ncol];

    f32x16 acc[kRB];
#pragma unroll
    for (int rb = 0; rb < kRB; ++rb) {
      acc[rb] = f32x16{};
#pragma unroll
      for (int kk = 0; kk < KS; ++kk)
        acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(af[rb][kk], bf[kk],
                                                         acc[rb], 0, 0, 0);
    }

    // Per (range, domain) pair: the 8 transforms' G are non-negative
    // integers in FP32, so their bit patterns order like unsigned integers
    // and max/min need no float canonicalisation.
    float gmx[kSlots], gmn[kSlots];
#pragma unroll
    for (int rb = 0; rb < kRB; ++rb)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        unsigned ux = __float_as_uint(acc[rb][8 * e]), un = ux;
#pragma unroll
        for (int k = 1; k < 8; ++k) {
          const unsigned u = __float_as_uint(acc[rb][8 * e + k]);
          ux = max(ux, u);
          un = min(un, u);
        }
        gmx[2 * rb + e] = __uint_as_float(ux);
        gmn[2 * rb + e] = __uint_as_float(un);
      }
    bool any_pass = false;
#pragma unroll
    for (int s = 0; s < kSlots; ++s)
      any_pass |= pair_passes(gmx[s], gmn[s], csa, bbar[s], wp[s], cdp);

    if (__any(any_pass)) {
      // append every passing pair, with its 8 G values, to the wave's queue
      // (ballot + mbcnt give each lane its position)
      bool drained = false;
#pragma unroll
      for (int rb = 0; rb < kRB; ++rb)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int s = 2 * rb + e;
          const bool ps =
              pair_passes(gmx[s], gmn[s], csa, bbar[s], wp[s], cdp);
          const unsigned long long m = __builtin_amdgcn_ballot_w64(ps);
          if (m == 0) continue;
          if (ps) {
            const int off = __builtin_amdgcn_mbcnt_hi(
                (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
            QEntry *q = &queue[qn + off];
            q->g0 = float4{acc[rb][8 * e], acc[rb][8 * e + 1],
                           acc[rb][8 * e + 2], acc[rb][8 * e + 3]};
            q->g1 = float4{acc[rb][8 * e + 4], acc[rb][8 * e + 5],
                           acc[rb][8 * e + 6], acc[rb][8 * e + 7]};
            q->saa = csaa;
            q->sa = csa;
            q->dp = cdp;
            q->dom = cdom;
            q->lr = 4 * rb + 2 * h + e;
          }
          qn += __popcll(m);
          if (qn >= 64) {
            drain(queue, cands, qn, qn & ~63, my_best, rstat, g);
            drained = true;
          }
        }
      if (drained) refresh_weights(wp, my_best, rstat, h, g);
    }

    const int jn = cb - c0 + 1;  // blocks done in this chunk
    if (jn == 1 || jn == 2 || slot == kSync - 1 || cb + 1 == c1) {
      // merge the global snapshot taken at the previous sync, publish this
      // wave's bests with a non-returning atomic and take a new snapshot
      // (the last block also drains what is left in the queue)
      if (cb + 1 == c1 && qn > 0)
        drain(queue, cands, qn, qn, my_best, rstat, g);
      if (lane < kWaveRanges) {
        const unsigned long long m = min(my_best[lane], gsnap);
        my_best[lane] = m;
        if (m < gsnap) atomicMin(&b.best[wr0 + lane], m);
        gsnap = load_best(&b.best[wr0 + lane]);
      }
      refresh_weights(wp, my_best, rstat, h, g);
    }

#pragma unroll
    for (int kk = 0; kk < KS; ++kk) bf[kk] = bn[kk];
    csa = nsa;
    cdp = ndp;
    cdom = ndom;
    csaa = nsaa;
  }
}

}  // namespace

hipError_t launch_search_mfma(const Geo &g, const EncBufs &b, int chunks,
                              int seeded_blocks, hipStream_t st) {
  static_assert(4 * kWaveRanges == kMfmaRangesPerWG, "tile");
  if (g.bits != 8) return hipErrorInvalidValue;
  const int rg = g.R_pad / kMfmaRangesPerWG;
  const int rest = g.NCB - seeded_blocks;
  if (rest <= 0) return hipSuccess;
  const int cbpc = (rest + chunks - 1) / chunks;
  const int nchunks = (rest + cbpc - 1) / cbpc;
  auto kern = g.K == 64 ? k_search_mfma_u8<64> : k_search_mfma_u8<16>;
  hipLaunchKernelGGL(kern, dim3(nchunks, rg), dim3(256), 0, st, g, b,
                     seeded_blocks, g.NCB, cbpc);
  return hipGetLastError();
}

}  // namespace fic
