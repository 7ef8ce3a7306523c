// fic_search_mfma.hip -- the range-domain search of Alg. 2/3 as a matrix-core
// contraction on CDNA4 (gfx950).
//
// For a range r, a domain d and a transform k the least-squares fit needs one
// range-specific inner product, G = sum_q A_d[sigma_k(q)] b_r[q] (the other
// sums of eqs. 9-10 are per-range or per-domain constants).  Putting the
// eight transforms on the range side (row 8 r + k of the range operand holds
// b_r scattered by sigma_k), all G form one product
//       G[(r, k), d] = sum_p Rop[(r, k), p] * Bop[d, p]
// of an (8 R) x K by K x ND pair of integer matrices.
//
// Both operands are centred on their block's rounded mean: the domain
// operand holds A - m_d (m_d = round(SA/K), |A - m_d| <= 1020) and the range
// operand b - m_r (m_r = round(Sb/K), |b - m_r| <= 255), integers exact in
// FP16.  With the centred sums bounded by Cauchy-Schwarz (norms <= 510.1
// sqrt(K) and 127.6 sqrt(K)), every partial sum of
//       H = sum_q (A[sigma_k(q)] - m_d)(b[q] - m_r)
// stays below 2^22 in magnitude, so v_mfma_f32_32x32x16_f16 with FP32
// accumulation produces H exactly, and
//       G = H + m_r SA + m_d Sb - K m_d m_r            (exact in FP64),
//       G - SA Sb / K = H - c,   c = K delta_d delta_r,
// with delta_d = SA/K - m_d and delta_r = Sb/K - m_r in [-1/2, 1/2], so the
// least-squares quantity of the prune differs from H by the same small c
// (|c| <= K/4) for all 8 transforms of a pair.
//
// The output is never stored.  Each 32x32 MFMA tile holds, per lane, one
// domain column and the 8 transforms of two ranges (the row order of the
// range operand is chosen for that), and the epilogue prunes with an
// exact-safe least-squares bound shared by the 8 transforms: a candidate can
// only tie or beat the range's best residual if
//       |G - SA Sb / K| >= sqrt(W' D'),
// so a (range, domain) pair can be skipped when max_k |H_k| + |c| is below
// that threshold: one max of absolute values, one product and one fused
// compare per pair.
// Pairs that pass are appended, with their 8 H values and the column's
// statistics, to a per-wave LDS queue; 64 at a time they are re-tested per
// transform, the surviving transforms are compacted into a list and fitted
// exactly in FP64, one per lane.
// The resulting packed (residual, candidate) keys are folded into a per-wave
// LDS table (ds_min) and, every few column blocks, into the global table
// with a 64-bit atomic min.  Keys order (residual, candidate)
// lexicographically, so the result does not depend on the order of the work.
#include <math.h>

#include "fic_finalize.h"

namespace fic {

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kRB = 4;              // row blocks (4 ranges each) per wave
constexpr int kSlots = 2 * kRB;     // ranges per lane
constexpr int kWaveRanges = 4 * kRB;
constexpr int kSync = 4;            // column blocks between global syncs
constexpr int kQueue = 128;         // pairs; >= 63 + 64 lanes

// A queued (range, domain) pair: the 8 transforms' centred products H, the
// column's statistics and dl = domain << 4 | wave-local range index.
struct __attribute__((aligned(16))) QEntry {
  float4 g0, g1;
  float sa, sc;
  unsigned saa;
  int dl;
};

// A surviving transform of a queued pair: H, and pair index << 3 | k.
struct Cand {
  float g;
  unsigned pk;
};

// max_k |H_k| over the 8 transforms of a pair (exact integers in FP32).
__device__ __forceinline__ float abs_max8(const f32x16 &a, int e) {
  // starting from 0 (a canonical value) lets every step fold into v_max3
  float m = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) m = fmaxf(m, fabsf(a[8 * e + k]));
  return m;
}

// Recompute the prune thresholds: lane l < 16 computes sqrt(W') of wave
// range l once and stores it at wtab[h][s] (range 4 (s / 2) + 2 h + s mod 2,
// the layout of a lane's 8 slots); the sweep reads its 8 from LDS.  W' is
// rounded down by 2^-20 (weight_from_key); the hardware square root (within
// 1 ulp) is scaled down by 2^-22, so the threshold stays below the exact
// root with room for the FP32 rounding of the test.
__device__ __forceinline__ void refresh_weights(const unsigned long long *best,
                                                const double2 *rstat,
                                                float *wtab, int lane,
                                                const Geo &g) {
  if (lane < kWaveRanges) {
    const double2 rs = rstat[lane];
    const float wv =
        weight_from_key(best[lane], (double)g.K * rs.y - rs.x * rs.x, g);
    const float sw = __builtin_amdgcn_sqrtf(wv) * (1.0f - 0x1p-22f);
    wtab[((lane >> 1) & 1) * kSlots + 2 * (lane >> 2) + (lane & 1)] = sw;
  }
  __builtin_amdgcn_wave_barrier();
}

// The 8 values of a lane's half h from a [2][kSlots] LDS table.
__device__ __forceinline__ void read_slots(const float *tab, int h,
                                           float (&v)[kSlots]) {
  const float4 *t = (const float4 *)(tab + h * kSlots);
  const float4 a = t[0], c = t[1];
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = c.x; v[5] = c.y; v[6] = c.z; v[7] = c.w;
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
        const float sa = q.sa, sc = q.sc;
        const int lr = q.dl & 15;
        const double2 rs = rstat[lr];
        // G - SA Sb/K = H - c with c = (SA - K m_d)(Sb - K m_r)/K, exact
        const float kf = (float)g.K, ik = (float)g.invK;
        const float sbf = (float)rs.x;
        const float dd = fmaf(-kf, centre_f(sa, ik), sa);
        const float dr = fmaf(-kf, centre_f(sbf, ik), sbf);
        const float c = dd * dr * ik;
        const float t =
            weight_from_key(best[lr], K * rs.y - rs.x * rs.x, g) * sc * sc;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const float a = gv[k] - c;
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
      const int lr = q.dl & 15;
      const double2 rs = rstat[lr];
      const Fit f = fit_exact(g_from_centred((double)cd.g, (double)q.sa, rs.x, g),
                              (double)q.sa, (double)q.saa, rs.x, rs.y, g);
      atomicMin(&best[lr], make_key(f.err, 8ll * (q.dl >> 4) + (cd.pk & 7), g));
    }
    __builtin_amdgcn_wave_barrier();
  }
  const int rem = qn - n;
  static_assert(sizeof(QEntry) == 48, "entry is three 16-byte words");
  uint4 t0 = uint4{0, 0, 0, 0}, t1 = t0, t2 = t0;
  if (lane < rem) {
    const uint4 *src = (const uint4 *)&queue[n + lane];
    t0 = src[0];
    t1 = src[1];
    t2 = src[2];
  }
  __builtin_amdgcn_wave_barrier();
  if (lane < rem) {
    uint4 *dst = (uint4 *)&queue[lane];
    dst[0] = t0;
    dst[1] = t1;
    dst[2] = t2;
  }
  qn = rem;
}

// Per-wave state of the sweep (lives in registers and LDS).
struct WaveState {
  unsigned long long *best;  // LDS: wave's best keys
  double2 *rstat;            // LDS: (Sb, Sbb) per range
  QEntry *queue;             // LDS: queued pairs
  Cand *cands;               // LDS: drain candidates
  float *wtab;               // LDS: prune thresholds sqrt(W') [2][kSlots]
  float *dtab;               // LDS: (Sb - K m_r) / K per range [2][kSlots]
  int *slots;                // LDS: range slot of each wave range (-1: none)
  int ci_next;               // column of the next block (-1: none)
  int nD;                    // searched domain columns
  int qn;                    // queued pairs (wave-uniform)
  unsigned long long gsnap;  // global keys as last read (lanes < 16)
  int wr0, h, cl, lane;
};

// Column ci of the domain operand and its record; ci < 0 (past the searched
// columns) reads column 0 and marks it flat, so it never passes the prune.
// FRAG: the operand is in fragment order (a full search), where lane
// (h, c mod 32) of k-step kk reads 16 bytes at block offset kk 1024 + 16 lane.
template <int K, bool FRAG>
__device__ __forceinline__ void load_column(const EncBufs &b, int ci, int h,
                                            half8 (&bn)[K / 16], ColRec &nsd) {
  const int c = ci >= 0 ? ci : 0;
  const _Float16 *bsrc =
      FRAG ? b.bop + (size_t)(c >> 5) * 32 * K + ((h << 5) | (c & 31)) * 8
           : b.bop + (size_t)c * K + 8 * h;
  constexpr int kstep = FRAG ? 512 : 16;
#pragma unroll
  for (int kk = 0; kk < K / 16; ++kk)
    bn[kk] = gld((const half8 *)(bsrc + kstep * kk));
  // as one 16-byte vector: a struct copy would go through a generic reference
  nsd = __builtin_bit_cast(ColRec, gld((const u32x4 *)&b.col_rec[c]));
  if (ci < 0) nsd.sc = __builtin_inff();
}

// Column of searched block cb for lane column cl (-1 past the list); with
// identity lists (ident) the list entry is its own index and is not read.
__device__ __forceinline__ int column_of(const EncBufs &b, int nD, int cb,
                                         int cl, int ident) {
  const int j = cb * 32 + cl;
  if (ident) return j < nD ? j : -1;
  return j < nD ? gld(&b.act_col[j]) : -1;
}

// One 32-column block: prefetch the next block's operand and column records
// into (bn, nsd), run the MFMA
// contraction with (bf, sd), prune, queue survivors, sync every few blocks.
template <int K, bool FRAG>
__device__ __forceinline__ void sweep_block(
    const Geo &g, const EncBufs &b, WaveState &w, const half8 (&af)[kRB][K / 16],
    const half8 (&bf)[K / 16], const ColRec &sd, half8 (&bn)[K / 16],
    ColRec &nsd, int cb, int c0, int c1) {
  constexpr int KS = K / 16;
  // the lane's 8 prune thresholds sqrt(W'), kept in LDS between blocks
  float sw[kSlots], rd[kSlots];
  read_slots(w.wtab, w.h, sw);
  if constexpr (K != 64) read_slots(w.dtab, w.h, rd);
  const int slot = (cb - c0) % kSync;
  {
    // the next block (its column index came a block earlier) and the index
    // of the block after it
    load_column<K, FRAG>(b, w.ci_next, w.h, bn, nsd);
    w.ci_next = cb + 2 < c1 ? column_of(b, w.nD, cb + 2, w.cl, g.ident) : -1;
  }
  // keep the prefetch ahead of the matrix-core work
  __builtin_amdgcn_sched_barrier(0);

  // k-step outer, row block inner: the four accumulator chains interleave,
  // so no MFMA waits for the one before it
  f32x16 acc[kRB];
#pragma unroll
  for (int rb = 0; rb < kRB; ++rb) acc[rb] = f32x16{};
#pragma unroll
  for (int kk = 0; kk < KS; ++kk)
#pragma unroll
    for (int rb = 0; rb < kRB; ++rb)
      acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(af[rb][kk], bf[kk],
                                                       acc[rb], 0, 0, 0);
  const float csa = sd.sa, csc = sd.sc;

  // Per (range, domain) pair: G_k - SA Sb/K = H_k - c with
  // c = (SA - K m_d)(Sb - K m_r)/K, the same c for all 8 transforms (the
  // column's SA - K m_d times the slot's (Sb - K m_r) / K, exact).  The pair
  // can only matter if max_k |H_k - c| >= sqrt(W') sqrt(D') (both roots
  // rounded down; +inf for a flat domain or range, and 0 * inf = NaN for a
  // flat domain against a useless bound: the compare fails both times).
  // 8x8 ranges bound max_k |H_k - c| by max_k |H_k| + |SA - K m_d| / 2
  // (>= |c|, small against the thresholds there); 4x4 ranges, whose
  // thresholds are often as small as |c|, take the exact
  // max(H_max - c, c - H_min).  Wave masks of the passing pairs, one per
  // slot, in scalar registers.
  const float cdd = fmaf(-(float)K, centre_f(csa, 1.0f / K), csa);
  const float cdh = 0.5f * fabsf(cdd);
  unsigned long long pm[kSlots], anym = 0;
#pragma unroll
  for (int rb = 0; rb < kRB; ++rb)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int s = 2 * rb + e;
      bool pass;
      if constexpr (K == 64) {
        // |c| <= |SA - K m_d| / 2, one bound per column
        pass = abs_max8(acc[rb], e) >= fmaf(sw[s], csc, -cdh);
      } else {
        const float c = cdd * rd[s];
        float hx = acc[rb][8 * e], hn = hx;
#pragma unroll
        for (int k = 1; k < 8; ++k) {
          hx = fmaxf(hx, acc[rb][8 * e + k]);
          hn = fminf(hn, acc[rb][8 * e + k]);
        }
        pass = fmaxf(hx - c, c - hn) >= sw[s] * csc;
      }
      pm[s] = __builtin_amdgcn_ballot_w64(pass);
      anym |= pm[s];
    }

  if (anym != 0) {
    // append every passing pair, with its 8 G values, to the wave's queue
    // (ballot + mbcnt give each lane its position)
    const int cdl = sd.dom << 4;
    bool drained = false;
#pragma unroll
    for (int rb = 0; rb < kRB; ++rb)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int s = 2 * rb + e;
        const unsigned long long m = pm[s];
        if (m == 0) continue;
        const bool ps = (m >> w.lane) & 1;
        if (ps) {
          const int off = __builtin_amdgcn_mbcnt_hi(
              (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
          QEntry *q = &w.queue[w.qn + off];
          q->g0 = float4{acc[rb][8 * e], acc[rb][8 * e + 1], acc[rb][8 * e + 2],
                         acc[rb][8 * e + 3]};
          q->g1 = float4{acc[rb][8 * e + 4], acc[rb][8 * e + 5],
                         acc[rb][8 * e + 6], acc[rb][8 * e + 7]};
          *(uint4 *)&q->sa =
              uint4{__float_as_uint(csa), __float_as_uint(csc), sd.saa,
                    (unsigned)(cdl | (4 * rb + 2 * w.h + e))};
        }
        w.qn += __popcll(m);
        if (w.qn >= 64) {
          drain(w.queue, w.cands, w.qn, w.qn & ~63, w.best, w.rstat, g);
          drained = true;
        }
      }
    if (drained) refresh_weights(w.best, w.rstat, w.wtab, w.lane, g);
  }

  const int jn = cb - c0 + 1;  // blocks done in this chunk
  if (jn == 1 || jn == 2 || slot == kSync - 1 || cb + 1 == c1) {
    // publish this wave's bests with a non-returning atomic where they
    // beat the global keys as last read, then read the global keys and use
    // them at once: waiting for the read costs less than sweeping on with a
    // stale bound (the last block first drains what is left in the queue;
    // its read is kept too, which measured faster than leaving it out)
    if (cb + 1 == c1 && w.qn > 0)
      drain(w.queue, w.cands, w.qn, w.qn, w.best, w.rstat, g);
    if (w.lane < kWaveRanges) {
      const int sl = w.slots[w.lane];
      if (sl >= 0) {
        const unsigned long long m = w.best[w.lane];
        if (m < w.gsnap) publish_best(&b.best[sl], m);
        w.gsnap = load_best(&b.best[sl]);
        w.best[w.lane] = min(m, w.gsnap);
      }
    }
    refresh_weights(w.best, w.rstat, w.wtab, w.lane, g);
  }
}

// Starting bound from the workgroup's first nb column blocks (nb <=
// kSeedBlocks).  Each lane ranks the 8 transforms of each of its ranges
// against its column of every block by the least-squares score H^2 / D'
// (H the centred product, which differs from G - SA Sb/K by at most K/4) and
// keeps the best; the bests are posted through LDS (the empty candidate and
// queue buffers) and lane l < 16 picks range l's best and fits that one
// candidate exactly.  Any candidate's exact residual is a valid bound; the
// sweep then covers these blocks as usual.
constexpr int kSeedBlocks = 1;
constexpr int kHBias = 1 << 22;  // |H| < 2^22: H + 2^22 fits 23 bits

template <int K, bool FRAG>
__device__ __forceinline__ void seed_blocks(const Geo &g, const EncBufs &b,
                                            WaveState &w,
                                            const half8 (&af)[kRB][K / 16],
                                            const half8 (&b0)[K / 16],
                                            const ColRec &sd0, int c0,
                                            int nb) {
  constexpr int KS = K / 16;
  // per (half, slot, column): score, and block << 27 | (H + 2^22) << 3 | k
  float *sc_tab = (float *)w.cands;
  unsigned *gk_tab = (unsigned *)w.cands + 2 * kSlots * 32;
  ColRec *col_tab = (ColRec *)w.queue;  // [kSeedBlocks][32]
  // per slot: best score (0: none), its H and block * 8 + transform
  float best[kSlots], bestg[kSlots];
  unsigned bestk[kSlots];
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    best[s] = 0.0f;
    bestg[s] = 0.0f;
    bestk[s] = 0;
  }
  half8 bf[KS];  // the first block is the sweep's, already loaded
  ColRec sd = sd0;
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) bf[kk] = b0[kk];
  for (int blk = 0; blk < nb; ++blk) {
    f32x16 acc[kRB];
#pragma unroll
    for (int rb = 0; rb < kRB; ++rb) {
      acc[rb] = f32x16{};
#pragma unroll
      for (int kk = 0; kk < KS; ++kk)
        acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(af[rb][kk], bf[kk],
                                                         acc[rb], 0, 0, 0);
    }
    const ColRec cur = sd;
    if (w.h == 0) col_tab[blk * 32 + w.cl] = cur;
    if (blk + 1 < nb)
      load_column<K, FRAG>(
          b, column_of(b, w.nD, c0 + blk + 1, w.cl, g.ident), w.h, bf, sd);
    // flat domains and padding columns (sqrt(D') = +inf) score 0 and take no
    // part (as does a candidate with H = 0)
    const float idp =
        cur.sc != __builtin_inff() ? 1.0f / (cur.sc * cur.sc) : 0.0f;
#pragma unroll
    for (int rb = 0; rb < kRB; ++rb)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int s = 2 * rb + e;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const float gv = acc[rb][8 * e + k];
          const float v = gv * gv * idp;
          const bool up = v > best[s];
          best[s] = up ? v : best[s];
          bestg[s] = up ? gv : bestg[s];
          bestk[s] = up ? (unsigned)(8 * blk + k) : bestk[s];
        }
      }
  }
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    sc_tab[(w.h * kSlots + s) * 32 + w.cl] = best[s];
    gk_tab[(w.h * kSlots + s) * 32 + w.cl] =
        ((bestk[s] >> 3) << 27) | ((unsigned)((int)bestg[s] + kHBias) << 3) |
        (bestk[s] & 7);
  }
  __builtin_amdgcn_wave_barrier();
  if (w.lane < kWaveRanges) {
    const int lr = w.lane, h = (lr >> 1) & 1, s = 2 * (lr >> 2) + (lr & 1);
    const float4 *row = (const float4 *)(sc_tab + (h * kSlots + s) * 32);
    float bv = 0.0f;
    int bc = -1;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float4 v = row[q];
      if (v.x > bv) { bv = v.x; bc = 4 * q; }
      if (v.y > bv) { bv = v.y; bc = 4 * q + 1; }
      if (v.z > bv) { bv = v.z; bc = 4 * q + 2; }
      if (v.w > bv) { bv = v.w; bc = 4 * q + 3; }
    }
    if (bc >= 0) {
      const unsigned t = gk_tab[(h * kSlots + s) * 32 + bc];
      const ColRec cr = col_tab[(t >> 27) * 32 + bc];
      const double2 rs = w.rstat[lr];
      const float hv = (float)((int)((t >> 3) & 0xFFFFFFu) - kHBias);
      const Fit f = fit_exact(g_from_centred((double)hv, (double)cr.sa, rs.x, g),
                              (double)cr.sa, (double)cr.saa, rs.x, rs.y, g);
      const unsigned long long key =
          make_key(f.err, 8ll * cr.dom + (t & 7), g);
      if (key < w.best[lr]) w.best[lr] = key;
    }
    // share it with the other chunks of these ranges right away
    const int sl = w.slots[lr];
    if (sl >= 0 && w.best[lr] < w.gsnap) publish_best(&b.best[sl], w.best[lr]);
  }
  __builtin_amdgcn_wave_barrier();
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
// LDS of one search workgroup.
struct SearchLds {
  unsigned long long best[4][kWaveRanges];
  double2 rstat[4][kWaveRanges];  // (Sb, Sbb) of each range
  QEntry queue[4][kQueue];
  Cand cands[4][8 * 64];
  float wtab[4][2 * kSlots];
  float dtab[4][2 * kSlots];
  int slots[4][kWaveRanges];
};

// Range operand fragments of 8x8 ranges built from the image (8-bit pixels)
// instead of read from the range operand.  The wave stages its 16 ranges'
// pixels in LDS (the empty queue), once row by row and once transposed, so
// that every transform of a fragment row is one 8-byte read of a range row or
// column, forward or reversed (sigma_k^-1 of the row, Section V).  Bytes
// become FP16 exactly: 0x64xx is 1024 + xx, and 1024 + m_r is then
// subtracted (an exact difference of two FP16 integers in [1024, 2047]).
__device__ __forceinline__ void range_fragments_from_pixels(
    const Geo &g, const uint8_t *img, WaveState &w, half8 (&af)[kRB][4]) {
  uint2 *rows = (uint2 *)w.queue;  // [16 ranges][8 rows], 8 pixels each
  uint2 *cols = rows + 16 * 8;     // [16 ranges][8 columns]
  {
    const int lr = w.lane >> 2, i0 = 2 * (w.lane & 3);
    const int sl = w.slots[lr];
    const int ri = sl >= 0 ? range_of_slot(g, sl) : g.R;
    uint2 r0 = uint2{0, 0}, r1 = uint2{0, 0};
    if (ri < g.R) {
      const uint8_t *p =
          img + (size_t)((ri / g.RW) * 8 + i0) * g.W + (size_t)(ri % g.RW) * 8;
      r0 = __builtin_bit_cast(uint2, gld((const u32x2 *)p));
      r1 = __builtin_bit_cast(uint2, gld((const u32x2 *)(p + g.W)));
    }
    rows[lr * 8 + i0] = r0;
    rows[lr * 8 + i0 + 1] = r1;
    // column j holds pixel (i, j) at byte i: this lane's bytes i0, i0 + 1
    unsigned short *ct = (unsigned short *)(cols + lr * 8);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const unsigned b0 = ((j < 4 ? r0.x : r0.y) >> (8 * (j & 3))) & 255u;
      const unsigned b1 = ((j < 4 ? r1.x : r1.y) >> (8 * (j & 3))) & 255u;
      ct[j * 4 + (i0 >> 1)] = (unsigned short)(b0 | (b1 << 8));
    }
  }
  __builtin_amdgcn_wave_barrier();
  // this lane's fragment row: range rl of each row block, transform k
  const int rho = w.lane & 31;
  const int gg = rho >> 3, hh = (rho >> 2) & 1, q = rho & 3;
  const int rl = 2 * hh + (gg >> 1), k = 4 * (gg & 1) + q;
  // row pi of sigma_k^-1: transforms 1, 3, 5, 7 read range columns; 2, 3, 6,
  // 7 read index 7 - pi; 1, 2, 4, 7 read the 8 pixels in reverse
  const bool colw = k & 1;
  const bool flip = k == 2 || k == 3 || k == 6 || k == 7;
  const bool rev = k == 1 || k == 2 || k == 4 || k == 7;
  const uint2 *tab = colw ? cols : rows;
  const unsigned c64 = 0x64646464u;
  const unsigned s0 = rev ? 0x04020403u : 0x04010400u;
  const unsigned s1 = rev ? 0x04000401u : 0x04030402u;
#pragma unroll
  for (int rb = 0; rb < kRB; ++rb) {
    // the range's rounded mean m_r is subtracted together with the 1024
    const _Float16 off = (_Float16)(
        1024.0f + centre_f((float)w.rstat[4 * rb + rl].x, 1.0f / 64.0f));
    const half8 koff = half8{off, off, off, off, off, off, off, off};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int pi = 2 * kk + w.h;
      const uint2 v = tab[(4 * rb + rl) * 8 + (flip ? 7 - pi : pi)];
      const unsigned lo = rev ? v.y : v.x, hi = rev ? v.x : v.y;
      const uint4 u = uint4{__builtin_amdgcn_perm(c64, lo, s0),
                            __builtin_amdgcn_perm(c64, lo, s1),
                            __builtin_amdgcn_perm(c64, hi, s0),
                            __builtin_amdgcn_perm(c64, hi, s1)};
      af[rb][kk] = __builtin_bit_cast(half8, u) - koff;
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// The workgroup's 64 searched ranges (entries row0 .. row0 + 63 of the range
// list) against searched column blocks [c0, c1).  nA, nD: lengths of the two
// lists.  img: the 8-bit image when the range fragments come from pixels
// (K = 64), else null (read the range operand).
template <int K, bool FRAG>
__device__ __forceinline__ void search_rows(const Geo &g, const EncBufs &b,
                                            const uint8_t *img,
                                            SearchLds &lds, int row0, int nA,
                                            int nD, int c0, int c1) {
  constexpr int KS = K / 16;
  WaveState w;
  w.lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  w.h = w.lane >> 5;
  w.cl = w.lane & 31;
  w.wr0 = row0 + wave * kWaveRanges;
  w.best = lds.best[wave];
  w.rstat = lds.rstat[wave];
  w.queue = lds.queue[wave];
  w.cands = lds.cands[wave];
  w.wtab = lds.wtab[wave];
  w.dtab = lds.dtab[wave];
  w.slots = lds.slots[wave];
  w.qn = 0;
  w.gsnap = ~0ull;
  w.nD = nD;
  if (c0 >= c1) return;

  // the wave's range slots, their keys and sums; the first two columns
  if (w.lane < kWaveRanges) {
    const int j = w.wr0 + w.lane;
    const int sl = j < nA ? (g.ident ? j : gld(&b.act_slot[j])) : -1;
    w.slots[w.lane] = sl;
    double sb = 0.0, sbb = 0.0;
    if (sl >= 0) {
      w.gsnap = load_best(&b.best[sl]);
      sb = gld(&b.rng_sb[sl]);
      sbb = gld(&b.rng_sbb[sl]);
    }
    w.best[w.lane] = w.gsnap;
    w.rstat[w.lane] = double2{sb, sbb};
  }
  const int ci0 = column_of(b, nD, c0, w.cl, g.ident);
  w.ci_next = c0 + 1 < c1 ? column_of(b, nD, c0 + 1, w.cl, g.ident) : -1;
  half8 bA[KS], bB[KS];  // two buffers for the streamed domain operand
  ColRec sdA, sdB;
  load_column<K, FRAG>(b, ci0, w.h, bA, sdA);
  __builtin_amdgcn_wave_barrier();

  half8 af[kRB][KS];
  if constexpr (K == 64) {
    if (img) range_fragments_from_pixels(g, img, w, af);
  }
  if (K != 64 || !img) {
    const int rho = w.lane & 31;
    const int gg = rho >> 3, hh = (rho >> 2) & 1, q = rho & 3;
    const int rl = 2 * hh + (gg >> 1), iso = 4 * (gg & 1) + q;
#pragma unroll
    for (int rb = 0; rb < kRB; ++rb) {
      const int sl = w.slots[4 * rb + rl];
      const _Float16 *src =
          b.aop + ((size_t)(sl >= 0 ? sl : 0) * 8 + iso) * K + 8 * w.h;
#pragma unroll
      for (int kk = 0; kk < KS; ++kk)
        af[rb][kk] = sl >= 0 ? gld((const half8 *)(src + 16 * kk)) : half8{};
    }
  }
  seed_blocks<K, FRAG>(g, b, w, af, bA, sdA, c0, min(kSeedBlocks, c1 - c0));
  // the range half of each pair's correction, (Sb - K m_r) / K (exact)
  if (w.lane < kWaveRanges) {
    const float sbf = (float)w.rstat[w.lane].x, ik = (float)g.invK;
    w.dtab[((w.lane >> 1) & 1) * kSlots + 2 * (w.lane >> 2) + (w.lane & 1)] =
        fmaf(-(float)g.K, centre_f(sbf, ik), sbf) * ik;
  }
  refresh_weights(w.best, w.rstat, w.wtab, w.lane, g);
  for (int cb = c0; cb < c1; cb += 2) {
    sweep_block<K, FRAG>(g, b, w, af, bA, sdA, bB, sdB, cb, c0, c1);
    if (cb + 1 < c1)
      sweep_block<K, FRAG>(g, b, w, af, bB, sdB, bA, sdA, cb + 1, c0, c1);
  }
}

// One image: a grid of G workgroups over the searched ranges and columns.
// The lists' lengths are read on the device; the rows of 64 ranges are each
// split into G / rows chunks of column blocks (at least one), but no chunk
// shorter than kMinChunkBlocks blocks: with few searched rows (a quadtree
// level of a few hundred ranges) hundreds of workgroups would otherwise
// share each range's key, and their syncs queue on its atomics.
constexpr int kMinChunkBlocks = 16;

template <int K>
__global__ __launch_bounds__(256, 2) void k_search_mfma_u8(Geo g, EncBufs b,
                                                           const uint8_t *img) {
  __shared__ SearchLds lds;
  const int nA = __builtin_amdgcn_readfirstlane(b.n_act[0]);
  const int nD = __builtin_amdgcn_readfirstlane(b.n_act[1]);
  const int rows = (nA + kMfmaRangesPerWG - 1) / kMfmaRangesPerWG;
  const int ncb = (nD + 31) / 32;
  if (rows == 0 || ncb == 0) return;
  const int chunks = max(
      1, min((int)gridDim.x / rows, (ncb + kMinChunkBlocks - 1) / kMinChunkBlocks));
  const int rg = blockIdx.x / chunks, chunk = blockIdx.x % chunks;
  if (rg >= rows) return;
  const int cbpc = (ncb + chunks - 1) / chunks;
  const int c0 = chunk * cbpc, c1 = min(c0 + cbpc, ncb);
  if (g.frag)
    search_rows<K, true>(g, b, img, lds, rg * kMfmaRangesPerWG, nA, nD, c0, c1);
  else
    search_rows<K, false>(g, b, img, lds, rg * kMfmaRangesPerWG, nA, nD, c0,
                          c1);
}

// Spin limit of a code-extraction item's wait (about a second): the wait
// always ends (every search item it waits for was taken earlier by a running
// workgroup and never waits itself), the limit only bounds a broken launch.
constexpr int kFinSpin = 1 << 24;

// Many slices: a persistent grid whose workgroups take work items from a
// shared counter, in the order of the work list (largest slices first).
// A search item (slice, row group, column blocks) sweeps part of a slice's
// candidate table; a code-extraction item (slice, -1, first pass, passes)
// turns part of its best keys into codes once every search item of that
// slice is done.  Such an item sits in the list after all of its slice's
// search items, so the items it waits for are already running.  When a
// slice's last code-extraction item is done, the workgroup that finished it
// records the slice's codes-ready tick (100 MHz).
template <int K>
__global__ __launch_bounds__(256, 2) void k_search_batch_u8(BatchDev bd) {
  constexpr int N = K == 64 ? 8 : 4;
  __shared__ SearchLds lds;
  __shared__ int s_item;
  if (threadIdx.x == 0)
    atomicMin(&bd.ticks[0], (unsigned long long)wall_clock64());
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(bd.counter, 1);
    __syncthreads();
    // uniform across the workgroup: keep the item and its slice in scalars
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= bd.n_items) break;
    const int4 w = load_uniform(&bd.items[it]);
    const Geo g = load_uniform(&bd.tab[w.x].g);
    const EncBufs b = load_uniform(&bd.tab[w.x].b);
    const uint8_t *img = (const uint8_t *)load_uniform(&bd.tab[w.x].image);
    if (w.y < 0) {
      // code extraction: wait until the slice's search is complete (the
      // acquire pairs with the search items' release below)
      if (threadIdx.x == 0) {
        int spins = 0;
        while (__hip_atomic_load(&bd.remaining[w.x], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT) > 0 &&
               ++spins < kFinSpin)
          __builtin_amdgcn_s_sleep(2);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      __syncthreads();
      const fic_codes out = load_uniform(&bd.tab[w.x].out);
      for (int q = 0; q < w.w; ++q) {
        finalize_body<uint8_t, N, N>(g, img, b, out, w.z + q);
        __syncthreads();  // the next pass reuses the body's LDS table
      }
      if (threadIdx.x == 0 && atomicSub(&bd.fin_remaining[w.x], 1) == 1)
        bd.ticks[1 + w.x] = (unsigned long long)wall_clock64();
      continue;
    }
    // the item's row and blocks within the slice's searched lists
    const int nA = __builtin_amdgcn_readfirstlane(gld(&b.n_act[0]));
    const int nD = __builtin_amdgcn_readfirstlane(gld(&b.n_act[1]));
    const int row0 = w.y * kMfmaRangesPerWG;
    const int c1 = min(w.w, (nD + 31) / 32);
    if (row0 < nA && w.z < c1) {
      if (g.frag)
        search_rows<K, true>(g, b, g.pix_a ? img : nullptr, lds, row0, nA, nD,
                             w.z, c1);
      else
        search_rows<K, false>(g, b, g.pix_a ? img : nullptr, lds, row0, nA,
                              nD, w.z, c1);
    }
    // every wave's key updates are complete and visible device-wide before
    // the count that lets code extraction start
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) atomicSub(&bd.remaining[w.x], 1);
  }
}

}  // namespace

hipError_t launch_search_batch(const BatchDev &bd, hipStream_t st) {
  if (bd.bits != 8) return hipErrorInvalidValue;
  if (bd.n_items <= 0) return hipSuccess;
  // about two workgroups per compute unit (256 CUs)
  const int grid = bd.n_items < kBatchSearchGrid ? bd.n_items : kBatchSearchGrid;
  auto kern = bd.rsize == 8 ? k_search_batch_u8<64> : k_search_batch_u8<16>;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, st, bd);
  return hipGetLastError();
}

hipError_t launch_search_mfma(const Geo &g, const EncBufs &b,
                              const void *image, int workgroups,
                              hipStream_t st) {
  static_assert(4 * kWaveRanges == kMfmaRangesPerWG, "tile");
  if (g.bits != 8) return hipErrorInvalidValue;
  if (workgroups < 1) workgroups = 1;
  const uint8_t *img = g.pix_a ? (const uint8_t *)image : nullptr;
  auto kern = g.K == 64 ? k_search_mfma_u8<64> : k_search_mfma_u8<16>;
  hipLaunchKernelGGL(kern, dim3(workgroups), dim3(256), 0, st, g, b, img);
  return hipGetLastError();
}

}  // namespace fic
