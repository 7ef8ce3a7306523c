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
// The few survivors are fitted exactly in FP64 and folded into the range's
// packed (residual, candidate) key: first in a per-workgroup LDS table
// (ds_min), then, every few column blocks, into the global table with a
// 64-bit atomic min.  Keys order (residual, candidate) lexicographically, so
// the result does not depend on the order in which tiles run.
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
constexpr int kQueue = 64 * (kSlots + 1);  // per-wave survivor queue entries

// A queued survivor: G as float bits, and col << 7 | local range << 3 | k.
struct QEntry {
  unsigned g;
  unsigned tag;
};

__device__ __forceinline__ unsigned long long load_best(
    const unsigned long long *p) {
  // bypass the non-coherent L1 so other workgroups' improvements are seen
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Prune weight from a packed key and the range's V = K Sbb - Sb^2.
__device__ __forceinline__ float weight_from_key(unsigned long long key,
                                                 double V, const Geo &g) {
  if (V == 0.0) return __builtin_inff();
  const double K = (double)g.K;
  const double Wd = V - K * key_err(key, g);
  if (!(Wd > 0.0)) return 0.0f;
  return (float)(Wd / (K * K)) * (1.0f - 0x1p-20f);
}

__device__ __forceinline__ void refresh_weights(float *wp,
                                                const unsigned long long *best,
                                                const double *V, int h,
                                                const Geo &g) {
#pragma unroll
  for (int s = 0; s < kSlots; ++s)
    wp[s] = weight_from_key(best[4 * (s >> 1) + 2 * h + (s & 1)], V[s], g);
}

// Fit the first n queued survivors exactly (64 per round, one per lane),
// fold them into the wave's best keys and keep the remaining qn - n entries
// (fewer than 64) at the front of the queue.
__device__ __forceinline__ void drain(QEntry *queue, int &qn, int n,
                                      unsigned long long *best, int wr0,
                                      const EncBufs &b, const Geo &g) {
  const int lane = threadIdx.x & 63;
  for (int base = 0; base < n; base += 64) {
    const int i = base + lane;
    if (i < n) {
      const QEntry q = queue[i];
      const int col = (int)(q.tag >> 7);
      const int lr = (int)((q.tag >> 3) & 15);
      const int k = (int)(q.tag & 7);
      const int r = wr0 + lr;
      const Fit f = fit_exact((double)__uint_as_float(q.g),
                              (double)b.col_sa[col], b.col_saa[col],
                              b.rng_sb[r], b.rng_sbb[r], g);
      const unsigned long long key =
          make_key(f.err, 8ll * b.col_dom[col] + k, g);
      atomicMin(&best[lr], key);
    }
  }
  const int rem = qn - n;
  QEntry t;
  if (lane < rem) t = queue[n + lane];
  __builtin_amdgcn_wave_barrier();
  if (lane < rem) queue[lane] = t;
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
  __shared__ unsigned long long s_best[4 * kWaveRanges];
  __shared__ QEntry s_queue[4][kQueue];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int h = lane >> 5;
  const int cl = lane & 31;
  const int wr0 = blockIdx.y * (4 * kWaveRanges) + wave * kWaveRanges;
  unsigned long long *my_best = s_best + wave * kWaveRanges;
  QEntry *queue = s_queue[wave];
  int qn = 0;  // queued survivors (wave-uniform)

  unsigned long long gsnap = ~0ull;  // global keys as last seen
  if (lane < kWaveRanges) {
    gsnap = load_best(&b.best[wr0 + lane]);
    my_best[lane] = gsnap;
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
  double V[kSlots];
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    const int r = wr0 + 4 * (s >> 1) + 2 * h + (s & 1);
    const double Sb = b.rng_sb[r], Sbb = b.rng_sbb[r];
    V[s] = (double)g.K * Sbb - Sb * Sb;
    bbar[s] = (float)(Sb / K);
  }
  __syncthreads();
  refresh_weights(wp, my_best, V, h, g);

  const int c0 = cb_begin + blockIdx.x * cb_per_chunk;
  const int c1 = min(c0 + cb_per_chunk, cb_end);
  if (c0 >= c1) return;

  half8 bf[KS];
  float csa, cdp;
  {
    const int col = c0 * 32 + cl;
    const _Float16 *bsrc = b.bop + (size_t)col * K + 8 * h;
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) bf[kk] = *(const half8 *)(bsrc + 16 * kk);
    csa = b.col_sa[col];
    cdp = b.col_dp[col];
  }

  for (int cb = c0; cb < c1; ++cb) {
    const int col = cb * 32 + cl;
    // prefetch the next column block
    half8 bn[KS];
    float nsa = 0.0f, ndp = 0.0f;
    const int ncol = (cb + 1 < c1 ? cb + 1 : cb) * 32 + cl;
    {
      const _Float16 *bsrc = b.bop + (size_t)ncol * K + 8 * h;
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) bn[kk] = *(const half8 *)(bsrc + 16 * kk);
      nsa = b.col_sa[ncol];
      ndp = b.col_dp[ncol];
    }

    f32x16 acc[kRB];
#pragma unroll
    for (int rb = 0; rb < kRB; ++rb) {
      acc[rb] = f32x16{};
#pragma unroll
      for (int kk = 0; kk < KS; ++kk)
        acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(af[rb][kk], bf[kk],
                                                         acc[rb], 0, 0, 0);
    }

    unsigned pm = 0;
#pragma unroll
    for (int rb = 0; rb < kRB; ++rb)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int s = 2 * rb + e;
        const float v0 = acc[rb][8 * e], v1 = acc[rb][8 * e + 1];
        float mx = fmaxf(v0, v1), mn = fminf(v0, v1);
#pragma unroll
        for (int k = 2; k < 8; k += 2) {
          const float va = acc[rb][8 * e + k], vb = acc[rb][8 * e + k + 1];
          mx = __builtin_fmaxf(mx, __builtin_fmaxf(va, vb));
          mn = __builtin_fminf(mn, __builtin_fminf(va, vb));
        }
        const float a0 = fmaf(-csa, bbar[s], mx);
        const float a1 = fmaf(-csa, bbar[s], mn);
        const float mm = fmaxf(fabsf(a0), fabsf(a1));
        pm |= (mm * mm >= wp[s] * cdp) ? (1u << s) : 0u;
      }

    if (__any(pm != 0u)) {
      // append every candidate that passes the per-transform test to the
      // wave's queue (ballot + mbcnt give each lane its slot)
#pragma unroll
      for (int rb = 0; rb < kRB; ++rb)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int s = 2 * rb + e;
          if (!__any((pm >> s) & 1u)) continue;
          const unsigned tag0 = ((unsigned)col << 7) | ((4 * rb + 2 * h + e) << 3);
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const float v = acc[rb][8 * e + k];
            const float a = fmaf(-csa, bbar[s], v);
            const bool f = ((pm >> s) & 1u) && a * a >= wp[s] * cdp;
            const unsigned long long m = __ballot(f);
            if (f) {
              const int off = __builtin_amdgcn_mbcnt_hi(
                  (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
              queue[qn + off] = QEntry{__float_as_uint(v), tag0 | k};
            }
            qn += __popcll(m);
          }
          if (qn >= 64) {
            drain(queue, qn, qn & ~63, my_best, wr0, b, g);
            refresh_weights(wp, my_best, V, h, g);
          }
        }
    }

    if (cb + 1 == c1 && qn > 0) drain(queue, qn, qn, my_best, wr0, b, g);
    if (((cb - c0) % kSync) == kSync - 1 || cb + 1 == c1) {
      // merge the global snapshot taken at the previous sync, publish this
      // wave's bests (non-returning atomic) and take a new snapshot
      if (lane < kWaveRanges) {
        const unsigned long long m = min(my_best[lane], gsnap);
        my_best[lane] = m;
        if (m < gsnap) atomicMin(&b.best[wr0 + lane], m);
        gsnap = load_best(&b.best[wr0 + lane]);
      }
      refresh_weights(wp, my_best, V, h, g);
    }

#pragma unroll
    for (int kk = 0; kk < KS; ++kk) bf[kk] = bn[kk];
    csa = nsa;
    cdp = ndp;
  }
}

}  // namespace

hipError_t launch_search_mfma(const Geo &g, const EncBufs &b, int chunks,
                              hipStream_t st) {
  static_assert(4 * kWaveRanges == kMfmaRangesPerWG, "tile");
  if (g.bits != 8) return hipErrorInvalidValue;
  const int rg = g.R_pad / kMfmaRangesPerWG;
  // Seed pass: every workgroup sweeps the first column blocks alone.  The
  // sweep order spreads any prefix of columns over the whole image, so this
  // gives every range a good best residual before the main pass splits the
  // remaining columns into chunks that run side by side.
  const int seed = g.NCB >= 64 ? 8 : 0;
  auto kern = g.K == 64 ? k_search_mfma_u8<64> : k_search_mfma_u8<16>;
  if (seed)
    hipLaunchKernelGGL(kern, dim3(1, rg), dim3(256), 0, st, g, b, 0, seed,
                       seed);
  const int rest = g.NCB - seed;
  const int cbpc = (rest + chunks - 1) / chunks;
  const int nchunks = (rest + cbpc - 1) / cbpc;
  hipLaunchKernelGGL(kern, dim3(nchunks, rg), dim3(256), 0, st, g, b, seed,
                     g.NCB, cbpc);
  return hipGetLastError();
}

}  // namespace fic
