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
// packed (residual, candidate) key with a 64-bit atomic min, so the result is
// independent of the order in which tiles run.
#include <math.h>

#include "fic_device.h"

namespace fic {

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Exact fit of one surviving candidate; returns the range's new prune weight.
__device__ __noinline__ float eval_survivor(float Gf, int col, int r, int k,
                                            const Geo &g, const EncBufs &b) {
  const double SA = (double)b.col_sa[col];
  const double SAA = b.col_saa[col];
  const double Sb = b.rng_sb[r], Sbb = b.rng_sbb[r];
  const long long d = b.col_dom[col];
  const Fit f = fit_exact((double)Gf, SA, SAA, Sb, Sbb, g);
  const unsigned long long key = make_key(f.err, 8 * d + k, g);
  const unsigned long long old = atomicMin(&b.best[r], key);
  const unsigned long long nb = key < old ? key : old;
  return prune_weight(key_err(nb, g), Sb, Sbb, g);
}

__device__ __forceinline__ unsigned long long load_best(const EncBufs &b,
                                                        int r) {
  // bypass the non-coherent L1 so other workgroups' improvements are seen
  return __hip_atomic_load(&b.best[r], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// grid: (chunks, R_pad / (16 RB)); block: 4 waves.  Wave w owns 4 RB ranges
// (RB row blocks of 32 rows = 4 ranges x 8 transforms) and sweeps the
// workgroup's chunk of 32-column blocks.
//
// Lane layout of v_mfma_f32_32x32x16_f16: lane l supplies row (l mod 32) of
// the A block and column (l mod 32) of the B block, k-slice 8 (l / 32) .. +7,
// and receives column (l mod 32), rows 8 (v / 4) + 4 (l / 32) + (v mod 4) of
// the result in accumulator v.  Row rho = 8 g + 4 h + q of a block is mapped
// to range 2 h + g / 2 and transform 4 (g mod 2) + q, so accumulators 0..7
// of lane l hold the 8 transforms of range 2 (l / 32) and accumulators 8..15
// those of range 2 (l / 32) + 1.
template <int K, int RB>
__global__ __launch_bounds__(256) void k_search_mfma_u8(Geo g, EncBufs b,
                                                        int cb_per_chunk) {
  constexpr int KS = K / 16;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int h = lane >> 5;
  const int cl = lane & 31;
  const int rbase = blockIdx.y * (16 * RB) + wave * (4 * RB);

  half8 af[RB][KS];
  {
    const int rho = lane & 31;
    const int gg = rho >> 3, hh = (rho >> 2) & 1, q = rho & 3;
    const int rl = 2 * hh + (gg >> 1), iso = 4 * (gg & 1) + q;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const _Float16 *src =
          b.aop + ((size_t)(rbase + 4 * rb + rl) * 8 + iso) * K + 8 * h;
#pragma unroll
      for (int kk = 0; kk < KS; ++kk)
        af[rb][kk] = *(const half8 *)(src + 16 * kk);
    }
  }

  float wp[2 * RB], bbar[2 * RB];
#pragma unroll
  for (int s = 0; s < 2 * RB; ++s) {
    const int r = rbase + 4 * (s >> 1) + 2 * h + (s & 1);
    const double Sb = b.rng_sb[r], Sbb = b.rng_sbb[r];
    bbar[s] = (float)(Sb / K);
    wp[s] = prune_weight(key_err(load_best(b, r), g), Sb, Sbb, g);
  }

  const int cb0 = blockIdx.x * cb_per_chunk;
  const int cb1 = min(cb0 + cb_per_chunk, g.NCB);
  for (int cb = cb0; cb < cb1; ++cb) {
    const int col = cb * 32 + cl;
    half8 bf[KS];
    const _Float16 *bsrc = b.bop + (size_t)col * K + 8 * h;
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) bf[kk] = *(const half8 *)(bsrc + 16 * kk);
    const float csa = b.col_sa[col];
    const float cdp = b.col_dp[col];

    f32x16 acc[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      acc[rb] = f32x16{};
#pragma unroll
      for (int kk = 0; kk < KS; ++kk)
        acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(af[rb][kk], bf[kk],
                                                         acc[rb], 0, 0, 0);
    }

    unsigned pm = 0;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int s = 2 * rb + e;
        float mx = acc[rb][8 * e], mn = mx;
#pragma unroll
        for (int k = 1; k < 8; ++k) {
          mx = fmaxf(mx, acc[rb][8 * e + k]);
          mn = fminf(mn, acc[rb][8 * e + k]);
        }
        const float a0 = fmaf(-csa, bbar[s], mx);
        const float a1 = fmaf(-csa, bbar[s], mn);
        const float mm = fmaxf(fabsf(a0), fabsf(a1));
        pm |= (mm * mm >= wp[s] * cdp) ? (1u << s) : 0u;
      }

    if (__any(pm != 0u)) {
      if (pm) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const int s = 2 * rb + e;
            if ((pm >> s) & 1u) {
              const int r = rbase + 4 * rb + 2 * h + e;
#pragma unroll
              for (int k = 0; k < 8; ++k) {
                const float v = acc[rb][8 * e + k];
                const float a = fmaf(-csa, bbar[s], v);
                if (a * a >= wp[s] * cdp) wp[s] = eval_survivor(v, col, r, k, g, b);
              }
            }
          }
      }
    }

    if ((cb & 7) == 7) {
#pragma unroll
      for (int s = 0; s < 2 * RB; ++s) {
        const int r = rbase + 4 * (s >> 1) + 2 * h + (s & 1);
        wp[s] = prune_weight(key_err(load_best(b, r), g), b.rng_sb[r],
                             b.rng_sbb[r], g);
      }
    }
  }
}

}  // namespace

hipError_t launch_search_mfma(const Geo &g, const EncBufs &b, int chunks,
                              hipStream_t st) {
  constexpr int RB = 2;
  static_assert(16 * RB == kMfmaRangesPerWG, "tile");
  const int cbpc = (g.NCB + chunks - 1) / chunks;
  const int nchunks = (g.NCB + cbpc - 1) / cbpc;
  dim3 grid(nchunks, g.R_pad / (16 * RB));
  if (g.bits != 8) return hipErrorInvalidValue;
  if (g.K == 64)
    hipLaunchKernelGGL((k_search_mfma_u8<64, RB>), grid, dim3(256), 0, st, g,
                       b, cbpc);
  else
    hipLaunchKernelGGL((k_search_mfma_u8<16, RB>), grid, dim3(256), 0, st, g,
                       b, cbpc);
  return hipGetLastError();
}

}  // namespace fic
