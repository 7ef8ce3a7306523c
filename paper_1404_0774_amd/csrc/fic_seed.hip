// fic_seed.hip -- a starting bound for every range before the search.
//
// The least-squares prune is only as tight as each range's best residual so
// far, and a cold start lets a large share of the first blocks' candidates
// through.  This kernel ranks every candidate of the first `nblocks` column
// blocks, spread over the whole GPU, and lowers each range's key with the
// exact residual of its top-ranked candidate.  (The search itself still
// covers these blocks.)
#include <limits.h>
#include <math.h>

#include "fic_device.h"

namespace fic {

namespace {

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));

// grid: R_pad / 8 workgroups; block: 256 threads.  Thread t owns row
// (range t / 32, transform (t / 4) mod 8) of the range operand and columns
// 8 (t mod 4) .. +7 of each 32-column block.  B12: 12-bit operands in two
// planes (b = 64 b_hi + b_lo, A = 128 A_hi + A_lo); the four partial sums
// are exact in FP32 and G is rebuilt exactly in FP64.  Both operands are
// staged in LDS as FP16 pairs.
//
// The seed only has to be some candidate's exact residual (any one is a
// valid bound), so candidates are ranked by their least-squares score
// N'^2 / D' in FP32 (the unquantised residual is (V - N'^2/D') / K), and
// only each range's top-ranked candidate is fitted exactly in FP64.
template <int K, bool B12>
__device__ __forceinline__ void seed_dense_body(const Geo &g, const EncBufs &b,
                                                int nblocks, int bid) {
  constexpr int KP = K / 2;                       // half2 pairs per row
  constexpr int NP = B12 ? 2 : 1;                 // operand planes
  constexpr int PER = K / 8;                      // 16-byte words per row
  __shared__ __attribute__((aligned(16))) half2_t sA[NP][KP][64];
  __shared__ __attribute__((aligned(16))) half2_t sB[NP][KP][32];
  __shared__ float s_sa[32], s_idp[32], s_dd[32];
  const int t = threadIdx.x;
  const int row = t >> 2, cgp = t & 3;
  const int rl = row >> 3, k = row & 7;
  const int r = bid * 8 + rl;

  const double Sb = b.rng_sb[r], Sbb = b.rng_sbb[r];
  const float sbf = (float)Sb;
  // centred 8-bit operands (g.ctr): N' = K H - (SA - K m_d)(Sb - K m_r)
  const float dr = fmaf(-(float)K, centre_f(sbf, 1.0f / K), sbf);
  // the workgroup's 64 rows (8 ranges x 8 transforms) of the range operand
  for (int i = t; nblocks > 0 && i < NP * 64 * PER; i += 256) {
    const int pl = i / (64 * PER), ii = i % (64 * PER);
    const int rw = ii / PER, p0 = (ii % PER) * 8;
    const half8_t v = *(const half8_t *)(b.aop + (size_t)pl * g.R_pad * 8 * K +
                                         ((size_t)bid * 64 + rw) * K + p0);
#pragma unroll
    for (int e = 0; e < 4; ++e)
      sA[pl][p0 / 2 + e][rw] = half2_t{v[2 * e], v[2 * e + 1]};
  }
  __syncthreads();

  float bscore = -1.0f;  // best N'^2 / D' seen by this thread
  float bg[NP * NP];     // its partial sums
  int bcol = -1;         // and its column
#pragma unroll
  for (int x = 0; x < NP * NP; ++x) bg[x] = 0.0f;

  for (int cb = 0; cb < nblocks; ++cb) {
    if (cb > 0) __syncthreads();
    for (int i = t; i < NP * 32 * PER; i += 256) {
      const int pl = i / (32 * PER), ii = i % (32 * PER);
      const int col = ii / PER, p0 = (ii % PER) * 8;
      const half8_t v = *(const half8_t *)(
          b.bop + (size_t)pl * g.NC_pad * K + bop_index(g, (long long)cb * 32 + col, p0));
#pragma unroll
      for (int e = 0; e < 4; ++e)
        sB[pl][p0 / 2 + e][col] = half2_t{v[2 * e], v[2 * e + 1]};
    }
    if (t < 32) {
      const float2 sadp = b.col_sadp[cb * 32 + t];
      s_sa[t] = sadp.x;
      s_dd[t] = fmaf(-(float)K, centre_f(sadp.x, 1.0f / K), sadp.x);
      // flat domains are seeded separately; padding columns are not domains
      s_idp[t] = sadp.y == __builtin_inff() ? -1.0f : 1.0f / sadp.y;
    }
    __syncthreads();

    // acc[x][y][c]: range plane x against domain plane y, column c
    float acc[NP][NP][8];
#pragma unroll
    for (int x = 0; x < NP; ++x)
#pragma unroll
      for (int y = 0; y < NP; ++y)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[x][y][c] = 0.0f;
#pragma unroll 4
    for (int pp = 0; pp < KP; ++pp) {
      half2_t av[NP];
#pragma unroll
      for (int x = 0; x < NP; ++x) av[x] = sA[x][pp][row];
#pragma unroll
      for (int y = 0; y < NP; ++y) {
        const half8_t b0 = *(const half8_t *)&sB[y][pp][8 * cgp];
        const half8_t b1 = *(const half8_t *)&sB[y][pp][8 * cgp + 4];
        const half2_t bv[8] = {half2_t{b0[0], b0[1]}, half2_t{b0[2], b0[3]},
                               half2_t{b0[4], b0[5]}, half2_t{b0[6], b0[7]},
                               half2_t{b1[0], b1[1]}, half2_t{b1[2], b1[3]},
                               half2_t{b1[4], b1[5]}, half2_t{b1[6], b1[7]}};
#pragma unroll
        for (int c = 0; c < 8; ++c)
#pragma unroll
          for (int x = 0; x < NP; ++x)
            acc[x][y][c] = __builtin_amdgcn_fdot2(av[x], bv[c], acc[x][y][c], false);
      }
    }

#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int cc = 8 * cgp + c;
      const float idp = s_idp[cc];
      // 12-bit: G = 8192 G_hh + 128 G_(A_hi b_lo) + 64 G_(A_lo b_hi) + G_ll
      const float gf = B12 ? fmaf(8192.0f, acc[0][0][c],
                                  fmaf(128.0f, acc[1][0][c],
                                       fmaf(64.0f, acc[0][NP - 1][c],
                                            acc[NP - 1][NP - 1][c])))
                           : acc[0][0][c];
      const float np = (!B12 && g.ctr) ? fmaf((float)g.K, gf, -s_dd[cc] * dr)
                                        : fmaf((float)g.K, gf, -s_sa[cc] * sbf);
      const float score = idp < 0.0f ? -1.0f : np * np * idp;
      if (score > bscore) {
        bscore = score;
        bcol = cb * 32 + cc;
#pragma unroll
        for (int x = 0; x < NP; ++x)
#pragma unroll
          for (int y = 0; y < NP; ++y) bg[x * NP + y] = acc[x][y][c];
      }
    }
  }

  // the top-ranked candidate of each range (8 transforms x 4 column groups =
  // 32 threads): the lowest thread holding the maximum fits it exactly
  float m = bscore;
#pragma unroll
  for (int o = 1; o < 32; o <<= 1) m = fmaxf(m, __shfl_xor(m, o, 32));
  const unsigned long long bal = __builtin_amdgcn_ballot_w64(bscore == m);
  const unsigned grp = (unsigned)(bal >> (t & 32));
  if ((t & 31) != __builtin_ctz(grp)) return;
  unsigned long long key = ~0ull;
  if (bcol >= 0) {
    const double G =
        B12 ? 8192.0 * bg[0] + 128.0 * bg[2] + 64.0 * bg[1] + (double)bg[3]
            : (g.ctr ? g_from_centred((double)bg[0], (double)b.col_sadp[bcol].x,
                                      Sb, g)
                     : (double)bg[0]);
    const Fit f = fit_exact(G, (double)b.col_sadp[bcol].x, b.col_saa[bcol],
                            Sb, Sbb, g);
    const unsigned long long k2 = make_key(f.err, 8ll * b.col_dom[bcol] + k, g);
    key = k2 < key ? k2 : key;
  }
  if (range_of_slot(g, r) < g.R && key < b.best[r]) b.best[r] = key;
}

template <int K, bool B12>
__global__ __launch_bounds__(256) void k_seed_dense(Geo g, EncBufs b,
                                                    int nblocks) {
  seed_dense_body<K, B12>(g, b, nblocks, blockIdx.x);
}

template <int K, bool B12>
__global__ __launch_bounds__(256) void k_seed_batch(BatchDev bd, int nblocks) {
  const int2 m = load_uniform(&bd.wg_map[bd.phase_base[2] + blockIdx.x]);
  const int nb = min(nblocks, load_uniform(&bd.tab[m.x].seed_blocks));
  const Geo g = load_uniform(&bd.tab[m.x].g);
  const EncBufs b = load_uniform(&bd.tab[m.x].b);
  seed_dense_body<K, B12>(g, b, nb, m.y);
}

}  // namespace

hipError_t launch_seed_batch(const BatchDev &bd, int nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  auto kern = bd.bits == 12 ? (bd.rsize == 8 ? k_seed_batch<64, true>
                                             : k_seed_batch<16, true>)
                            : (bd.rsize == 8 ? k_seed_batch<64, false>
                                             : k_seed_batch<16, false>);
  hipLaunchKernelGGL(kern, dim3(bd.phase_total[2]), dim3(256), 0, st, bd,
                     nblocks);
  return hipGetLastError();
}

hipError_t launch_seed_dense(const Geo &g, const EncBufs &b, int nblocks,
                             hipStream_t st) {
  if (nblocks <= 0 || g.K > 64) return hipSuccess;
  const dim3 grid(g.R_pad / 8);
  auto kern = g.bits == 12 ? (g.K == 64 ? k_seed_dense<64, true>
                                        : k_seed_dense<16, true>)
                           : (g.K == 64 ? k_seed_dense<64, false>
                                        : k_seed_dense<16, false>);
  hipLaunchKernelGGL(kern, grid, dim3(256), 0, st, g, b, nblocks);
  return hipGetLastError();
}

}  // namespace fic
