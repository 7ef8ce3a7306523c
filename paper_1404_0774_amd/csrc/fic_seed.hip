// fic_seed.hip -- dense exact evaluation of the first column blocks.
//
// Before the pruned search starts, every range needs a good best residual:
// the least-squares prune is only as tight as that bound, and a cold start
// lets a large share of the first block's candidates through.  This kernel
// fits every candidate of the first `nblocks` column blocks exactly (no
// prune), spread over the whole GPU, and lowers each range's seeded key.
// The sweep order puts a quasi-uniform sample of the image's domains in any
// prefix of columns, so one or two blocks already give a bound close to the
// final one.
#include <math.h>

#include "fic_device.h"

namespace fic {

namespace {

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));

// grid: R_pad / 8 workgroups; block: 256 threads.  Thread t owns row
// (range t / 32, transform (t / 4) mod 8) of the range operand and columns
// 8 (t mod 4) .. +7 of each 32-column block.
template <int K>
__global__ __launch_bounds__(256) void k_seed_dense_u8(Geo g, EncBufs b,
                                                       int nblocks) {
  constexpr int KP = K / 2;                       // half2 pairs per row
  __shared__ __attribute__((aligned(16))) half2_t sB[KP][32];
  __shared__ float s_sa[32], s_dp[32];
  __shared__ double s_saa[32];
  __shared__ int s_dom[32];
  const int t = threadIdx.x;
  const int row = t >> 2, cgp = t & 3;
  const int rl = row >> 3, k = row & 7;
  const int r = blockIdx.x * 8 + rl;

  half2_t a[KP];
  {
    const half8_t *src = (const half8_t *)(b.aop + ((size_t)r * 8 + k) * K);
#pragma unroll
    for (int i = 0; i < K / 8; ++i) {
      const half8_t v = src[i];
#pragma unroll
      for (int e = 0; e < 4; ++e) a[4 * i + e] = half2_t{v[2 * e], v[2 * e + 1]};
    }
  }
  const double Sb = b.rng_sb[r], Sbb = b.rng_sbb[r];
  unsigned long long best = ~0ull;

  for (int cb = 0; cb < nblocks; ++cb) {
    __syncthreads();
    {
      // stage the block: thread t loads 8 cell sums of column t / (K / 8)
      constexpr int PER = K / 8;
      for (int i = t; i < 32 * PER; i += 256) {
        const int col = i / PER, p0 = (i % PER) * 8;
        const half8_t v =
            *(const half8_t *)(b.bop + ((size_t)cb * 32 + col) * K + p0);
#pragma unroll
        for (int e = 0; e < 4; ++e)
          sB[p0 / 2 + e][col] = half2_t{v[2 * e], v[2 * e + 1]};
      }
      if (t < 32) {
        const int col = cb * 32 + t;
        s_sa[t] = b.col_sa[col];
        s_dp[t] = b.col_dp[col];
        s_saa[t] = b.col_saa[col];
        s_dom[t] = b.col_dom[col];
      }
    }
    __syncthreads();

    float acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.0f;
#pragma unroll
    for (int pp = 0; pp < KP; ++pp) {
      const half2_t *bp = &sB[pp][8 * cgp];
#pragma unroll
      for (int c = 0; c < 8; ++c)
        acc[c] = __builtin_amdgcn_fdot2(a[pp], bp[c], acc[c], false);
    }

#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int cc = 8 * cgp + c;
      // flat domains are seeded separately; padding columns are not domains
      if (s_dp[cc] == __builtin_inff()) continue;
      const Fit f = fit_exact((double)acc[c], (double)s_sa[cc], s_saa[cc], Sb,
                              Sbb, g);
      const unsigned long long key =
          make_key(f.err, 8ll * s_dom[cc] + k, g);
      best = key < best ? key : best;
    }
  }

  // minimum over the 32 threads (8 transforms x 4 column groups) of a range
#pragma unroll
  for (int o = 1; o < 32; o <<= 1) {
    const unsigned long long v = __shfl_xor(best, o, 32);
    best = v < best ? v : best;
  }
  if ((t & 31) == 0 && r < g.R && best < b.best[r]) b.best[r] = best;
}

}  // namespace

hipError_t launch_seed_dense(const Geo &g, const EncBufs &b, int nblocks,
                             hipStream_t st) {
  if (g.bits != 8) return hipErrorInvalidValue;
  if (nblocks <= 0) return hipSuccess;
  const dim3 grid(g.R_pad / 8);
  if (g.K == 64)
    hipLaunchKernelGGL(k_seed_dense_u8<64>, grid, dim3(256), 0, st, g, b,
                       nblocks);
  else
    hipLaunchKernelGGL(k_seed_dense_u8<16>, grid, dim3(256), 0, st, g, b,
                       nblocks);
  return hipGetLastError();
}

}  // namespace fic
