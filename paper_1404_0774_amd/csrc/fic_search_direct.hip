// fic_search_direct.hip -- the plain method: Alg. 3's per-candidate sums
// computed directly on the vector ALUs, with the operands staged in LDS.
//
// Each thread owns one range and four domain columns and accumulates the 32
// inner products sum_p Rop[(r, k), p] * Bop[d, p] (8 transforms x 4 domains)
// with scalar FP32 multiply-adds (exact: integers below 2^24).  The range
// tile (32 ranges x 8 transforms x K) stays in LDS for the workgroup's whole
// sweep; each 32-domain block is staged once and read by all 256 threads.
// The prune, exact fit and key update are the same as the matrix-core
// kernel's, so both produce identical codes.
#include <math.h>

#include "fic_device.h"

namespace fic {

namespace {

__device__ __noinline__ float eval_survivor_d(float Gf, int col, int r, int k,
                                              const Geo &g, const EncBufs &b) {
  const double SA = (double)b.col_sadp[col].x;
  const double SAA = b.col_saa[col];
  const double Sb = b.rng_sb[r], Sbb = b.rng_sbb[r];
  const long long d = b.col_dom[col];
  const Fit f = fit_exact((double)Gf, SA, SAA, Sb, Sbb, g);
  const unsigned long long key = make_key(f.err, 8 * d + k, g);
  const unsigned long long old = atomicMin(&b.best[r], key);
  const unsigned long long nb = key < old ? key : old;
  return prune_weight(key_err(nb, g), Sb, Sbb, g);
}

// grid: (chunks, R_pad / 32); block: 256 threads.  Thread t: range slot
// t / 8 of the tile, columns 4 (t mod 8) .. +3 of each 32-column block.
template <int K>
__global__ __launch_bounds__(256) void k_search_direct_u8(Geo g, EncBufs b,
                                                          int cb_begin,
                                                          int cb_per_chunk) {
  __shared__ __attribute__((aligned(16))) float As[K][256];  // [p][8 rs + k]
  __shared__ __attribute__((aligned(16))) float Bs[K][32];   // [p][column]
  const int t = threadIdx.x;
  const int rs = t >> 3, cg = t & 7;
  const int r0 = blockIdx.y * 32;
  const int r = r0 + rs;

  // stage the range tile (transposed so that a thread's 8 rows are adjacent)
  for (int i = t; i < 256 * K; i += 256) {
    const int row = i / K, p = i % K;
    As[p][row] = (float)b.aop[((size_t)r0 * 8 + row) * K + p];
  }
  const double Sb = b.rng_sb[r], Sbb = b.rng_sbb[r];
  const float bbar = (float)(Sb / K);
  float wp = prune_weight(key_err(b.best[r], g), Sb, Sbb, g);

  const int cb0 = cb_begin + blockIdx.x * cb_per_chunk;
  const int cb1 = min(cb0 + cb_per_chunk, g.NCB);
  for (int cb = cb0; cb < cb1; ++cb) {
    __syncthreads();
    for (int i = t; i < 32 * K; i += 256) {
      const int c = i / K, p = i % K;
      Bs[p][c] = (float)b.bop[((size_t)cb * 32 + c) * K + p];
    }
    __syncthreads();

    float acc[4][8];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int k = 0; k < 8; ++k) acc[c][k] = 0.0f;
#pragma unroll 4
    for (int p = 0; p < K; ++p) {
      const float4 a0 = *(const float4 *)&As[p][8 * rs];
      const float4 a1 = *(const float4 *)&As[p][8 * rs + 4];
      const float4 bv = *(const float4 *)&Bs[p][4 * cg];
      const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
      const float bw[4] = {bv.x, bv.y, bv.z, bv.w};
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[c][k] = fmaf(av[k], bw[c], acc[c][k]);
    }

#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int col = cb * 32 + 4 * cg + c;
      const float2 sadp = b.col_sadp[col];
      const float csa = sadp.x, cdp = sadp.y;
      float mx = acc[c][0], mn = mx;
#pragma unroll
      for (int k = 1; k < 8; ++k) {
        mx = fmaxf(mx, acc[c][k]);
        mn = fminf(mn, acc[c][k]);
      }
      const float a0 = fmaf(-csa, bbar, mx), a1 = fmaf(-csa, bbar, mn);
      const float mm = fmaxf(fabsf(a0), fabsf(a1));
      if (mm * mm >= wp * cdp) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const float a = fmaf(-csa, bbar, acc[c][k]);
          if (a * a >= wp * cdp) wp = eval_survivor_d(acc[c][k], col, r, k, g, b);
        }
      }
    }
    if ((cb & 7) == 7)
      wp = prune_weight(
          key_err(__hip_atomic_load(&b.best[r], __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT),
                  g),
          Sb, Sbb, g);
  }
}

// 12-bit plain method: grid (chunks, R_pad / 16); block 256 threads.  Thread
// t: range slot t / 16 of the tile, columns 2 (t mod 16), +1 of each block.
// Three exact FP32 partial sums per candidate (as in the matrix-core split:
// G = 8192 G_hh + 64 M + G_ll), rebuilt exactly in FP64 for the test.
template <int K>
__global__ __launch_bounds__(256) void k_search_direct_12(Geo g, EncBufs b,
                                                          int cb_begin,
                                                          int cb_per_chunk) {
  __shared__ __attribute__((aligned(16))) float Ah[K][128];  // [p][8 rs + k]
  __shared__ __attribute__((aligned(16))) float Al[K][128];
  __shared__ __attribute__((aligned(16))) float Bh[K][32];   // [p][column]
  __shared__ __attribute__((aligned(16))) float Bl[K][32];
  const int t = threadIdx.x;
  const int rs = t >> 4, cg = t & 15;
  const int r0 = blockIdx.y * 16;
  const int r = r0 + rs;
  const size_t aplane = (size_t)g.R_pad * 8 * K;
  const size_t bplane = (size_t)g.NC_pad * K;

  for (int i = t; i < 128 * K; i += 256) {
    const int row = i / K, p = i % K;
    const size_t o = ((size_t)r0 * 8 + row) * K + p;
    Ah[p][row] = (float)b.aop[o];
    Al[p][row] = (float)b.aop[aplane + o];
  }
  const double Sb = b.rng_sb[r], Sbb = b.rng_sbb[r];
  const double Kd = (double)g.K;
  float wp = prune_weight(key_err(b.best[r], g), Sb, Sbb, g);

  const int cb0 = cb_begin + blockIdx.x * cb_per_chunk;
  const int cb1 = min(cb0 + cb_per_chunk, g.NCB);
  for (int cb = cb0; cb < cb1; ++cb) {
    __syncthreads();
    for (int i = t; i < 32 * K; i += 256) {
      const int c = i / K, p = i % K;
      const size_t o = ((size_t)cb * 32 + c) * K + p;
      Bh[p][c] = (float)b.bop[o];
      Bl[p][c] = (float)b.bop[bplane + o];
    }
    __syncthreads();

    float hh[2][8], mid[2][8], ll[2][8];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int k = 0; k < 8; ++k) hh[c][k] = mid[c][k] = ll[c][k] = 0.0f;
#pragma unroll 2
    for (int p = 0; p < K; ++p) {
      const float4 h0 = *(const float4 *)&Ah[p][8 * rs];
      const float4 h1 = *(const float4 *)&Ah[p][8 * rs + 4];
      const float4 l0 = *(const float4 *)&Al[p][8 * rs];
      const float4 l1 = *(const float4 *)&Al[p][8 * rs + 4];
      const float2 bh = *(const float2 *)&Bh[p][2 * cg];
      const float2 bl = *(const float2 *)&Bl[p][2 * cg];
      const float ah[8] = {h0.x, h0.y, h0.z, h0.w, h1.x, h1.y, h1.z, h1.w};
      const float al[8] = {l0.x, l0.y, l0.z, l0.w, l1.x, l1.y, l1.z, l1.w};
      const float bhv[2] = {bh.x, bh.y}, blv[2] = {bl.x, bl.y};
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          hh[c][k] = fmaf(ah[k], bhv[c], hh[c][k]);
          ll[c][k] = fmaf(al[k], blv[c], ll[c][k]);
          mid[c][k] = fmaf(al[k], 2.0f * bhv[c], mid[c][k]);
          mid[c][k] = fmaf(ah[k], blv[c], mid[c][k]);
        }
    }

#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int col = cb * 32 + 2 * cg + c;
      const float2 sadp = b.col_sadp[col];
      const float cdp = sadp.y;
      const double csa = (double)sadp.x;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const double G = fma(8192.0, (double)hh[c][k],
                             fma(64.0, (double)mid[c][k], (double)ll[c][k]));
        const double a = G - csa * Sb / Kd;
        if (a * a >= (double)(wp * cdp)) {
          const Fit f = fit_exact(G, csa, b.col_saa[col], Sb, Sbb, g);
          const unsigned long long key =
              make_key(f.err, 8ll * b.col_dom[col] + k, g);
          const unsigned long long old = atomicMin(&b.best[r], key);
          wp = prune_weight(key_err(key < old ? key : old, g), Sb, Sbb, g);
        }
      }
    }
    if ((cb & 7) == 7)
      wp = prune_weight(
          key_err(__hip_atomic_load(&b.best[r], __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT),
                  g),
          Sb, Sbb, g);
  }
}

}  // namespace

hipError_t launch_search_direct(const Geo &g, const EncBufs &b, int chunks,
                                int first_block, hipStream_t st) {
  const int rest = g.NCB - first_block;
  if (rest <= 0) return hipSuccess;
  if (chunks > rest) chunks = rest;
  if (chunks < 1) chunks = 1;
  const int cbpc = (rest + chunks - 1) / chunks;
  const int nchunks = (rest + cbpc - 1) / cbpc;
  if (g.bits == 12) {
    const dim3 grid12(nchunks, g.R_pad / 16);
    if (g.K == 64)
      hipLaunchKernelGGL(k_search_direct_12<64>, grid12, dim3(256), 0, st, g,
                         b, first_block, cbpc);
    else
      hipLaunchKernelGGL(k_search_direct_12<16>, grid12, dim3(256), 0, st, g,
                         b, first_block, cbpc);
    return hipGetLastError();
  }
  dim3 grid(nchunks, g.R_pad / kDirectRangesPerWG);
  if (g.K == 64)
    hipLaunchKernelGGL(k_search_direct_u8<64>, grid, dim3(256), 0, st, g, b,
                       first_block, cbpc);
  else
    hipLaunchKernelGGL(k_search_direct_u8<16>, grid, dim3(256), 0, st, g, b,
                       first_block, cbpc);
  return hipGetLastError();
}

}  // namespace fic
