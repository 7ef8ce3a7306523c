// fic_search_direct.hip -- the plain method: Alg. 3's per-candidate sums
// computed directly on the vector ALUs, with the operands staged in LDS.
//
// Both walk the same lists of range slots and domain columns as the
// matrix-core kernels (all of them in a full search, those with variance
// otherwise), so the two methods evaluate the same candidates.
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

// The workgroup's share of the searched lists: entries [r0, r0 + nr) of the
// range-slot list (written to s_slot, -1 past its end) and column blocks
// [cb0, cb1) of the column list, from the list lengths read on the device.
// Returns false when the workgroup has nothing to do (uniform).
__device__ __forceinline__ bool direct_share(const EncBufs &b, int nr,
                                             int *s_slot, int &cb0, int &cb1) {
  const int nA = b.n_act[0], nD = b.n_act[1];
  const int r0 = blockIdx.y * nr;
  const int ncb = (nD + 31) / 32;
  const int cbpc = (ncb + (int)gridDim.x - 1) / (int)gridDim.x;
  cb0 = blockIdx.x * cbpc;
  cb1 = min(cb0 + cbpc, ncb);
  if (r0 >= nA || cb0 >= cb1) return false;
  if ((int)threadIdx.x < nr)
    s_slot[threadIdx.x] = r0 + (int)threadIdx.x < nA
                              ? b.act_slot[r0 + threadIdx.x] : -1;
  return true;
}

// Columns of searched block cb (-1 past the list) into s_col.
__device__ __forceinline__ void direct_columns(const EncBufs &b, int cb,
                                               int *s_col) {
  if (threadIdx.x < 32) {
    const int j = cb * 32 + (int)threadIdx.x;
    s_col[threadIdx.x] = j < b.n_act[1] ? b.act_col[j] : -1;
  }
}

// grid: (chunks, R_pad / 32); block: 256 threads.  Workgroup y takes entries
// 32 y .. 32 y + 31 of the searched range list; thread t owns entry t / 8 and
// columns 4 (t mod 8) .. +3 of each 32-column block of the searched column
// list.
template <int K>
__global__ __launch_bounds__(256) void k_search_direct_u8(Geo g, EncBufs b) {
  __shared__ __attribute__((aligned(16))) float As[K][256];  // [p][8 rs + k]
  __shared__ __attribute__((aligned(16))) float Bs[K][32];   // [p][column]
  __shared__ int s_slot[32], s_col[32];
  int cb0, cb1;
  if (!direct_share(b, 32, s_slot, cb0, cb1)) return;
  const int t = threadIdx.x;
  const int rs = t >> 3, cg = t & 7;
  __syncthreads();

  // stage the range tile (transposed so that a thread's 8 rows are adjacent)
  for (int i = t; i < 256 * K; i += 256) {
    const int row = i / K, p = i % K;
    const int sl = s_slot[row >> 3];
    As[p][row] =
        sl >= 0 ? (float)b.aop[((size_t)sl * 8 + (row & 7)) * K + p] : 0.0f;
  }
  const int r = s_slot[rs];
  double Sb = 0.0, Sbb = 0.0;
  float wp = __builtin_inff();  // no range: nothing passes
  if (r >= 0) {
    Sb = b.rng_sb[r];
    Sbb = b.rng_sbb[r];
    wp = prune_weight(key_err(b.best[r], g), Sb, Sbb, g);
  }
  const float bbar = (float)(Sb / K);

  for (int cb = cb0; cb < cb1; ++cb) {
    __syncthreads();
    direct_columns(b, cb, s_col);
    __syncthreads();
    for (int i = t; i < 32 * K; i += 256) {
      const int c = i / K, p = i % K;
      const int col = s_col[c];
      Bs[p][c] = col >= 0 ? (float)b.bop[(size_t)col * K + p] : 0.0f;
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
      const int col = s_col[4 * cg + c];
      // past the list: a flat column, which never passes
      const float2 sadp =
          col >= 0 ? b.col_sadp[col] : float2{0.0f, __builtin_inff()};
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
    if (((cb - cb0) & 7) == 7 && r >= 0)
      wp = prune_weight(
          key_err(__hip_atomic_load(&b.best[r], __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT),
                  g),
          Sb, Sbb, g);
  }
}

// 12-bit plain method: grid (chunks, R_pad / 16); block 256 threads.
// Workgroup y takes entries 16 y .. 16 y + 15 of the searched range list;
// thread t owns entry t / 16 and columns 2 (t mod 16), +1 of each block.
// Three exact FP32 partial sums per candidate (as in the matrix-core split:
// G = 8192 G_hh + 64 M + G_ll), rebuilt exactly in FP64 for the test.
template <int K>
__global__ __launch_bounds__(256) void k_search_direct_12(Geo g, EncBufs b) {
  __shared__ __attribute__((aligned(16))) float Ah[K][128];  // [p][8 rs + k]
  __shared__ __attribute__((aligned(16))) float Al[K][128];
  __shared__ __attribute__((aligned(16))) float Bh[K][32];   // [p][column]
  __shared__ __attribute__((aligned(16))) float Bl[K][32];
  __shared__ int s_slot[16], s_col[32];
  int cb0, cb1;
  if (!direct_share(b, 16, s_slot, cb0, cb1)) return;
  const int t = threadIdx.x;
  const int rs = t >> 4, cg = t & 15;
  const size_t aplane = (size_t)g.R_pad * 8 * K;
  const size_t bplane = (size_t)g.NC_pad * K;
  __syncthreads();

  for (int i = t; i < 128 * K; i += 256) {
    const int row = i / K, p = i % K;
    const int sl = s_slot[row >> 3];
    const size_t o = ((size_t)(sl >= 0 ? sl : 0) * 8 + (row & 7)) * K + p;
    Ah[p][row] = sl >= 0 ? (float)b.aop[o] : 0.0f;
    Al[p][row] = sl >= 0 ? (float)b.aop[aplane + o] : 0.0f;
  }
  const int r = s_slot[rs];
  double Sb = 0.0, Sbb = 0.0;
  float wp = __builtin_inff();  // no range: nothing passes
  if (r >= 0) {
    Sb = b.rng_sb[r];
    Sbb = b.rng_sbb[r];
    wp = prune_weight(key_err(b.best[r], g), Sb, Sbb, g);
  }
  const double Kd = (double)g.K;

  for (int cb = cb0; cb < cb1; ++cb) {
    __syncthreads();
    direct_columns(b, cb, s_col);
    __syncthreads();
    for (int i = t; i < 32 * K; i += 256) {
      const int c = i / K, p = i % K;
      const int col = s_col[c];
      const size_t o = (size_t)(col >= 0 ? col : 0) * K + p;
      Bh[p][c] = col >= 0 ? (float)b.bop[o] : 0.0f;
      Bl[p][c] = col >= 0 ? (float)b.bop[bplane + o] : 0.0f;
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
      const int col = s_col[2 * cg + c];
      if (col < 0) continue;  // past the list
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
    if (((cb - cb0) & 7) == 7 && r >= 0)
      wp = prune_weight(
          key_err(__hip_atomic_load(&b.best[r], __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT),
                  g),
          Sb, Sbb, g);
  }
}

}  // namespace

hipError_t launch_search_direct(const Geo &g, const EncBufs &b, int chunks,
                                hipStream_t st) {
  // the lists' lengths are read on the device: the grid covers the longest
  // possible lists and workgroups past them leave at once
  if (chunks > g.NCB) chunks = g.NCB;
  if (chunks < 1) chunks = 1;
  if (g.bits == 12) {
    const dim3 grid12(chunks, g.R_pad / 16);
    if (g.K == 64)
      hipLaunchKernelGGL(k_search_direct_12<64>, grid12, dim3(256), 0, st, g,
                         b);
    else
      hipLaunchKernelGGL(k_search_direct_12<16>, grid12, dim3(256), 0, st, g,
                         b);
    return hipGetLastError();
  }
  dim3 grid(chunks, g.R_pad / kDirectRangesPerWG);
  if (g.K == 64)
    hipLaunchKernelGGL(k_search_direct_u8<64>, grid, dim3(256), 0, st, g, b);
  else
    hipLaunchKernelGGL(k_search_direct_u8<16>, grid, dim3(256), 0, st, g, b);
  return hipGetLastError();
}

}  // namespace fic
