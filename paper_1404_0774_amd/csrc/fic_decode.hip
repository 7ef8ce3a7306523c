// fic_decode.hip -- iterating the partitioned IFS map (eq. 6) and its
// reverse-mode derivative with respect to the contrast s and offset o.
//
// Forward: one thread per output pixel,
//   x_{t+1}[p] = s_r * ((x00 + x01) + (x10 + x11)) * 0.25 + o_r
// where p is pixel (i, j) of range r and x.. is the 2x2 cell sigma_k(i, j)
// of the range's domain in x_t; one launch per iteration, or for small
// images one launch per three iterations with the intermediate values a
// pixel needs recomputed.
//
// Reverse: with g_{t+1} = dL/dx_{t+1} and u_t[p] the cell mean read by p,
//   dL/ds_r += sum_{p in r} g_{t+1}[p] u_t[p],  dL/do_r += sum_{p in r} g_{t+1}[p]
//   g_t[q]   = sum over range pixels p whose cell contains q of s_r g_{t+1}[p] / 4.
// The last sum is a gather, never a float atomic.  A table lists, for every
// domain, the ranges that use it in increasing range order (a stable sort of
// the range -> domain map, in one workgroup's LDS when it fits).  The gather
// runs over units (the 2x2 cells of an even domain grid, else pixels): a
// padded table holds each light unit's (pixel, weight) entries, and each
// heavy unit (a domain shared by many ranges, such as flat background) gets
// a workgroup of its own.  One launch per reverse step does the heavy units,
// dL/ds and dL/do, and the light units; every sum has a fixed order, so the
// result is bitwise reproducible.
#include <algorithm>
#include <utility>

#include "fic_device.h"

namespace fic {

namespace {

// Code entries come from the caller: keep every access inside the image even
// for out-of-range values (those ranges then decode from the clamped domain).
__device__ __forceinline__ int clamp_dom(int d, int nd) {
  return d < 0 ? 0 : (d >= nd ? nd - 1 : d);
}

// One iteration for ranges of side N (4 or 8), a workgroup per RPW = 256 / N
// consecutive ranges of one image.  Phase 1: thread (range, a) pools cell row
// a of the range's domain, reading two image rows of 2N floats (16-byte loads
// when V = 4), into LDS.  Phase 2: thread (row i, range) writes row i of the
// range, pixel (i, j) = s * pooled[sigma_k(i, j)] + o, adjacent threads
// writing adjacent ranges.  Pooling and the affine step are the expressions
//   u = ((x00 + x01) + (x10 + x11)) * 0.25,  x' = fma(s, u, o)
// for every pixel, whatever the launch shape.
//
// Batches: image b (of gridDim.x / wpi) has its codes at entry b R and its
// iterates t and t + 1 at xs + b xstride and ys + b xstride.  With xcd_map,
// workgroup L takes virtual workgroup (L mod 8) G/8 + L/8 (G a multiple of
// 8): workgroups go to the 8 XCDs in turn, so each XCD then holds a run of
// whole images and reads iterate t from the L2 that wrote it.
//
// MODE 0: one iteration, x_{t+1} at ys from x_t at xs.  MODE 1: the first
// iteration from the constant start x0, with no reads of an iterate: every
// cell pools to u0 (the same expression on four x0); the launch writes
// x_0 = x0 (at xs) and x_1 (at ys) over its ranges.  MODE 2: the first two
// iterations: as MODE 1, and x_2 (at ys + tstride) from x_1, whose pixels
// phase 1 forms from the codes of the ranges holding them, fma(s, u0, o),
// the value MODE 1 writes, so the result is bitwise that of two launches.
template <int N, int V, int MODE>
__global__ __launch_bounds__(256) void k_decode_pool(
    Geo g, int wpi, int xcd_map, const int32_t *domain, const uint8_t *iso,
    const float *s, const float *o, const float *xs, float *ys,
    long long xstride, long long tstride, float x0) {
  constexpr int RPW = 256 / N;
  constexpr int PS = N * N + 1;  // padded: phase 2 reads at stride PS
  __shared__ float pool[RPW * PS];
  const int L = blockIdx.x;
  const int v = xcd_map ? (L & 7) * (int)(gridDim.x >> 3) + (L >> 3) : L;
  const int b = v / wpi;
  const int r0 = (v - b * wpi) * RPW;
  const size_t cb = (size_t)b * g.R;
  const float *x = xs + (size_t)b * xstride;
  float *y = ys + (size_t)b * xstride;
  const float u0c = ((x0 + x0) + (x0 + x0)) * 0.25f;
  if constexpr (MODE != 1) {
    const int rl = threadIdx.x / N, a = threadIdx.x % N;
    const int r = r0 + rl;
    if (r < g.R) {
      const int d = clamp_dom(domain[cb + r], g.ND);
      const int Y = (d / g.NX) * g.step, X = (d % g.NX) * g.step;
      float u0[2 * N], u1[2 * N];
      if constexpr (MODE == 2) {
        // x_1 at the two cell rows: fma(s, u0, o) of the range holding each
        // pixel; a row's 2N pixels meet at most three ranges (the two rows
        // can lie in different rows of ranges when STEP is odd)
        const size_t ra = cb + (size_t)((Y + 2 * a) / N) * g.RW;
        const size_t rb = cb + (size_t)((Y + 2 * a + 1) / N) * g.RW;
        const int rx0 = X / N;
        float va[3], vb[3];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          const int rx = min(rx0 + e, g.RW - 1);
          va[e] = fmaf(s[ra + rx], u0c, o[ra + rx]);
          vb[e] = fmaf(s[rb + rx], u0c, o[rb + rx]);
        }
#pragma unroll
        for (int q = 0; q < 2 * N; ++q) {
          const int e = (X + q) / N - rx0;
          u0[q] = e == 0 ? va[0] : (e == 1 ? va[1] : va[2]);
          u1[q] = e == 0 ? vb[0] : (e == 1 ? vb[1] : vb[2]);
        }
      } else {
        const float *p0 = x + (size_t)(Y + 2 * a) * g.W + X;
        const float *p1 = p0 + g.W;
        if constexpr (V == 4) {
#pragma unroll
          for (int q = 0; q < 2 * N; q += 4) {
            const float4 e = *(const float4 *)(p0 + q);
            const float4 f = *(const float4 *)(p1 + q);
            u0[q] = e.x; u0[q + 1] = e.y; u0[q + 2] = e.z; u0[q + 3] = e.w;
            u1[q] = f.x; u1[q + 1] = f.y; u1[q + 2] = f.z; u1[q + 3] = f.w;
          }
        } else {
#pragma unroll
          for (int q = 0; q < 2 * N; ++q) {
            u0[q] = p0[q];
            u1[q] = p1[q];
          }
        }
      }
#pragma unroll
      for (int c = 0; c < N; ++c)
        pool[rl * PS + a * N + c] =
            ((u0[2 * c] + u0[2 * c + 1]) + (u1[2 * c] + u1[2 * c + 1])) * 0.25f;
    }
  }
  if constexpr (MODE != 1) __syncthreads();
  {
    const int i = threadIdx.x / RPW, rl = threadIdx.x % RPW;
    const int r = r0 + rl;
    if (r < g.R) {
      const int k = iso[cb + r];
      const float sv = s[cb + r], ov = o[cb + r];
      const int ry = r / g.RW, rx = r - ry * g.RW;
      float out[N], first[N];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        first[j] = fmaf(sv, u0c, ov);  // x_1 (MODES 1 and 2)
        if constexpr (MODE != 1) {
          int si, sj;
          sigma(k, i, j, N - 1, si, sj);
          out[j] = fmaf(sv, pool[rl * PS + si * N + sj], ov);
        } else {
          out[j] = first[j];
        }
      }
      const size_t off = (size_t)(ry * N + i) * g.W + rx * N;
      // MODE 0: y gets x_{t+1}.  MODE 1: x gets x_0, y x_1.  MODE 2: x gets
      // x_0, y x_1, y + tstride x_2 (x_0 and x_1 are written, never read).
      float *q = MODE == 2 ? y + tstride + off : y + off;
      float *q0 = (float *)x + off;
      float *q1 = y + off;
      if constexpr (V == 4) {
#pragma unroll
        for (int j = 0; j < N; j += 4) {
          *(float4 *)(q + j) = float4{out[j], out[j + 1], out[j + 2], out[j + 3]};
          if constexpr (MODE != 0) *(float4 *)(q0 + j) = float4{x0, x0, x0, x0};
          if constexpr (MODE == 2)
            *(float4 *)(q1 + j) =
                float4{first[j], first[j + 1], first[j + 2], first[j + 3]};
        }
      } else {
#pragma unroll
        for (int j = 0; j < N; ++j) {
          q[j] = out[j];
          if constexpr (MODE != 0) q0[j] = x0;
          if constexpr (MODE == 2) q1[j] = first[j];
        }
      }
    }
  }
}

// Any range size n (a decode at another scale): one thread per output pixel.
// MODE as k_decode_pool's: 0 one iteration (x -> y); 1 the first from the
// constant x0 (writes x_0 at x and x_1 at y, reads no iterate); 2 the first
// two (also x_2 at y + tstride, from x_1 at the cell's four pixels formed
// from the codes of the ranges holding them, the values MODE 1 writes).
template <int MODE>
__global__ void k_decode_step_any(DecGeo d, const int32_t *domain,
                                  const uint8_t *iso, const float *s,
                                  const float *o, float *x, float *y,
                                  long long tstride, float x0) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= d.H * d.W) return;
  const int py = p / d.W, px = p % d.W;
  const int ry = py / d.n, rx = px / d.n, i = py % d.n, j = px % d.n;
  const int r = ry * d.RW + rx;
  const float u0c = ((x0 + x0) + (x0 + x0)) * 0.25f;
  float u = u0c;
  if constexpr (MODE != 1) {
    const int dm = clamp_dom(domain[r], d.ND);
    int si, sj;
    sigma(iso[r], i, j, d.n - 1, si, sj);
    const int cy = (dm / d.NX) * d.step + 2 * si;
    const int cx = (dm % d.NX) * d.step + 2 * sj;
    if constexpr (MODE == 0) {
      const float *c = x + (size_t)cy * d.W + cx;
      u = ((c[0] + c[1]) + (c[d.W] + c[d.W + 1])) * 0.25f;
    } else {
      auto x1 = [&](int yy, int xx) {
        const int rr = (yy / d.n) * d.RW + xx / d.n;
        return fmaf(s[rr], u0c, o[rr]);
      };
      u = ((x1(cy, cx) + x1(cy, cx + 1)) + (x1(cy + 1, cx) + x1(cy + 1, cx + 1))) *
          0.25f;
    }
  }
  const float v = fmaf(s[r], u, o[r]);
  if constexpr (MODE == 0) {
    y[p] = v;
  } else if constexpr (MODE == 1) {
    x[p] = x0;
    y[p] = v;
  } else {
    x[p] = x0;
    y[p] = fmaf(s[r], u0c, o[r]);
    y[tstride + p] = v;
  }
}

// traj[b][0] = x0 for every image b: blockIdx.y is the image.
__global__ void k_fill_first_batch(float *traj, int HW, long long stride,
                                   float v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < HW) traj[(size_t)blockIdx.y * stride + i] = v;
}

__global__ void k_fill_f32(float *p, long long n, float v) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Pointer p moved by `bytes` (per-image offsets of batched calls).
template <class T>
__device__ __forceinline__ T *bump(T *p, long long bytes) {
  return reinterpret_cast<T *>(reinterpret_cast<uintptr_t>(p) + bytes);
}

// --- the domain -> ranges table --------------------------------------------
//
// srt[e], e < R: the ranges sorted by domain, in increasing range order within
// a domain (a stable sort of the range -> domain map); domain d's entries are
// srt[off[d] .. off[d + 1]).  Built once per set of domains.

// Number of entries of the sorted keys key[0 .. n) below v.
__device__ __forceinline__ int lower_bound(const int32_t *key, int n, int v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (key[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// off[0 .. ND] from the ranges sorted by domain (a binary search per domain
// instead of counting with atomics, which would queue up on a domain that
// thousands of ranges share).
__global__ void k_bounds(Geo g, const int32_t *sorted, int32_t *off) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d <= g.ND) off[d] = lower_bound(sorted, g.R, d);
}

// Exclusive scan of in[i], i < n, into out[0..n]; one workgroup of 1024
// threads, each owning a contiguous slice.
__global__ __launch_bounds__(1024) void k_scan(const int32_t *in, int n,
                                               int32_t *out) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int b0 = min(t * per, n), b1 = min(b0 + per, n);
  int s = 0;
  for (int i = b0; i < b1; ++i) s += in[i];
  part[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = t ? part[t - 1] : 0;
  for (int i = b0; i < b1; ++i) {
    out[i] = run;
    run += in[i];
  }
  if (t == 1023) out[n] = part[1023];
}

// Large tables: stable LSD radix sort of (domain, range) pairs by domain, 8
// bits a pass, blocks of 256 pairs: block histograms, one scan, stable
// scatter.  k_rs_init also clears the heavy-unit count.
__global__ void k_rs_init(Geo g, const int32_t *domain, int32_t *key,
                          int32_t *val, int32_t *nheavy) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r == 0) *nheavy = 0;
  if (r >= g.R) return;
  key[r] = clamp_dom(domain[r], g.ND);
  val[r] = r;
}

__global__ __launch_bounds__(256) void k_rs_hist(const int32_t *key, int n,
                                                 int shift, int32_t *hist) {
  __shared__ int h[256];
  const int t = threadIdx.x, i = blockIdx.x * 256 + t;
  h[t] = 0;
  __syncthreads();
  if (i < n) atomicAdd(&h[(key[i] >> shift) & 255], 1);
  __syncthreads();
  hist[t * gridDim.x + blockIdx.x] = h[t];  // digit-major
}

__global__ __launch_bounds__(256) void k_rs_scatter(const int32_t *kin,
                                                    const int32_t *vin, int n,
                                                    int shift,
                                                    const int32_t *base,
                                                    int32_t *kout,
                                                    int32_t *vout) {
  __shared__ int dig[256];
  const int t = threadIdx.x, i = blockIdx.x * 256 + t;
  const int k = i < n ? kin[i] : 0;
  const int dg = i < n ? (k >> shift) & 255 : -1;
  dig[t] = dg;
  __syncthreads();
  if (i >= n) return;
  int rank = 0;
  for (int j = 0; j < t; ++j) rank += dig[j] == dg;
  const int pos = base[dg * gridDim.x + blockIdx.x] + rank;
  kout[pos] = k;
  vout[pos] = vin[i];
}

// Small tables (R <= kSortR, ND <= kSortND): the whole sort in one
// workgroup, in LDS.  Keys (domain << kRBits) | range, stable LSD passes of
// at most 6 bits over the domain bits.  Wave w owns keys [w C, (w + 1) C) in
// rounds of 64; a key's rank among the earlier keys of its wave with the
// same digit comes from the digit's bits as ballots (the lanes agreeing on
// every bit), plus the wave's running count of that digit in LDS.  The
// counts, scanned digit-major and wave-minor, give every key its place:
// equal digits keep their order, so the sort is stable and its result is
// fixed.  Then off[d] by binary search over the sorted keys.
constexpr int kSortR = 8192;
constexpr int kSortND = 16384;
constexpr int kRBits = 13;  // kSortR = 2^kRBits

// Inclusive scan (sum, or minimum when MIN) across the 64 lanes of a wave:
// shifts by 1, 2, 4, 8 within rows of 16 lanes, then each row takes the
// last lane of the row before (row broadcasts 15 and 31).  Lanes without a
// source take the identity.
template <bool MIN>
__device__ __forceinline__ int wave_scan(int v) {
  const int id = MIN ? 0x7fffffff : 0;
  int x;
#define FIC_SCAN_STEP(ctrl, rows)                                      \
  x = __builtin_amdgcn_update_dpp(id, v, ctrl, rows, 0xf, false);     \
  v = MIN ? min(v, x) : v + x;
  FIC_SCAN_STEP(0x111, 0xf)  // row_shr:1
  FIC_SCAN_STEP(0x112, 0xf)  // row_shr:2
  FIC_SCAN_STEP(0x114, 0xf)  // row_shr:4
  FIC_SCAN_STEP(0x118, 0xf)  // row_shr:8
  FIC_SCAN_STEP(0x142, 0xa)  // row_bcast:15 into rows 1 and 3
  FIC_SCAN_STEP(0x143, 0xc)  // row_bcast:31 into rows 2 and 3
#undef FIC_SCAN_STEP
  return v;
}

// off[c0 + q] = min(st[c0 + q ..]), chunk c0 = (1023 - t) per of P >= per
// entries a thread: the chunk's own suffix minima, then a forward minimum
// scan over the threads (the later chunks).
template <int P>
__device__ __forceinline__ void suffix_min_off(const int *st, int n1, int per,
                                               int R, int t, int *wtot,
                                               int32_t *off) {
  const int lane = t & 63, w = t >> 6;
  const int c0 = (1023 - t) * per;
  int sv[P];
#pragma unroll
  for (int q = 0; q < P; ++q) sv[q] = q < per && c0 + q < n1 ? st[c0 + q] : R;
#pragma unroll
  for (int q = P - 2; q >= 0; --q) sv[q] = min(sv[q], sv[q + 1]);
  const int inc = wave_scan<true>(sv[0]);
  if (lane == 63) wtot[w] = inc;
  __syncthreads();
  int later = R;
#pragma unroll
  for (int y = 0; y < 15; ++y) later = y < w ? min(later, wtot[y]) : later;
  const int prev = __shfl_up(inc, 1);
  if (lane > 0) later = min(later, prev);
#pragma unroll
  for (int q = 0; q < P; ++q)
    if (q < per && c0 + q < n1) off[c0 + q] = min(sv[q], later);
}

// Batches: image blockIdx.y reads its codes at domain + y R and writes its
// table ws_stride bytes after the previous image's.
__global__ __launch_bounds__(1024) void k_sort_small(Geo g,
                                                     const int32_t *domain,
                                                     int32_t *srt, int32_t *off,
                                                     int32_t *nheavy,
                                                     long long ws_stride) {
  __shared__ uint32_t kb[2][kSortR];
  __shared__ int st[kSortND + 1];  // first sorted position of each domain
  __shared__ int cnt[16 * 64];     // [wave][digit], then the digits' bases
  __shared__ unsigned long long msk[16 * 64];  // [wave][digit]: lanes of a round
  __shared__ int wtot[16];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int R = g.R;
  domain += (size_t)blockIdx.y * R;
  srt = bump(srt, blockIdx.y * ws_stride);
  off = bump(off, blockIdx.y * ws_stride);
  nheavy = bump(nheavy, blockIdx.y * ws_stride);
  if (t == 0) *nheavy = 0;
  msk[t] = 0;
  {
    int dv[kSortR / 1024];  // all loads in flight before the first store
#pragma unroll
    for (int u = 0; u < kSortR / 1024; ++u)
      dv[u] = t + 1024 * u < R ? domain[t + 1024 * u] : 0;
#pragma unroll
    for (int u = 0; u < kSortR / 1024; ++u)
      if (t + 1024 * u < R)
        kb[0][t + 1024 * u] = ((uint32_t)clamp_dom(dv[u], g.ND) << kRBits) |
                              (uint32_t)(t + 1024 * u);
  }
  int bits = 0;
  while ((1 << bits) < g.ND) ++bits;
  const int np = (bits + 5) / 6;
  const int wd = np ? (bits + np - 1) / np : 0;
  const int C = (R + 15) >> 4;  // keys per wave, <= 512
  int cur = 0;
  for (int p = 0; p < np; ++p) {
    const int sh = kRBits + p * wd, D = 1 << wd;
    cnt[t] = 0;
    __syncthreads();
    uint32_t v[8];
    int dg[8], loc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {  // the wave's keys, all reads in flight
      const int ci = j * 64 + lane, i = w * C + ci;
      const bool valid = ci < C && i < R;
      v[j] = valid ? kb[cur][i] : 0;
      dg[j] = valid ? (int)((v[j] >> sh) & (uint32_t)(D - 1)) : -1;
      loc[j] = 0;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j * 64 < C && dg[j] >= 0) {  // j * 64 < C: the same for the wave
        // the lanes with this digit: each ORs its bit into the digit's mask
        // (one instruction for the wave; a wave's LDS operations complete in
        // order, so the read after it sees every lane's bit)
        const int a = w * 64 + dg[j];
        atomicOr(&msk[a], 1ull << lane);
        const uint64_t m = msk[a];
        const int base = cnt[a];
        const int below = __builtin_amdgcn_mbcnt_hi(
            (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
        loc[j] = base + below;
        if (below == 0) {  // the digit's first lane: count and clear
          cnt[a] = base + __popcll(m);
          msk[a] = 0;
        }
      }
    }
    __syncthreads();
    // exclusive scan of the counts, digit q and wave x at position 16 q + x
    const int q = t >> 4, x = t & 15;
    const int val = q < D ? cnt[x * 64 + q] : 0;
    const int inc = wave_scan<false>(val);
    if (lane == 63) wtot[w] = inc;
    __syncthreads();
    int pre = 0;
#pragma unroll
    for (int y = 0; y < 15; ++y) pre += y < w ? wtot[y] : 0;
    if (q < D) cnt[x * 64 + q] = pre + inc - val;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (dg[j] >= 0) kb[cur ^ 1][cnt[w * 64 + dg[j]] + loc[j]] = v[j];
    cur ^= 1;
    __syncthreads();
  }
  __syncthreads();  // with no pass (one domain), after the key loads
  const uint32_t *ks = kb[cur];
  for (int i = t; i < R; i += 1024)
    srt[i] = (int)(ks[i] & ((1u << kRBits) - 1));
  // off[d]: st[d] = the first sorted position of domain d (R if absent),
  // then off[d] = the minimum of st over d' >= d.  Thread t takes chunk
  // 1023 - t of per entries, so a forward minimum scan over the threads is a
  // minimum over the later chunks.
  const int n1 = g.ND + 1;
  for (int d = t; d < n1; d += 1024) st[d] = R;
  __syncthreads();
  for (int i = t; i < R; i += 1024) {
    const uint32_t dk = ks[i] >> kRBits;
    if (i == 0 || (ks[i - 1] >> kRBits) != dk) st[dk] = i;
  }
  __syncthreads();
  const int per = (n1 + 1023) >> 10;
  if (per <= 4)
    suffix_min_off<4>(st, n1, per, R, t, wtot, off);
  else
    suffix_min_off<(kSortND + 1 + 1023) / 1024>(st, n1, per, R, t, wtot, off);
}

// --- per-unit tables --------------------------------------------------------
//
// The reverse step's gather works on units: 2x2 pixel blocks when STEP is
// even (every cell of every domain is then such a block, and its four pixels
// receive the same sum), single pixels when STEP is odd.  A unit is covered
// by the domains dy0..dy1 x dx0..dx1; its entries are those domains' lists
// in that order (row-major), each list in range order.  A unit with at most
// kEll entries is light: its entries (pixel p read by the range, weight
// s_r / 4) sit in a padded table, slot pairs as planes of U int4, padding
// pixel -1.  A heavier unit is marked -2 in slot 0 and listed in heavy[],
// with the bounds of its covering lists when at most 2 x 2 domains cover a
// unit (STEP >= n).

constexpr int kEll = 16;

__device__ __forceinline__ size_t ell_at(int slot, int u, int U) {
  return ((size_t)(slot >> 1) * U + u) * 2 + (slot & 1);
}

// Domains covering pixel (qy, qx) (for a 2x2 unit at even (qy, qx) and an
// even STEP, exactly those covering the whole unit).
__device__ __forceinline__ void cover(const Geo &g, int qy, int qx, int &dy0,
                                      int &dy1, int &dx0, int &dx1) {
  const int span = 2 * g.n;
  const int ly = qy - span + 1, lx = qx - span + 1;
  dy0 = ly <= 0 ? 0 : (ly + g.step - 1) / g.step;
  dx0 = lx <= 0 ? 0 : (lx + g.step - 1) / g.step;
  dy1 = min(qy / g.step, g.NY - 1);
  dx1 = min(qx / g.step, g.NX - 1);
}

struct UnitArgs {
  Geo g;
  const int32_t *domain, *srt, *off;
  const uint8_t *iso;
  const float *s;
  int2 *ell;
  int32_t *pk, *heavy, *nheavy;
  int4 *hbeg, *hlen;
  float *pw;
  int U, UW, nbu;
  long long ws_stride;  // bytes between images' tables (batches)
};

// Workgroups [0, nbu): one thread per unit, padding or the heavy mark (these
// depend on the domains only).  The rest: one thread per (list entry e,
// domain cell c): the entry's slot in the units that cell covers, and for
// c = 0 the entry's packed range (top-left pixel << 3 | transform) and
// weight s_r / 4 for the heavy units.
template <int N, int UNIT>
__global__ __launch_bounds__(256) void k_adj_units(UnitArgs a) {
  const Geo &g = a.g;
  if (blockIdx.y > 0) {  // image blockIdx.y of a batch
    const long long wb = blockIdx.y * a.ws_stride;
    const size_t rb = (size_t)blockIdx.y * g.R;
    a.domain += rb;
    a.iso += rb;
    a.s += rb;
    a.srt = bump(a.srt, wb);
    a.off = bump(a.off, wb);
    a.ell = bump(a.ell, wb);
    a.pk = bump(a.pk, wb);
    a.heavy = bump(a.heavy, wb);
    a.nheavy = bump(a.nheavy, wb);
    a.hbeg = bump(a.hbeg, wb);
    a.hlen = bump(a.hlen, wb);
    a.pw = bump(a.pw, wb);
  }
  if ((int)blockIdx.x < a.nbu) {
    const int u = blockIdx.x * 256 + threadIdx.x;
    if (u >= a.U) return;
    const int qy = (u / a.UW) * UNIT, qx = (u % a.UW) * UNIT;
    int dy0, dy1, dx0, dx1;
    cover(g, qy, qx, dy0, dy1, dx0, dx1);
    int E = 0;
    for (int dy = dy0; dy <= dy1; ++dy)
      for (int dx = dx0; dx <= dx1; ++dx) {
        const int d = dy * g.NX + dx;
        E += a.off[d + 1] - a.off[d];
      }
    if (E <= kEll) {
      for (int sl = E; sl < kEll; ++sl) a.ell[ell_at(sl, u, a.U)] = int2{-1, 0};
    } else {
      a.ell[ell_at(0, u, a.U)] = int2{-2, 0};
      const int h = atomicAdd(a.nheavy, 1);
      a.heavy[h] = u;
      if (g.step >= g.n) {  // at most 2 x 2 covering domains: their lists
        int b4[4], l4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int dy = dy0 + (q >> 1), dx = dx0 + (q & 1);
          const bool ok = dy <= dy1 && dx <= dx1;
          const int d = ok ? dy * g.NX + dx : 0;
          b4[q] = ok ? a.off[d] : 0;
          l4[q] = ok ? a.off[d + 1] - b4[q] : 0;
        }
        a.hbeg[h] = int4{b4[0], b4[1], b4[2], b4[3]};
        a.hlen[h] = int4{l4[0], l4[1], l4[2], l4[3]};
      }
    }
    return;
  }
  constexpr int K = N * N;
  const int tid = (blockIdx.x - a.nbu) * 256 + threadIdx.x;
  const int e = tid / K, c = tid % K;
  if (e >= g.R) return;
  const int r = min(max(a.srt[e], 0), g.R - 1);
  const int d = clamp_dom(a.domain[r], g.ND), k = a.iso[r];
  const float w = a.s[r] * 0.25f;
  const int ci = c / N, cj = c % N;
  int i, j;
  sigma_inv(k, ci, cj, N - 1, i, j);
  const int ry = r / g.RW, rx = r % g.RW;
  const int pbase = (ry * N) * g.W + rx * N;
  if (c == 0) {
    a.pk[e] = (pbase << 3) | k;
    a.pw[e] = w;
  }
  const int p = pbase + i * g.W + j;
  const int ddy = d / g.NX, ddx = d % g.NX;
  const int Y = ddy * g.step + 2 * ci, X = ddx * g.step + 2 * cj;
#pragma unroll
  for (int sub = 0; sub < (UNIT == 1 ? 4 : 1); ++sub) {
    const int qy = Y + (sub >> 1), qx = X + (sub & 1);
    int dy0, dy1, dx0, dx1;
    cover(g, qy, qx, dy0, dy1, dx0, dx1);
    int pre = 0, E = 0;
    for (int dy = dy0; dy <= dy1; ++dy)
      for (int dx = dx0; dx <= dx1; ++dx) {
        const int dd = dy * g.NX + dx;
        const int b = a.off[dd], L = a.off[dd + 1] - b;
        if (dy < ddy || (dy == ddy && dx < ddx)) pre += L;
        if (dd == d) pre += e - b;
        E += L;
      }
    if (E <= kEll && pre >= 0 && pre < E) {
      const int u = (qy / UNIT) * a.UW + qx / UNIT;
      a.ell[ell_at(pre, u, a.U)] = int2{p, __float_as_int(w)};
    }
  }
}

// --- reverse steps ----------------------------------------------------------

// One lane per range pixel, K = N^2 lanes per range (a wave holds 64 / K
// ranges): dL/ds and dL/do of step t summed over the range by a fixed
// butterfly (first = true overwrites the outputs).
template <int N>
__device__ __forceinline__ void grad_so_body(Geo g, const int32_t *domain,
                                             const uint8_t *iso,
                                             const float *x,
                                             const float *gnext,
                                             float *grad_s, float *grad_o,
                                             int first, int bid) {
  constexpr int K = N * N;
  const long long tid = (long long)bid * blockDim.x + threadIdx.x;
  const int r = (int)(tid / K), pix = (int)(tid % K);
  const bool live = r < g.R;
  float as = 0.0f, ao = 0.0f;
  if (live) {
    const int i = pix / N, j = pix % N;
    const int ry = r / g.RW, rx = r % g.RW;
    const int d = clamp_dom(domain[r], g.ND), k = iso[r];
    const int Y = (d / g.NX) * g.step, X = (d % g.NX) * g.step;
    int si, sj;
    sigma(k, i, j, N - 1, si, sj);
    const float *c = x + (size_t)(Y + 2 * si) * g.W + X + 2 * sj;
    const float u = ((c[0] + c[1]) + (c[g.W] + c[g.W + 1])) * 0.25f;
    const float gv = gnext[(size_t)(ry * N + i) * g.W + rx * N + j];
    as = gv * u;
    ao = gv;
  }
#pragma unroll
  for (int o = K / 2; o > 0; o >>= 1) {
    as += __shfl_xor(as, o, K);
    ao += __shfl_xor(ao, o, K);
  }
  if (!live || pix != 0) return;
  if (first) {
    grad_s[r] = as;
    grad_o[r] = ao;
  } else {
    grad_s[r] += as;
    grad_o[r] += ao;
  }
}

struct StepArgs {
  Geo g;
  const int32_t *domain;
  const uint8_t *iso;
  const float *x, *gnext;
  float *grad_s, *grad_o, *gout;
  const int32_t *off, *pk, *heavy, *nheavy;
  const int4 *hbeg, *hlen;
  const float *pw;
  const int2 *ell;
  int first, nb_hv, nb_so, U, UW;
  // batches: bytes between images' tables and between their g_{t+1}
  // images, floats between their trajectories
  long long ws_stride, gn_stride, x_stride;
};

// g_t over the unit whose top-left pixel is (qy, qx).
template <int UNIT>
__device__ __forceinline__ void put_unit(const Geo &g, float *gout, int qy,
                                         int qx, float v) {
  float *q = gout + (size_t)qy * g.W + qx;
  if constexpr (UNIT == 2) {
    *(float2 *)q = float2{v, v};
    *(float2 *)(q + g.W) = float2{v, v};
  } else {
    *q = v;
  }
}

// Entry e of a list, read for the unit cell (cy, cx) of its domain:
// weight * g_{t+1}[the range pixel that reads that cell].
template <int N>
__device__ __forceinline__ int entry_pixel(const Geo &g, int pk, int cy,
                                           int cx) {
  int i, j;
  sigma_inv(pk & 7, cy, cx, N - 1, i, j);
  return min(max((pk >> 3) + i * g.W + j, 0), g.H * g.W - 1);
}

// One workgroup per heavy unit (a loop when there are more heavy units than
// workgroups): lane l sums the unit's entries l, l + 256, ... in order, in
// batches of 8 independent loads, then a fixed butterfly per wave and the
// four waves in order.  C2: at most 2 x 2 domains cover a unit (STEP >= n),
// and their list bounds are loaded together.
template <int N, int UNIT, bool C2>
__device__ __forceinline__ void heavy_body(const StepArgs &a, int hb) {
  __shared__ float red[4];
  const Geo &g = a.g;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // the first unit's records are read with the count (hb < nb_hv <= U keeps
  // them inside the arrays; they are used only if hb < nh)
  const int u_first = a.heavy[hb];
  int4 b_first, l_first;
  if constexpr (C2) {
    b_first = a.hbeg[hb];
    l_first = a.hlen[hb];
  }
  const int nh = *a.nheavy;
  for (int h = hb; h < nh; h += a.nb_hv) {
    const int u = h == hb ? u_first : a.heavy[h];
    const int qy = (u / a.UW) * UNIT, qx = (u % a.UW) * UNIT;
    int dy0, dy1, dx0, dx1;
    cover(g, qy, qx, dy0, dy1, dx0, dx1);
    float acc = 0.0f;
    if constexpr (C2) {
      const int4 B = h == hb ? b_first : a.hbeg[h];
      const int4 Lq = h == hb ? l_first : a.hlen[h];
      const int beg[4] = {B.x, B.y, B.z, B.w};
      const int len[4] = {Lq.x, Lq.y, Lq.z, Lq.w};
      int cy[4], cx[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        cy[q] = (qy - (dy0 + (q >> 1)) * g.step) >> 1;
        cx[q] = (qx - (dx0 + (q & 1)) * g.step) >> 1;
      }
      const int c1 = len[0], c2 = c1 + len[1], c3 = c2 + len[2];
      const int E = c3 + len[3];
      for (int f0 = threadIdx.x; f0 < E; f0 += 256 * 8) {
        int pkv[8], qv[8];
        float wv8[8], gv[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int f = f0 + 256 * j;
          const int q = (f >= c1) + (f >= c2) + (f >= c3);
          const int b = q == 0 ? beg[0] : q == 1 ? beg[1] : q == 2 ? beg[2] : beg[3];
          const int o = q == 0 ? 0 : q == 1 ? c1 : q == 2 ? c2 : c3;
          const int e = min(max(b + f - o, 0), g.R - 1);
          qv[j] = q;
          pkv[j] = f < E ? a.pk[e] : 0;
          wv8[j] = f < E ? a.pw[e] : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int q = qv[j];
          const int y = q == 0 ? cy[0] : q == 1 ? cy[1] : q == 2 ? cy[2] : cy[3];
          const int x = q == 0 ? cx[0] : q == 1 ? cx[1] : q == 2 ? cx[2] : cx[3];
          gv[j] = f0 + 256 * j < E ? a.gnext[entry_pixel<N>(g, pkv[j], y, x)]
                                   : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (f0 + 256 * j < E) acc = fmaf(wv8[j], gv[j], acc);
      }
    } else {
      for (int dy = dy0; dy <= dy1; ++dy)
        for (int dx = dx0; dx <= dx1; ++dx) {
          const int d = dy * g.NX + dx;
          const int b = a.off[d], L = a.off[d + 1] - b;
          const int y = (qy - dy * g.step) >> 1, x = (qx - dx * g.step) >> 1;
          for (int f0 = threadIdx.x; f0 < L; f0 += 256 * 8) {
            int pkv[8];
            float wv8[8], gv[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const int f = f0 + 256 * j;
              const int e = min(max(b + f, 0), g.R - 1);
              pkv[j] = f < L ? a.pk[e] : 0;
              wv8[j] = f < L ? a.pw[e] : 0.0f;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j)
              gv[j] = f0 + 256 * j < L
                          ? a.gnext[entry_pixel<N>(g, pkv[j], y, x)]
                          : 0.0f;
#pragma unroll
            for (int j = 0; j < 8; ++j)
              if (f0 + 256 * j < L) acc = fmaf(wv8[j], gv[j], acc);
          }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
      put_unit<UNIT>(g, a.gout, qy, qx, (red[0] + red[1]) + (red[2] + red[3]));
    __syncthreads();
  }
}

// One lane per light unit: its kEll slots (one load per slot pair), then
// g_{t+1} at the slots' pixels, summed in slot order.
template <int N, int UNIT>
__device__ __forceinline__ void light_body(const StepArgs &a, int lb) {
  const int u = lb * 256 + threadIdx.x;
  if (u >= a.U) return;
  const int4 *e4 = (const int4 *)a.ell;
  int4 sl[kEll / 2];
#pragma unroll
  for (int q = 0; q < kEll / 2; ++q) sl[q] = e4[(size_t)q * a.U + u];
  if (sl[0].x == -2) return;  // a heavy unit
  float gv[kEll];
  const int last = a.g.H * a.g.W - 1;  // entries are pixels of the image
#pragma unroll
  for (int q = 0; q < kEll / 2; ++q) {
    gv[2 * q] = sl[q].x >= 0 ? a.gnext[min(sl[q].x, last)] : 0.0f;
    gv[2 * q + 1] = sl[q].z >= 0 ? a.gnext[min(sl[q].z, last)] : 0.0f;
  }
  float acc = 0.0f;
#pragma unroll
  for (int q = 0; q < kEll / 2; ++q) {
    if (sl[q].x >= 0) acc = fmaf(__int_as_float(sl[q].y), gv[2 * q], acc);
    if (sl[q].z >= 0) acc = fmaf(__int_as_float(sl[q].w), gv[2 * q + 1], acc);
  }
  const int qy = (u / a.UW) * UNIT, qx = (u % a.UW) * UNIT;
  put_unit<UNIT>(a.g, a.gout, qy, qx, acc);
}

// One reverse step in one launch: workgroups [0, nb_hv) take the heavy
// units, the next nb_so form dL/ds and dL/do, the rest the light units (the
// unit parts only while g_t is needed, t > 0).
template <int N, int UNIT, bool C2>
__global__ __launch_bounds__(256) void k_adj_step(StepArgs a) {
  if (blockIdx.y > 0) {  // image blockIdx.y of a batch
    const long long wb = blockIdx.y * a.ws_stride;
    const size_t rb = (size_t)blockIdx.y * a.g.R;
    a.domain += rb;
    a.iso += rb;
    a.grad_s += rb;
    a.grad_o += rb;
    a.x += (size_t)blockIdx.y * a.x_stride;
    a.gnext = bump(a.gnext, blockIdx.y * a.gn_stride);
    a.gout = bump(a.gout, wb);
    a.off = bump(a.off, wb);
    a.pk = bump(a.pk, wb);
    a.heavy = bump(a.heavy, wb);
    a.nheavy = bump(a.nheavy, wb);
    a.hbeg = bump(a.hbeg, wb);
    a.hlen = bump(a.hlen, wb);
    a.pw = bump(a.pw, wb);
    a.ell = bump(a.ell, wb);
  }
  const int b = blockIdx.x;
  if (b < a.nb_hv)
    heavy_body<N, UNIT, C2>(a, b);
  else if (b < a.nb_hv + a.nb_so)
    grad_so_body<N>(a.g, a.domain, a.iso, a.x, a.gnext, a.grad_s, a.grad_o,
                    a.first, b - a.nb_hv);
  else
    light_body<N, UNIT>(a, b - a.nb_hv - a.nb_so);
}

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace of the adjoint: the domain table (built once per set of
// domains), the per-unit tables (again whenever s changes) and the two
// gradient images.
struct AdjWs {
  int32_t *off, *key0, *val0, *key1, *val1, *hist, *base, *pk, *heavy,
      *nheavy;
  float *pw, *gbuf0, *gbuf1;
  int4 *hbeg, *hlen;  // heavy units' covering lists (at most 2 x 2 domains)
  int2 *ell;
  int32_t *srt;  // val0, val1 or the small sort's output
  int nbr, unit, U, UW;
  bool small;
  size_t total;
};

AdjWs adj_layout(const Geo &g, void *ws) {
  const size_t HW = (size_t)g.H * g.W;
  AdjWs a;
  a.nbr = (g.R + 255) / 256;
  a.unit = g.step % 2 == 0 ? 2 : 1;
  a.UW = g.W / a.unit;
  a.U = (g.H / a.unit) * a.UW;
  a.small = g.R <= kSortR && g.ND <= kSortND;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += a256(bytes);
    return ws ? (char *)ws + at : nullptr;
  };
  a.off = (int32_t *)take(sizeof(int32_t) * (g.ND + 1));
  a.val0 = (int32_t *)take(sizeof(int32_t) * g.R);
  a.key0 = a.key1 = a.val1 = a.hist = a.base = nullptr;
  if (!a.small) {
    a.key0 = (int32_t *)take(sizeof(int32_t) * g.R);
    a.key1 = (int32_t *)take(sizeof(int32_t) * g.R);
    a.val1 = (int32_t *)take(sizeof(int32_t) * g.R);
    a.hist = (int32_t *)take(sizeof(int32_t) * (256 * (size_t)a.nbr + 1));
    a.base = (int32_t *)take(sizeof(int32_t) * (256 * (size_t)a.nbr + 1));
  }
  a.pk = (int32_t *)take(sizeof(int32_t) * g.R);
  a.pw = (float *)take(sizeof(float) * g.R);
  a.heavy = (int32_t *)take(sizeof(int32_t) * a.U);
  a.hbeg = (int4 *)take(sizeof(int4) * a.U);
  a.hlen = (int4 *)take(sizeof(int4) * a.U);
  a.nheavy = (int32_t *)take(sizeof(int32_t));
  a.ell = (int2 *)take(sizeof(int2) * kEll * (size_t)a.U);
  a.gbuf0 = (float *)take(sizeof(float) * HW);
  a.gbuf1 = (float *)take(sizeof(float) * HW);
  a.srt = a.val0;
  a.total = off;
  return a;
}

// The domain -> ranges table for these domains (clears the heavy count).
void build_adjoint_table(const Geo &g, const int32_t *domain, AdjWs &a,
                         hipStream_t st, int n_img = 1) {
  if (a.small) {
    hipLaunchKernelGGL(k_sort_small, dim3(1, (unsigned)n_img), dim3(1024), 0,
                       st, g, domain, a.val0, a.off, a.nheavy,
                       (long long)a.total);
    a.srt = a.val0;
    return;
  }
  const int bs = 256;
  hipLaunchKernelGGL(k_rs_init, dim3((g.R + bs - 1) / bs), dim3(bs), 0, st, g,
                     domain, a.key0, a.val0, a.nheavy);
  int bits = 0;
  while ((1ll << bits) < (long long)g.ND) ++bits;
  int32_t *kin = a.key0, *vin = a.val0, *kout = a.key1, *vout = a.val1;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3(a.nbr), dim3(256), 0, st, kin, g.R,
                       shift, a.hist);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, a.hist, 256 * a.nbr,
                       a.base);
    hipLaunchKernelGGL(k_rs_scatter, dim3(a.nbr), dim3(256), 0, st, kin, vin,
                       g.R, shift, a.base, kout, vout);
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  a.srt = vin;
  hipLaunchKernelGGL(k_bounds, dim3((g.ND + 1 + bs - 1) / bs), dim3(bs), 0, st,
                     g, kin, a.off);
}

// The per-unit tables for the current s; with_units also writes the padding
// and the heavy list (once per domain table).
template <int N>
void build_unit_tables(const Geo &g, const int32_t *domain,
                       const uint8_t *iso, const float *s, const AdjWs &a,
                       bool with_units, hipStream_t st, int n_img = 1) {
  UnitArgs u;
  u.g = g;
  u.domain = domain;
  u.srt = a.srt;
  u.off = a.off;
  u.iso = iso;
  u.s = s;
  u.ell = a.ell;
  u.pk = a.pk;
  u.heavy = a.heavy;
  u.nheavy = a.nheavy;
  u.hbeg = a.hbeg;
  u.hlen = a.hlen;
  u.pw = a.pw;
  u.U = a.U;
  u.UW = a.UW;
  u.nbu = with_units ? (a.U + 255) / 256 : 0;
  u.ws_stride = (long long)a.total;
  const long long ne = (long long)g.R * N * N;
  const dim3 grid((unsigned)(u.nbu + (ne + 255) / 256), (unsigned)n_img);
  if (a.unit == 2)
    hipLaunchKernelGGL((k_adj_units<N, 2>), grid, dim3(256), 0, st, u);
  else
    hipLaunchKernelGGL((k_adj_units<N, 1>), grid, dim3(256), 0, st, u);
}

// The reverse steps, with the tables built.
template <int N, int UNIT, bool C2>
void adjoint_steps_t(const Geo &g, const int32_t *domain, const uint8_t *iso,
                     int iters, const float *traj, const float *grad_xT,
                     float *grad_s, float *grad_o, const AdjWs &a,
                     hipStream_t st, int n_img) {
  const size_t HW = (size_t)g.H * g.W;
  StepArgs p;
  p.ws_stride = (long long)a.total;
  p.x_stride = (long long)HW * (iters + 1);
  p.g = g;
  p.domain = domain;
  p.iso = iso;
  p.grad_s = grad_s;
  p.grad_o = grad_o;
  p.off = a.off;
  p.pk = a.pk;
  p.heavy = a.heavy;
  p.nheavy = a.nheavy;
  p.hbeg = a.hbeg;
  p.hlen = a.hlen;
  p.pw = a.pw;
  p.ell = a.ell;
  p.U = a.U;
  p.UW = a.UW;
  p.nb_so = (int)(((long long)g.R * N * N + 255) / 256);
  const int nb_lt = (a.U + 255) / 256;
  // heavy-unit workgroups (each loops over the units past the first pass;
  // those past the count leave at once)
  const int nb_hv = std::min(a.U, 256);
  const float *gnext = grad_xT;
  float *bufs[2] = {a.gbuf0, a.gbuf1};
  for (int t = iters - 1; t >= 0; --t) {
    p.x = traj + (size_t)t * HW;
    p.gnext = gnext;
    // the caller's dL/dx_T images are HW floats apart, the workspace's
    // gradient images a workspace apart
    p.gn_stride = t == iters - 1 ? (long long)(HW * sizeof(float))
                                 : (long long)a.total;
    p.gout = bufs[t & 1];
    p.first = t == iters - 1 ? 1 : 0;
    // g_t is needed only while t > 0
    p.nb_hv = t > 0 ? nb_hv : 0;
    const int nb = p.nb_hv + p.nb_so + (t > 0 ? nb_lt : 0);
    hipLaunchKernelGGL((k_adj_step<N, UNIT, C2>),
                       dim3((unsigned)nb, (unsigned)n_img), dim3(256), 0, st,
                       p);
    gnext = p.gout;
  }
}

template <int N>
void adjoint_steps(const Geo &g, const int32_t *domain, const uint8_t *iso,
                   int iters, const float *traj, const float *grad_xT,
                   float *grad_s, float *grad_o, const AdjWs &a,
                   hipStream_t st, int n_img) {
  const bool c2 = g.step >= N;
  if (a.unit == 2) {
    if (c2)
      adjoint_steps_t<N, 2, true>(g, domain, iso, iters, traj, grad_xT, grad_s,
                                  grad_o, a, st, n_img);
    else
      adjoint_steps_t<N, 2, false>(g, domain, iso, iters, traj, grad_xT,
                                   grad_s, grad_o, a, st, n_img);
  } else {
    if (c2)
      adjoint_steps_t<N, 1, true>(g, domain, iso, iters, traj, grad_xT, grad_s,
                                  grad_o, a, st, n_img);
    else
      adjoint_steps_t<N, 1, false>(g, domain, iso, iters, traj, grad_xT,
                                   grad_s, grad_o, a, st, n_img);
  }
}

// Tables for these codes and s, then the reverse steps; n_img images (a
// batch needs the one-workgroup sort: the workspace holds one table per
// image, a.total bytes apart).
void adjoint(const Geo &g, const int32_t *domain, const uint8_t *iso,
             const float *s, int iters, const float *traj,
             const float *grad_xT, float *grad_s, float *grad_o, AdjWs &a,
             bool table_built, hipStream_t st, int n_img = 1) {
  if (!table_built) build_adjoint_table(g, domain, a, st, n_img);
  if (g.n == 8) {
    build_unit_tables<8>(g, domain, iso, s, a, !table_built, st, n_img);
    adjoint_steps<8>(g, domain, iso, iters, traj, grad_xT, grad_s, grad_o, a,
                     st, n_img);
  } else {
    build_unit_tables<4>(g, domain, iso, s, a, !table_built, st, n_img);
    adjoint_steps<4>(g, domain, iso, iters, traj, grad_xT, grad_s, grad_o, a,
                     st, n_img);
  }
}

void zero_grads(const Geo &g, float *grad_s, float *grad_o, hipStream_t st) {
  const int bs = 256;
  hipLaunchKernelGGL(k_fill_f32, dim3((g.R + bs - 1) / bs), dim3(bs), 0, st,
                     grad_s, (long long)g.R, 0.0f);
  hipLaunchKernelGGL(k_fill_f32, dim3((g.R + bs - 1) / bs), dim3(bs), 0, st,
                     grad_o, (long long)g.R, 0.0f);
}

// --- refinement: loss gradient and Adam ------------------------------------

// g = dL/dx for L = mean((x - I)^2), and per-block partial sums of (x - I)^2
// (tree in LDS, fixed order).
template <typename Pix>
__global__ __launch_bounds__(256) void k_mse_grad(long long HW, const float *x,
                                                  const Pix *img, float *gout,
                                                  double *partial) {
  __shared__ double red[256];
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  double d2 = 0.0;
  if (i < HW) {
    const float d = x[i] - (float)img[i];
    gout[i] = 2.0f * d / (float)HW;
    // the loss takes the difference exactly (both operands fit a double)
    const double dd = (double)x[i] - (double)img[i];
    d2 = dd * dd;
  }
  red[threadIdx.x] = d2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// loss[slot] = sum(partial) / HW, summed by one workgroup in a fixed order.
__global__ __launch_bounds__(256) void k_loss(const double *partial, int n,
                                              long long HW, double *loss,
                                              int slot) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[slot] = red[0] / (double)HW;
}

// One Adam step on (s, o); c1, c2 are the bias corrections 1 - beta^t.
__global__ void k_adam(int R, float *s, float *o, const float *gs,
                       const float *go, float *mom, float lr_s, float lr_o,
                       float b1, float b2, float c1, float c2, float eps,
                       float s_lim) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  float *ms = mom, *vs = mom + R, *mo = mom + 2 * R, *vo = mom + 3 * R;
  ms[r] = b1 * ms[r] + (1.0f - b1) * gs[r];
  vs[r] = b2 * vs[r] + (1.0f - b2) * gs[r] * gs[r];
  mo[r] = b1 * mo[r] + (1.0f - b1) * go[r];
  vo[r] = b2 * vo[r] + (1.0f - b2) * go[r] * go[r];
  const float ss = s[r] - lr_s * (ms[r] / c1) / (sqrtf(vs[r] / c2) + eps);
  s[r] = fminf(fmaxf(ss, -s_lim), s_lim);
  o[r] = o[r] - lr_o * (mo[r] / c1) / (sqrtf(vo[r] / c2) + eps);
}

}  // namespace

size_t decode_backward_ws_bytes(const Geo &g) {
  return adj_layout(g, nullptr).total;
}

DecGeo dec_geo(const Geo &g) {
  DecGeo d;
  d.H = g.H;
  d.W = g.W;
  d.n = g.n;
  d.step = g.step;
  d.RW = g.RW;
  d.NX = g.NX;
  d.ND = g.ND;
  return d;
}

// One iteration of n_img images (iterates at xs, ys; image stride xstride
// floats) with the pooled range kernel.
template <int N, int MODE>
void decode_pool_step(const Geo &g, int n_img, const int32_t *domain,
                      const uint8_t *iso, const float *s, const float *o,
                      const float *xs, float *ys, long long xstride, bool vec,
                      float x0, hipStream_t st) {
  constexpr int RPW = 256 / N;
  const int wpi = (g.R + RPW - 1) / RPW;
  const long long nwg = (long long)wpi * n_img;
  const int xcd_map = n_img > 1 && nwg % 8 == 0 ? 1 : 0;
  const long long tstride = (long long)g.H * g.W;
  if (vec)
    hipLaunchKernelGGL((k_decode_pool<N, 4, MODE>), dim3((unsigned)nwg),
                       dim3(256), 0, st, g, wpi, xcd_map, domain, iso, s, o, xs,
                       ys, xstride, tstride, x0);
  else
    hipLaunchKernelGGL((k_decode_pool<N, 1, MODE>), dim3((unsigned)nwg),
                       dim3(256), 0, st, g, wpi, xcd_map, domain, iso, s, o, xs,
                       ys, xstride, tstride, x0);
}

// 16-byte loads and stores need image rows, domain corners and range rows
// on 4-float boundaries, and a 16-byte aligned trajectory.
bool decode_vec_ok(const Geo &g, const float *traj) {
  return g.W % 4 == 0 && g.step % 4 == 0 && g.n % 4 == 0 &&
         ((uintptr_t)traj & 15) == 0;
}

template <int N>
void decode_steps_n(const Geo &g, int n_img, const int32_t *domain,
                    const uint8_t *iso, const float *s, const float *o,
                    int iters, float x0, float *traj, long long img_stride,
                    bool vec, hipStream_t st) {
  const long long HW = (long long)g.H * g.W;
  // the first launch writes x_0 .. x_2 (x_0 and x_1 for a single iteration)
  if (iters >= 2)
    decode_pool_step<N, 2>(g, n_img, domain, iso, s, o, traj, traj + HW,
                           img_stride, vec, x0, st);
  else
    decode_pool_step<N, 1>(g, n_img, domain, iso, s, o, traj, traj + HW,
                           img_stride, vec, x0, st);
  for (int t = 2; t < iters; ++t)
    decode_pool_step<N, 0>(g, n_img, domain, iso, s, o, traj + (size_t)t * HW,
                           traj + (size_t)(t + 1) * HW, img_stride, vec, x0,
                           st);
}

// All iterations, iters >= 1.
void decode_steps(const Geo &g, int n_img, const int32_t *domain,
                  const uint8_t *iso, const float *s, const float *o,
                  int iters, float x0, float *traj, long long img_stride,
                  hipStream_t st) {
  const bool vec = decode_vec_ok(g, traj);
  if (g.n == 8)
    decode_steps_n<8>(g, n_img, domain, iso, s, o, iters, x0, traj, img_stride,
                      vec, st);
  else
    decode_steps_n<4>(g, n_img, domain, iso, s, o, iters, x0, traj, img_stride,
                      vec, st);
}

hipError_t launch_decode(const Geo &g, const int32_t *domain,
                         const uint8_t *iso, const float *s, const float *o,
                         int iters, float x0, float *traj, hipStream_t st) {
  if (g.n != 4 && g.n != 8)  // other range sizes: the generic step
    return launch_decode_scaled(dec_geo(g), domain, iso, s, o, iters, x0, traj,
                                st);
  const long long HW = (long long)g.H * g.W;
  const int bs = 256;
  const dim3 grid((unsigned)((HW + bs - 1) / bs));
  if (iters == 0)
    hipLaunchKernelGGL(k_fill_f32, grid, dim3(bs), 0, st, traj, HW, x0);
  else
    decode_steps(g, 1, domain, iso, s, o, iters, x0, traj, 0, st);
  return hipGetLastError();
}

hipError_t launch_decode_batch(const Geo &g, int n_images,
                               const int32_t *domain, const uint8_t *iso,
                               const float *s, const float *o, int iters,
                               float x0, float *traj, hipStream_t st) {
  const long long HW = (long long)g.H * g.W;
  const long long stride = HW * (iters + 1);  // floats per trajectory
  const int bs = 256;
  if (iters == 0)
    hipLaunchKernelGGL(k_fill_first_batch,
                       dim3((unsigned)((HW + bs - 1) / bs), (unsigned)n_images),
                       dim3(bs), 0, st, traj, (int)HW, stride, x0);
  else
    decode_steps(g, n_images, domain, iso, s, o, iters, x0, traj, stride, st);
  return hipGetLastError();
}

hipError_t launch_decode_scaled(const DecGeo &d, const int32_t *domain,
                                const uint8_t *iso, const float *s,
                                const float *o, int iters, float x0,
                                float *traj, hipStream_t st) {
  const long long HW = (long long)d.H * d.W;
  const int bs = 256;
  const dim3 grid((unsigned)((HW + bs - 1) / bs));
  if (iters == 0) {
    hipLaunchKernelGGL(k_fill_f32, grid, dim3(bs), 0, st, traj, HW, x0);
    return hipGetLastError();
  }
  // the first launch writes x_0 .. x_2 (x_0 and x_1 for a single iteration)
  if (iters == 1)
    hipLaunchKernelGGL(k_decode_step_any<1>, grid, dim3(bs), 0, st, d, domain,
                       iso, s, o, traj, traj + HW, HW, x0);
  else
    hipLaunchKernelGGL(k_decode_step_any<2>, grid, dim3(bs), 0, st, d, domain,
                       iso, s, o, traj, traj + HW, HW, x0);
  for (int t = 2; t < iters; ++t)
    hipLaunchKernelGGL(k_decode_step_any<0>, grid, dim3(bs), 0, st, d, domain,
                       iso, s, o, traj + (size_t)t * HW,
                       traj + (size_t)(t + 1) * HW, HW, x0);
  return hipGetLastError();
}

hipError_t launch_decode_backward(const Geo &g, const int32_t *domain,
                                  const uint8_t *iso, const float *s,
                                  const float *o, int iters, const float *traj,
                                  const float *grad_xT, float *grad_s,
                                  float *grad_o, void *ws, hipStream_t st) {
  (void)o;
  if (iters == 0) {
    zero_grads(g, grad_s, grad_o, st);
    return hipGetLastError();
  }
  AdjWs a = adj_layout(g, ws);
  adjoint(g, domain, iso, s, iters, traj, grad_xT, grad_s, grad_o, a, false,
          st);
  return hipGetLastError();
}

size_t decode_backward_batch_ws_bytes(const Geo &g, int n_images) {
  return adj_layout(g, nullptr).total * (size_t)n_images;
}

bool decode_backward_batch_ok(const Geo &g) {
  return adj_layout(g, nullptr).small;
}

hipError_t launch_decode_backward_batch(const Geo &g, int n_images,
                                        const int32_t *domain,
                                        const uint8_t *iso, const float *s,
                                        int iters, const float *traj,
                                        const float *grad_xT, float *grad_s,
                                        float *grad_o, void *ws,
                                        hipStream_t st) {
  const int bs = 256;
  const long long nR = (long long)g.R * n_images;
  if (iters == 0) {
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((nR + bs - 1) / bs)),
                       dim3(bs), 0, st, grad_s, nR, 0.0f);
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((nR + bs - 1) / bs)),
                       dim3(bs), 0, st, grad_o, nR, 0.0f);
    return hipGetLastError();
  }
  AdjWs a = adj_layout(g, ws);
  adjoint(g, domain, iso, s, iters, traj, grad_xT, grad_s, grad_o, a, false,
          st, n_images);
  return hipGetLastError();
}

}  // namespace fic

namespace fic {

size_t refine_ws_bytes(const Geo &g, int iters) {
  const size_t HW = (size_t)g.H * g.W;
  const size_t nb = (HW + 255) / 256;
  return a256(sizeof(float) * HW * (size_t)(iters + 1)) +  // trajectory
         a256(sizeof(float) * HW) +                        // dL/dx_T
         a256(sizeof(float) * 2 * g.R) +                   // dL/ds, dL/do
         a256(sizeof(float) * 4 * g.R) +                   // Adam moments
         a256(sizeof(double) * nb) +                       // loss partials
         decode_backward_ws_bytes(g);
}

hipError_t launch_refine(const Geo &g, const int32_t *domain, const uint8_t *iso,
                         float *s, float *o, const void *image, int iters,
                         float x0, int steps, float lr_s, float lr_o,
                         double *loss, void *ws, hipStream_t st) {
  const size_t HW = (size_t)g.H * g.W;
  const int nb = (int)((HW + 255) / 256);
  char *w = (char *)ws;
  float *traj = (float *)w;   w += a256(sizeof(float) * HW * (size_t)(iters + 1));
  float *gx = (float *)w;     w += a256(sizeof(float) * HW);
  float *gso = (float *)w;    w += a256(sizeof(float) * 2 * g.R);
  float *mom = (float *)w;    w += a256(sizeof(float) * 4 * g.R);
  double *part = (double *)w; w += a256(sizeof(double) * nb);
  AdjWs adj = adj_layout(g, w);
  bool table_built = false;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f, s_lim = 0.999f;
  hipLaunchKernelGGL(k_fill_f32, dim3((4 * g.R + 255) / 256), dim3(256), 0, st,
                     mom, (long long)4 * g.R, 0.0f);
  float p1 = 1.0f, p2 = 1.0f;
  for (int step = 0; step <= steps; ++step) {
    hipError_t e = launch_decode(g, domain, iso, s, o, iters, x0, traj, st);
    if (e != hipSuccess) return e;
    const float *xT = traj + (size_t)iters * HW;
    if (g.bits == 12)
      hipLaunchKernelGGL(k_mse_grad<uint16_t>, dim3(nb), dim3(256), 0, st,
                         (long long)HW, xT, (const uint16_t *)image, gx, part);
    else
      hipLaunchKernelGGL(k_mse_grad<uint8_t>, dim3(nb), dim3(256), 0, st,
                         (long long)HW, xT, (const uint8_t *)image, gx, part);
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, st, part, nb,
                       (long long)HW, loss, step);
    if (step == steps) break;
    if (iters == 0) {
      zero_grads(g, gso, gso + g.R, st);
    } else {
      // the domains do not change: their table is built once; the
      // per-unit tables follow s
      adjoint(g, domain, iso, s, iters, traj, gx, gso, gso + g.R, adj,
              table_built, st);
      table_built = true;
    }
    p1 *= b1;
    p2 *= b2;
    hipLaunchKernelGGL(k_adam, dim3((g.R + 255) / 256), dim3(256), 0, st, g.R,
                       s, o, gso, gso + g.R, mom, lr_s, lr_o, b1, b2, 1.0f - p1,
                       1.0f - p2, eps, s_lim);
  }
  return hipGetLastError();
}

}  // namespace fic
