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
// domain, the ranges that use it in increasing range order (a stable radix
// sort of the range -> domain map).  The lists are cut into segments of
// kSeg ranges; per step, one thread per (segment, cell) sums the segment's
// contributions to that cell, and one thread per pixel q adds the segments
// of the domains covering q, domains and segments in increasing order.  A
// domain shared by thousands of ranges (flat background) thus costs a short
// sum per pixel, and every sum has a fixed order, so the result is bitwise
// reproducible.
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
// FIRST: the first iteration from the constant start x0, with no reads of an
// iterate: every cell pools to u0 (the same expression on four x0), and the
// launch writes both x_0 = x0 (at xs) and x_1 (at ys) over its ranges.
template <int N, int V, bool FIRST>
__global__ __launch_bounds__(256) void k_decode_pool(
    Geo g, int wpi, int xcd_map, const int32_t *domain, const uint8_t *iso,
    const float *s, const float *o, const float *xs, float *ys,
    long long xstride, float x0) {
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
  if constexpr (!FIRST) {
    const int rl = threadIdx.x / N, a = threadIdx.x % N;
    const int r = r0 + rl;
    if (r < g.R) {
      const int d = clamp_dom(domain[cb + r], g.ND);
      const int Y = (d / g.NX) * g.step, X = (d % g.NX) * g.step;
      const float *p0 = x + (size_t)(Y + 2 * a) * g.W + X;
      const float *p1 = p0 + g.W;
      float u0[2 * N], u1[2 * N];
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
#pragma unroll
      for (int c = 0; c < N; ++c)
        pool[rl * PS + a * N + c] =
            ((u0[2 * c] + u0[2 * c + 1]) + (u1[2 * c] + u1[2 * c + 1])) * 0.25f;
    }
  }
  if constexpr (!FIRST) __syncthreads();
  {
    const int i = threadIdx.x / RPW, rl = threadIdx.x % RPW;
    const int r = r0 + rl;
    if (r < g.R) {
      const int k = iso[cb + r];
      const float sv = s[cb + r], ov = o[cb + r];
      const int ry = r / g.RW, rx = r - ry * g.RW;
      const float u0 = ((x0 + x0) + (x0 + x0)) * 0.25f;
      float out[N];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        if constexpr (FIRST) {
          out[j] = fmaf(sv, u0, ov);
        } else {
          int si, sj;
          sigma(k, i, j, N - 1, si, sj);
          out[j] = fmaf(sv, pool[rl * PS + si * N + sj], ov);
        }
      }
      const size_t off = (size_t)(ry * N + i) * g.W + rx * N;
      float *q = y + off;
      float *q0 = (float *)x + off;  // FIRST: x_0 is written, never read
      if constexpr (V == 4) {
#pragma unroll
        for (int j = 0; j < N; j += 4) {
          *(float4 *)(q + j) = float4{out[j], out[j + 1], out[j + 2], out[j + 3]};
          if constexpr (FIRST) *(float4 *)(q0 + j) = float4{x0, x0, x0, x0};
        }
      } else {
#pragma unroll
        for (int j = 0; j < N; ++j) {
          q[j] = out[j];
          if constexpr (FIRST) q0[j] = x0;
        }
      }
    }
  }
}

// Any range size n (a decode at another scale): one thread per output pixel.
__global__ void k_decode_step_any(DecGeo d, const int32_t *domain,
                                  const uint8_t *iso, const float *s,
                                  const float *o, const float *x, float *y) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= d.H * d.W) return;
  const int py = p / d.W, px = p % d.W;
  const int ry = py / d.n, rx = px / d.n, i = py % d.n, j = px % d.n;
  const int r = ry * d.RW + rx;
  const int dm = clamp_dom(domain[r], d.ND);
  int si, sj;
  sigma(iso[r], i, j, d.n - 1, si, sj);
  const int cy = (dm / d.NX) * d.step + 2 * si;
  const int cx = (dm % d.NX) * d.step + 2 * sj;
  const float *c = x + (size_t)cy * d.W + cx;
  const float u = ((c[0] + c[1]) + (c[d.W] + c[d.W + 1])) * 0.25f;
  y[p] = fmaf(s[r], u, o[r]);
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

// --- the domain -> ranges table --------------------------------------------

constexpr int kSeg = 16;     // ranges per list segment
constexpr int kGather = 32;  // segment partials loaded per round

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

// From the ranges sorted by domain: where each domain's list starts
// (off[0 .. ND]) and its length (cnt[0 .. ND)).  A binary search per domain
// instead of counting with atomics, which would queue up on a domain that
// thousands of ranges share.
__global__ void k_bounds(Geo g, const int32_t *sorted, int32_t *off,
                         int32_t *cnt) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d > g.ND) return;
  const int a = lower_bound(sorted, g.R, d);
  off[d] = a;
  if (d < g.ND) cnt[d] = lower_bound(sorted, g.R, d + 1) - a;
}

// Exclusive scan of ceil(in[i] / div), i < n, into out[0..n]; one workgroup
// of 1024 threads, each owning a contiguous slice.
__global__ __launch_bounds__(1024) void k_scan(const int32_t *in, int n,
                                               int div, int32_t *out) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int b0 = min(t * per, n), b1 = min(b0 + per, n);
  int s = 0;
  for (int i = b0; i < b1; ++i) s += (in[i] + div - 1) / div;
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
    run += (in[i] + div - 1) / div;
  }
  if (t == 1023) out[n] = part[1023];
}

// Stable LSD radix sort of (domain, range) pairs by domain, 8 bits a pass,
// blocks of 256 pairs: block histograms, one scan, stable scatter.
__global__ void k_rs_init(Geo g, const int32_t *domain, int32_t *key,
                          int32_t *val) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
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

// Segment table: segment s covers list entries [beg, end) of one domain.
// One thread per segment; its domain is the last d with segoff[d] <= s.
__global__ void k_seg_fill(Geo g, const int32_t *off, const int32_t *segoff,
                           int max_seg, int2 *seg) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= max_seg || s >= segoff[g.ND]) return;
  int lo = 0, hi = g.ND - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segoff[mid] <= s)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int x = off[lo] + (s - segoff[lo]) * kSeg;
  seg[s] = int2{x, min(x + kSeg, off[lo + 1])};
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

// One thread per (segment, cell): the segment's share of s_r g_{t+1}[p] / 4
// over the range pixels p that read that cell of the domain.
// `nseg` points at the segment count the table build wrote (the grid is
// sized for the largest possible count).  The segment's entries are loaded
// in three independent batches (list, codes, gradient) before the ordered
// sum, so a thread waits for three memory round trips, not 3 kSeg.
template <int N>
__device__ __forceinline__ void seg_partial_body(
    Geo g, const int32_t *nseg, const int2 *seg, const int32_t *list,
    const uint8_t *iso, const float *s, const float *gnext, float *partial,
    int bid) {
  constexpr int K = N * N;
  const int tid = bid * blockDim.x + threadIdx.x;
  const int sg = tid / K, c = tid % K, ci = c / N, cj = c % N;
  if (sg >= *nseg) return;
  const int2 be = seg[sg];
  int rr[kSeg];
#pragma unroll
  for (int u = 0; u < kSeg; ++u)
    rr[u] = be.x + u < be.y ? list[be.x + u] : -1;
  float w[kSeg];
  int pix[kSeg];
#pragma unroll
  for (int u = 0; u < kSeg; ++u) {
    const int r = rr[u] < 0 ? rr[0] : rr[u];
    int i, j;
    sigma_inv(iso[r], ci, cj, N - 1, i, j);
    const int ry = r / g.RW, rx = r % g.RW;
    pix[u] = (ry * N + i) * g.W + rx * N + j;
    w[u] = s[r] * 0.25f;
  }
  float gv[kSeg];
#pragma unroll
  for (int u = 0; u < kSeg; ++u) gv[u] = gnext[pix[u]];
  float acc = 0.0f;
#pragma unroll
  for (int u = 0; u < kSeg; ++u)
    if (rr[u] >= 0) acc = fmaf(w[u], gv[u], acc);
  partial[tid] = acc;
}

// One launch for the two independent parts of a reverse step: workgroups
// [0, nb_so) form dL/ds and dL/do, the rest (if any) the segment partials.
template <int N>
__global__ __launch_bounds__(256) void k_adj_step(
    Geo g, const int32_t *domain, const uint8_t *iso, const float *x,
    const float *gnext, float *grad_s, float *grad_o, int first, int nb_so,
    const int32_t *nseg, const int2 *seg, const int32_t *list, const float *s,
    float *partial) {
  if ((int)blockIdx.x < nb_so)
    grad_so_body<N>(g, domain, iso, x, gnext, grad_s, grad_o, first,
                    blockIdx.x);
  else
    seg_partial_body<N>(g, nseg, seg, list, iso, s, gnext, partial,
                        blockIdx.x - nb_so);
}

// One thread per pixel q: g_t[q] = sum of the segment partials of the
// cells containing q, over the domains covering q (loads batched by
// kGather: a domain shared by a thousand flat ranges has ~100 segments, and
// the pixels it covers would otherwise wait for ~13 rounds of loads).
template <int N>
__device__ __forceinline__ void grad_x_body(const Geo &g,
                                            const int32_t *segoff,
                                            const float *partial, float *gout,
                                            int bid) {
  constexpr int K = N * N;
  const int q = bid * blockDim.x + threadIdx.x;
  if (q >= g.H * g.W) return;
  const int qy = q / g.W, qx = q % g.W;
  const int span = 2 * N;
  int dy0 = qy - span + 1;
  dy0 = dy0 <= 0 ? 0 : (dy0 + g.step - 1) / g.step;
  int dx0 = qx - span + 1;
  dx0 = dx0 <= 0 ? 0 : (dx0 + g.step - 1) / g.step;
  const int dy1 = min(qy / g.step, g.NY - 1), dx1 = min(qx / g.step, g.NX - 1);
  float acc = 0.0f;
  for (int dy = dy0; dy <= dy1; ++dy)
    for (int dx = dx0; dx <= dx1; ++dx) {
      const int d = dy * g.NX + dx;
      const int s0 = segoff[d], s1 = segoff[d + 1];
      const int cell = ((qy - dy * g.step) >> 1) * N + ((qx - dx * g.step) >> 1);
      for (int sb = s0; sb < s1; sb += kGather) {
        float v[kGather];
#pragma unroll
        for (int u = 0; u < kGather; ++u)
          v[u] = sb + u < s1 ? partial[(size_t)(sb + u) * K + cell] : 0.0f;
#pragma unroll
        for (int u = 0; u < kGather; ++u)
          if (sb + u < s1) acc += v[u];
      }
    }
  gout[q] = acc;
}

template <int N>
__global__ __launch_bounds__(256) void k_grad_x(Geo g, const int32_t *segoff,
                                                const float *partial,
                                                float *gout) {
  grad_x_body<N>(g, segoff, partial, gout, blockIdx.x);
}

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace of the adjoint: the table (built once per code set) and the
// per-step buffers.
struct AdjWs {
  int32_t *cnt, *off, *segoff, *key0, *val0, *key1, *val1, *hist, *base;
  int2 *seg;
  float *partial, *gbuf0, *gbuf1;
  int32_t *list;  // points at val0 or val1 after the sort
  int nbr, max_seg;
  size_t total;
};

AdjWs adj_layout(const Geo &g, void *ws) {
  const size_t HW = (size_t)g.H * g.W;
  AdjWs a;
  a.nbr = (g.R + 255) / 256;
  a.max_seg = g.R + (g.R + kSeg - 1) / kSeg;  // non-empty domains <= R
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += a256(bytes);
    return ws ? (char *)ws + at : nullptr;
  };
  a.cnt = (int32_t *)take(sizeof(int32_t) * (g.ND + 1));
  a.off = (int32_t *)take(sizeof(int32_t) * (g.ND + 1));
  a.segoff = (int32_t *)take(sizeof(int32_t) * (g.ND + 1));
  a.key0 = (int32_t *)take(sizeof(int32_t) * g.R);
  a.val0 = (int32_t *)take(sizeof(int32_t) * g.R);
  a.key1 = (int32_t *)take(sizeof(int32_t) * g.R);
  a.val1 = (int32_t *)take(sizeof(int32_t) * g.R);
  a.hist = (int32_t *)take(sizeof(int32_t) * (256 * (size_t)a.nbr + 1));
  a.base = (int32_t *)take(sizeof(int32_t) * (256 * (size_t)a.nbr + 1));
  a.seg = (int2 *)take(sizeof(int2) * a.max_seg);
  a.partial = (float *)take(sizeof(float) * (size_t)a.max_seg * g.K);
  a.gbuf0 = (float *)take(sizeof(float) * HW);
  a.gbuf1 = (float *)take(sizeof(float) * HW);
  a.list = a.val0;
  a.total = off;
  return a;
}

// Build the domain -> ranges table for these codes.
void build_adjoint_table(const Geo &g, const int32_t *domain, AdjWs &a,
                         hipStream_t st) {
  const int bs = 256;
  hipLaunchKernelGGL(k_rs_init, dim3((g.R + bs - 1) / bs), dim3(bs), 0, st, g,
                     domain, a.key0, a.val0);
  int bits = 0;
  while ((1ll << bits) < (long long)g.ND) ++bits;
  int32_t *kin = a.key0, *vin = a.val0, *kout = a.key1, *vout = a.val1;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3(a.nbr), dim3(256), 0, st, kin, g.R,
                       shift, a.hist);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, a.hist, 256 * a.nbr,
                       1, a.base);
    hipLaunchKernelGGL(k_rs_scatter, dim3(a.nbr), dim3(256), 0, st, kin, vin,
                       g.R, shift, a.base, kout, vout);
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  a.list = vin;
  hipLaunchKernelGGL(k_bounds, dim3((g.ND + 1 + bs - 1) / bs), dim3(bs), 0, st,
                     g, kin, a.off, a.cnt);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, a.cnt, g.ND, kSeg,
                     a.segoff);
  hipLaunchKernelGGL(k_seg_fill, dim3((a.max_seg + bs - 1) / bs), dim3(bs), 0,
                     st, g, a.off, a.segoff, a.max_seg, a.seg);
}

// The reverse steps, with the table already built.
template <int N>
void adjoint_steps(const Geo &g, const int32_t *domain, const uint8_t *iso,
                   const float *s, int iters, const float *traj,
                   const float *grad_xT, float *grad_s, float *grad_o,
                   const AdjWs &a, hipStream_t st) {
  const size_t HW = (size_t)g.H * g.W;
  const int bs = 256;
  const float *gnext = grad_xT;
  float *bufs[2] = {a.gbuf0, a.gbuf1};
  for (int t = iters - 1; t >= 0; --t) {
    const float *x = traj + (size_t)t * HW;
    const long long nso = (long long)g.R * N * N;
    const int nb_so = (int)((nso + bs - 1) / bs);
    // the segment partials feed g_t, needed only while t > 0
    const long long np = t > 0 ? (long long)a.max_seg * N * N : 0;
    const int nb_sp = (int)((np + bs - 1) / bs);
    hipLaunchKernelGGL((k_adj_step<N>), dim3((unsigned)(nb_so + nb_sp)),
                       dim3(bs), 0, st, g, domain, iso, x, gnext, grad_s,
                       grad_o, t == iters - 1 ? 1 : 0, nb_so,
                       a.segoff + g.ND, a.seg, a.list, s, a.partial);
    if (t > 0) {
      float *gout = bufs[t & 1];
      hipLaunchKernelGGL((k_grad_x<N>), dim3((HW + bs - 1) / bs), dim3(bs), 0,
                         st, g, a.segoff, a.partial, gout);
      gnext = gout;
    }
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
template <int N, bool FIRST>
void decode_pool_step(const Geo &g, int n_img, const int32_t *domain,
                      const uint8_t *iso, const float *s, const float *o,
                      const float *xs, float *ys, long long xstride, bool vec,
                      float x0, hipStream_t st) {
  constexpr int RPW = 256 / N;
  const int wpi = (g.R + RPW - 1) / RPW;
  const long long nwg = (long long)wpi * n_img;
  const int xcd_map = n_img > 1 && nwg % 8 == 0 ? 1 : 0;
  if (vec)
    hipLaunchKernelGGL((k_decode_pool<N, 4, FIRST>), dim3((unsigned)nwg),
                       dim3(256), 0, st, g, wpi, xcd_map, domain, iso, s, o, xs,
                       ys, xstride, x0);
  else
    hipLaunchKernelGGL((k_decode_pool<N, 1, FIRST>), dim3((unsigned)nwg),
                       dim3(256), 0, st, g, wpi, xcd_map, domain, iso, s, o, xs,
                       ys, xstride, x0);
}

// 16-byte loads and stores need image rows, domain corners and range rows
// on 4-float boundaries, and a 16-byte aligned trajectory.
bool decode_vec_ok(const Geo &g, const float *traj) {
  return g.W % 4 == 0 && g.step % 4 == 0 && g.n % 4 == 0 &&
         ((uintptr_t)traj & 15) == 0;
}

// All iterations, iters >= 1: the first writes x_0 and x_1.
void decode_steps(const Geo &g, int n_img, const int32_t *domain,
                  const uint8_t *iso, const float *s, const float *o,
                  int iters, float x0, float *traj, long long img_stride,
                  hipStream_t st) {
  const long long HW = (long long)g.H * g.W;
  const bool vec = decode_vec_ok(g, traj);
  for (int t = 0; t < iters; ++t) {
    float *x = traj + (size_t)t * HW;
    float *y = traj + (size_t)(t + 1) * HW;
    if (g.n == 8) {
      if (t == 0)
        decode_pool_step<8, true>(g, n_img, domain, iso, s, o, x, y,
                                  img_stride, vec, x0, st);
      else
        decode_pool_step<8, false>(g, n_img, domain, iso, s, o, x, y,
                                   img_stride, vec, x0, st);
    } else {
      if (t == 0)
        decode_pool_step<4, true>(g, n_img, domain, iso, s, o, x, y,
                                  img_stride, vec, x0, st);
      else
        decode_pool_step<4, false>(g, n_img, domain, iso, s, o, x, y,
                                   img_stride, vec, x0, st);
    }
  }
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
  hipLaunchKernelGGL(k_fill_f32, grid, dim3(bs), 0, st, traj, HW, x0);
  for (int t = 0; t < iters; ++t)
    hipLaunchKernelGGL(k_decode_step_any, grid, dim3(bs), 0, st, d, domain,
                       iso, s, o, traj + (size_t)t * HW,
                       traj + (size_t)(t + 1) * HW);
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
  build_adjoint_table(g, domain, a, st);
  if (g.n == 8)
    adjoint_steps<8>(g, domain, iso, s, iters, traj, grad_xT, grad_s, grad_o,
                     a, st);
  else
    adjoint_steps<4>(g, domain, iso, s, iters, traj, grad_xT, grad_s, grad_o,
                     a, st);
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
    // the codes' domains do not change: the table is built once
    if (iters == 0) {
      zero_grads(g, gso, gso + g.R, st);
    } else {
      if (!table_built) build_adjoint_table(g, domain, adj, st);
      table_built = true;
      if (g.n == 8)
        adjoint_steps<8>(g, domain, iso, s, iters, traj, gx, gso, gso + g.R,
                         adj, st);
      else
        adjoint_steps<4>(g, domain, iso, s, iters, traj, gx, gso, gso + g.R,
                         adj, st);
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
