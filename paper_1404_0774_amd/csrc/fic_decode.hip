// fic_decode.hip -- iterating the partitioned IFS map (eq. 6) and its
// reverse-mode derivative with respect to the contrast s and offset o.
//
// Forward: one launch per iteration, one thread per output pixel:
//   x_{t+1}[p] = s_r * ((x00 + x01) + (x10 + x11)) * 0.25 + o_r
// where p is pixel (i, j) of range r and x.. is the 2x2 cell sigma_k(i, j)
// of the range's domain in x_t.
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
#include <hip/hip_cooperative_groups.h>

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

template <int N>
__global__ void k_decode_step(Geo g, const int32_t *domain, const uint8_t *iso,
                              const float *s, const float *o, const float *x,
                              float *y) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.H * g.W) return;
  const int py = p / g.W, px = p % g.W;
  const int ry = py / N, rx = px / N, i = py % N, j = px % N;
  const int r = ry * g.RW + rx;
  const int d = clamp_dom(domain[r], g.ND);
  int si, sj;
  sigma(iso[r], i, j, N - 1, si, sj);
  const int cy = (d / g.NX) * g.step + 2 * si, cx = (d % g.NX) * g.step + 2 * sj;
  const float *c = x + (size_t)cy * g.W + cx;
  const float u = ((c[0] + c[1]) + (c[g.W] + c[g.W + 1])) * 0.25f;
  y[p] = fmaf(s[r], u, o[r]);
}

// All iterations in one cooperative launch: every thread keeps the source
// cell offset, s and o of up to PPT pixels (p = thread + i * threads) in
// registers and the grid synchronises once per iteration, instead of one
// launch per iteration that looks the codes up again.  The arithmetic is
// k_decode_step's, so the iterates are identical.
template <int N, int PPT>
__global__ __launch_bounds__(256) void k_decode_persist(
    Geo g, const int32_t *domain, const uint8_t *iso, const float *s,
    const float *o, int iters, float x0, float *traj) {
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  const int HW = g.H * g.W;
  const int nth = gridDim.x * blockDim.x;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  int src[PPT];
  float sv[PPT], ov[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int p = tid + q * nth;
    src[q] = -1;
    sv[q] = ov[q] = 0.0f;
    if (p < HW) {
      const int py = p / g.W, px = p % g.W;
      const int r = (py / N) * g.RW + px / N;
      const int d = clamp_dom(domain[r], g.ND);
      int si, sj;
      sigma(iso[r], py % N, px % N, N - 1, si, sj);
      src[q] = ((d / g.NX) * g.step + 2 * si) * g.W + (d % g.NX) * g.step +
               2 * sj;
      sv[q] = s[r];
      ov[q] = o[r];
      traj[p] = x0;
    }
  }
  for (int t = 0; t < iters; ++t) {
    grid.sync();  // iterate t is complete everywhere
    const float *x = traj + (size_t)t * HW;
    float *y = traj + (size_t)(t + 1) * HW;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      if (src[q] < 0) continue;
      const float *c = x + src[q];
      const float u = ((c[0] + c[1]) + (c[g.W] + c[g.W + 1])) * 0.25f;
      y[tid + q * nth] = fmaf(sv[q], u, ov[q]);
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

// Many images of one geometry, each with its own codes: one thread per
// pixel of the whole batch.  Image b's codes start at entry b R; its
// trajectory is traj[b][t][pixel] ((iters + 1) images of H W floats each).
template <int N>
__global__ __launch_bounds__(256) void k_decode_step_batch(
    Geo g, long long total, const int32_t *domain, const uint8_t *iso,
    const float *s, const float *o, float *traj, int t, int iters) {
  const long long gp = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gp >= total) return;
  const int HW = g.H * g.W;
  const long long b = gp / HW;
  const int p = (int)(gp - b * HW);
  const int py = p / g.W, px = p % g.W;
  const int ry = py / N, rx = px / N, i = py % N, j = px % N;
  const long long r = b * g.R + ry * g.RW + rx;
  const int d = clamp_dom(domain[r], g.ND);
  int si, sj;
  sigma(iso[r], i, j, N - 1, si, sj);
  const int cy = (d / g.NX) * g.step + 2 * si, cx = (d % g.NX) * g.step + 2 * sj;
  float *x = traj + (size_t)b * (iters + 1) * HW + (size_t)t * HW;
  const float *c = x + (size_t)cy * g.W + cx;
  const float u = ((c[0] + c[1]) + (c[g.W] + c[g.W + 1])) * 0.25f;
  x[HW + p] = fmaf(s[r], u, o[r]);  // the image's iterate t + 1
}

// traj[b][0] = x0 for every image b.
__global__ void k_fill_first_batch(float *traj, long long HW, int iters,
                                   long long total, float v) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const long long b = i / HW;
  traj[b * (iters + 1) * HW + (i - b * HW)] = v;
}

__global__ void k_fill_f32(float *p, long long n, float v) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// --- the domain -> ranges table --------------------------------------------

// Decode in one cooperative launch when the image fits the resident grid.
constexpr bool kDecodePersistent = true;

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

// Device pointers of the adjoint table and per-step buffers.
struct AdjDev {
  const int32_t *nseg, *segoff, *list;
  const int2 *seg;
  float *partial, *gbuf0, *gbuf1;
};

// All reverse steps in one cooperative launch: each step's two parts are
// the per-step kernels' bodies run over virtual workgroups, with a grid
// synchronisation after the segment partials and after the gradient image,
// so every sum keeps its order and the result equals the per-step launches.
template <int N>
__global__ __launch_bounds__(256) void k_adj_persist(
    Geo g, const int32_t *domain, const uint8_t *iso, const float *s,
    int iters, const float *traj, const float *grad_xT, float *grad_s,
    float *grad_o, AdjDev a, int nb_so, int nb_sp, int nb_gx) {
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  const size_t HW = (size_t)g.H * g.W;
  const float *gnext = grad_xT;
  for (int t = iters - 1; t >= 0; --t) {
    const float *x = traj + (size_t)t * HW;
    for (int vb = blockIdx.x; vb < nb_so; vb += gridDim.x)
      grad_so_body<N>(g, domain, iso, x, gnext, grad_s, grad_o,
                      t == iters - 1 ? 1 : 0, vb);
    if (t == 0) break;
    for (int vb = blockIdx.x; vb < nb_sp; vb += gridDim.x)
      seg_partial_body<N>(g, a.nseg, a.seg, a.list, iso, s, gnext, a.partial,
                          vb);
    grid.sync();  // the step's segment partials are complete
    float *gout = (t & 1) ? a.gbuf1 : a.gbuf0;
    for (int vb = blockIdx.x; vb < nb_gx; vb += gridDim.x)
      grad_x_body<N>(g, a.segoff, a.partial, gout, vb);
    grid.sync();  // g_t is complete
    gnext = gout;
  }
}

constexpr int kMaxDevices = 64;

// Workgroups of 256 threads that can be resident at once for a kernel on
// the current device (0 if unknown).
template <typename Kern>
int resident_groups(Kern kern) {
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipGetDeviceProperties(&prop, dev) != hipSuccess ||
      !prop.cooperativeLaunch ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0) !=
          hipSuccess)
    return 0;
  return per_cu * prop.multiProcessorCount;
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
bool adjoint_persist(const Geo &g, const int32_t *domain, const uint8_t *iso,
                     const float *s, int iters, const float *traj,
                     const float *grad_xT, float *grad_s, float *grad_o,
                     const AdjWs &a, hipStream_t st) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess ||
      cap != hipStreamCaptureStatusNone)
    return false;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return false;
  static int groups_max[kMaxDevices];
  static bool known[kMaxDevices];
  if (!known[dev]) {
    groups_max[dev] = resident_groups(k_adj_persist<N>);
    known[dev] = true;
  }
  const long long HW = (long long)g.H * g.W;
  int nb_so = (int)(((long long)g.R * N * N + 255) / 256);
  int nb_sp = (int)(((long long)a.max_seg * N * N + 255) / 256);
  int nb_gx = (int)((HW + 255) / 256);
  int groups = std::max(nb_so, std::max(nb_sp, nb_gx));
  groups = std::min(groups, groups_max[dev]);
  if (groups < 1) return false;
  AdjDev d;
  d.nseg = a.segoff + g.ND;
  d.segoff = a.segoff;
  d.list = a.list;
  d.seg = a.seg;
  d.partial = a.partial;
  d.gbuf0 = a.gbuf0;
  d.gbuf1 = a.gbuf1;
  Geo gg = g;
  void *args[] = {&gg,         (void *)&domain, (void *)&iso,   (void *)&s,
                  &iters,      (void *)&traj,   (void *)&grad_xT,
                  (void *)&grad_s, (void *)&grad_o, &d, &nb_so, &nb_sp, &nb_gx};
  return hipLaunchCooperativeKernel((const void *)k_adj_persist<N>,
                                    dim3((unsigned)groups), dim3(256), args, 0,
                                    st) == hipSuccess;
}

template <int N>
void adjoint_steps(const Geo &g, const int32_t *domain, const uint8_t *iso,
                   const float *s, int iters, const float *traj,
                   const float *grad_xT, float *grad_s, float *grad_o,
                   const AdjWs &a, hipStream_t st) {
  if (kDecodePersistent && iters > 0 &&
      adjoint_persist<N>(g, domain, iso, s, iters, traj, grad_xT, grad_s,
                         grad_o, a, st))
    return;
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

// One cooperative launch for the whole decode when the image fits the
// resident grid at up to kPersistPixels pixels per thread; returns false
// (nothing enqueued) when it does not or the device cannot launch it.
constexpr int kPersistPixels = 4;

template <int N, int PPT>
bool decode_persist_try(const Geo &g, const int32_t *domain,
                        const uint8_t *iso, const float *s, const float *o,
                        int iters, float x0, float *traj, hipStream_t st,
                        int groups_max) {
  const long long HW = (long long)g.H * g.W;
  const long long groups = (HW + 256LL * PPT - 1) / (256LL * PPT);
  if (groups > groups_max) return false;
  Geo gg = g;
  void *args[] = {&gg,    (void *)&domain, (void *)&iso, (void *)&s,
                  (void *)&o, &iters,      &x0,          &traj};
  return hipLaunchCooperativeKernel((const void *)k_decode_persist<N, PPT>,
                                    dim3((unsigned)groups), dim3(256), args, 0,
                                    st) == hipSuccess;
}

template <int N>
bool decode_persist(const Geo &g, const int32_t *domain, const uint8_t *iso,
                    const float *s, const float *o, int iters, float x0,
                    float *traj, hipStream_t st) {
  // a stream under capture takes the per-iteration launches instead
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess ||
      cap != hipStreamCaptureStatusNone)
    return false;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return false;
  // resident workgroups per device and pixels-per-thread choice (computed
  // once; concurrent first calls compute the same values)
  static int groups_max[kMaxDevices][2];
  static bool known[kMaxDevices];
  if (!known[dev]) {
    groups_max[dev][0] = resident_groups(k_decode_persist<N, 1>);
    groups_max[dev][1] = resident_groups(k_decode_persist<N, kPersistPixels>);
    known[dev] = true;
  }
  return decode_persist_try<N, 1>(g, domain, iso, s, o, iters, x0, traj, st,
                                  groups_max[dev][0]) ||
         decode_persist_try<N, kPersistPixels>(g, domain, iso, s, o, iters, x0,
                                               traj, st, groups_max[dev][1]);
}

hipError_t launch_decode(const Geo &g, const int32_t *domain,
                         const uint8_t *iso, const float *s, const float *o,
                         int iters, float x0, float *traj, hipStream_t st) {
  if (g.n != 4 && g.n != 8)  // other range sizes: the generic step
    return launch_decode_scaled(dec_geo(g), domain, iso, s, o, iters, x0, traj,
                                st);
  if (kDecodePersistent && iters > 0 &&
      (g.n == 8 ? decode_persist<8>(g, domain, iso, s, o, iters, x0, traj, st)
                : decode_persist<4>(g, domain, iso, s, o, iters, x0, traj, st)))
    return hipGetLastError();
  const long long HW = (long long)g.H * g.W;
  const int bs = 256;
  const dim3 grid((unsigned)((HW + bs - 1) / bs));
  hipLaunchKernelGGL(k_fill_f32, grid, dim3(bs), 0, st, traj, HW, x0);
  for (int t = 0; t < iters; ++t) {
    const float *x = traj + (size_t)t * HW;
    float *y = traj + (size_t)(t + 1) * HW;
    if (g.n == 8)
      hipLaunchKernelGGL(k_decode_step<8>, grid, dim3(bs), 0, st, g, domain,
                         iso, s, o, x, y);
    else
      hipLaunchKernelGGL(k_decode_step<4>, grid, dim3(bs), 0, st, g, domain,
                         iso, s, o, x, y);
  }
  return hipGetLastError();
}

hipError_t launch_decode_batch(const Geo &g, int n_images,
                               const int32_t *domain, const uint8_t *iso,
                               const float *s, const float *o, int iters,
                               float x0, float *traj, hipStream_t st) {
  const long long HW = (long long)g.H * g.W;
  const long long total = HW * n_images;
  const int bs = 256;
  const dim3 grid((unsigned)((total + bs - 1) / bs));
  hipLaunchKernelGGL(k_fill_first_batch, grid, dim3(bs), 0, st, traj, HW,
                     iters, total, x0);
  for (int t = 0; t < iters; ++t) {
    if (g.n == 8)
      hipLaunchKernelGGL(k_decode_step_batch<8>, grid, dim3(bs), 0, st, g,
                         total, domain, iso, s, o, traj, t, iters);
    else
      hipLaunchKernelGGL(k_decode_step_batch<4>, grid, dim3(bs), 0, st, g,
                         total, domain, iso, s, o, traj, t, iters);
  }
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
