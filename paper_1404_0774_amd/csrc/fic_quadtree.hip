// fic_quadtree.hip -- adaptive range partition (Section V's quadtree
// method; Section II's adaptive fractal coding): ranges whose best residual
// exceeds a tolerance are split into their four quadrants and searched again
// at half the size.  The searches are ordinary encodes of each level with a
// range mask; the kernels here decide the splits and lay out the leaves.
//
// A level's ranges are numbered row-major on its own grid (RW ranges per
// row); range (ry, rx) of level l has the quadrants (2 ry + a, 2 rx + b) of
// level l + 1, a, b in {0, 1}.  Leaves are written top-level range by
// top-level range, each one's leaves in Z order ((0,0), (0,1), (1,0), (1,1)
// recursively).
#include "fic_internal.h"

namespace fic {

namespace {

// Split flags of one level and the range mask of the next: a range is split
// when it was searched (mask, null: every range) and its residual exceeds
// lim = tau * n^2.  Every range of the next level has exactly one parent,
// which writes its mask byte.
__global__ void k_qt_split(int RW, int R, const uint8_t *mask,
                           const double *err, double lim, uint8_t *split,
                           uint8_t *mask_next) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int ry = r / RW, rx = r % RW;
  const uint8_t sp = (!mask || mask[r]) && err[r] > lim ? 1 : 0;
  split[r] = sp;
  const int RWn = 2 * RW;
  mask_next[(2 * ry) * RWn + 2 * rx] = sp;
  mask_next[(2 * ry) * RWn + 2 * rx + 1] = sp;
  mask_next[(2 * ry + 1) * RWn + 2 * rx] = sp;
  mask_next[(2 * ry + 1) * RWn + 2 * rx + 1] = sp;
}

// Leaves under each range of a level: 1 unless split (split null: no range
// splits), else the sum over its quadrants (cnt_next: the next level's
// counts; null: one leaf each).
__global__ void k_qt_count(int RW, int R, const uint8_t *split,
                           const int32_t *cnt_next, int32_t *cnt) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  int c = 1;
  if (split && split[r]) {
    const int ry = r / RW, rx = r % RW, RWn = 2 * RW;
    c = 0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        c += cnt_next ? cnt_next[(2 * ry + a) * RWn + 2 * rx + b] : 1;
  }
  cnt[r] = c;
}

// Exclusive scan of cnt[0 .. n) into off[0 .. n]; off[n] is also the leaf
// count.  One workgroup of 1024 threads, each owning a contiguous slice.
__global__ __launch_bounds__(1024) void k_qt_scan(const int32_t *cnt, int n,
                                                  int32_t *off,
                                                  int32_t *n_leaves) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int b0 = min(t * per, n), b1 = min(b0 + per, n);
  int s = 0;
  for (int i = b0; i < b1; ++i) s += cnt[i];
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
    off[i] = run;
    run += cnt[i];
  }
  if (t == 1023) {
    off[n] = part[1023];
    *n_leaves = part[1023];
  }
}

__device__ __forceinline__ void put_leaf(const QtLevel &L, int ry, int rx,
                                         int at, const fic_quadtree_out &out) {
  const int r = ry * L.RW + rx;
  out.y[at] = ry * L.n;
  out.x[at] = rx * L.n;
  out.size[at] = (uint8_t)L.n;
  out.codes.domain[at] = L.codes.domain[r];
  out.codes.iso[at] = L.codes.iso[r];
  out.codes.s_idx[at] = L.codes.s_idx[r];
  out.codes.o_idx[at] = L.codes.o_idx[r];
  out.codes.err[at] = L.codes.err[r];
}

// One thread per top-level range: its leaves, in Z order, from off[r].
__global__ void k_qt_leaves(QtLevels q, const int32_t *off,
                            fic_quadtree_out out) {
  const int r0 = blockIdx.x * blockDim.x + threadIdx.x;
  if (r0 >= q.R0) return;
  int at = off[r0];
  const int ry0 = r0 / q.lv[0].RW, rx0 = r0 % q.lv[0].RW;
  if (q.L == 1 || !q.lv[0].split[r0]) {
    put_leaf(q.lv[0], ry0, rx0, at, out);
    return;
  }
  for (int q1 = 0; q1 < 4; ++q1) {
    const int ry1 = 2 * ry0 + (q1 >> 1), rx1 = 2 * rx0 + (q1 & 1);
    if (q.L == 2 || !q.lv[1].split[ry1 * q.lv[1].RW + rx1]) {
      put_leaf(q.lv[1], ry1, rx1, at++, out);
      continue;
    }
    for (int q2 = 0; q2 < 4; ++q2)
      put_leaf(q.lv[2], 2 * ry1 + (q2 >> 1), 2 * rx1 + (q2 & 1), at++, out);
  }
}

}  // namespace

hipError_t launch_qt_split(int RW, int R, const uint8_t *mask,
                           const double *err, double lim, uint8_t *split,
                           uint8_t *mask_next, hipStream_t st) {
  hipLaunchKernelGGL(k_qt_split, dim3((R + 255) / 256), dim3(256), 0, st, RW,
                     R, mask, err, lim, split, mask_next);
  return hipGetLastError();
}

hipError_t launch_qt_count(int RW, int R, const uint8_t *split,
                           const int32_t *cnt_next, int32_t *cnt,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_qt_count, dim3((R + 255) / 256), dim3(256), 0, st, RW,
                     R, split, cnt_next, cnt);
  return hipGetLastError();
}

hipError_t launch_qt_leaves(const QtLevels &q, const int32_t *cnt0,
                            int32_t *off, const fic_quadtree_out &out,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_qt_scan, dim3(1), dim3(1024), 0, st, cnt0, q.R0, off,
                     out.n_leaves);
  hipLaunchKernelGGL(k_qt_leaves, dim3((q.R0 + 255) / 256), dim3(256), 0, st,
                     q, (const int32_t *)off, out);
  return hipGetLastError();
}

}  // namespace fic
