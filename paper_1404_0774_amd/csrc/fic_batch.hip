// fic_batch.hip -- host side of the batched encode: many slices of uneven
// size in one workspace, one launch per phase, and a persistent search grid
// fed from a largest-first work list.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <utility>
#include <vector>

#include "fic_internal.h"

namespace fic {
namespace {

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

// Code-extraction work items: this many workgroup passes of 256 lanes each
// (a range per N lanes: 32 ranges a pass for 8x8 ranges).
constexpr int kFinPasses = 4;

struct BatchPlan {
  std::vector<Geo> geo;
  std::vector<Tune> tune;
  std::vector<int4> items;
  std::vector<int2> wg_map;          // [sum of phase_total]
  std::vector<int> items_per_slice;  // [n] search items
  std::vector<int> fin_per_slice;    // [n] code-extraction items
  std::vector<size_t> slice_off;     // workspace offset of each slice
  size_t off_tab, off_items, off_map, off_ips, off_fps, off_rem, off_frem,
      off_counter, off_ticks, total;
  int phase_total[4], phase_base[4];
};

int plan_batch(const fic_params *slices, int n, BatchPlan &pl) {
  if (!slices) return abi_fail(FIC_E_INVALID, "slice params are NULL");
  if (n < 1) return abi_fail(FIC_E_INVALID, "n_slices < 1");
  pl.geo.resize(n);
  pl.tune.resize(n);
  for (int s = 0; s < n; ++s) {
    const int st = make_geo_for_batch(&slices[s], pl.geo[s]);
    if (st) return st;
    // 8x8 ranges build their range fragments from the image (confirmed per
    // image, for alignment, in fic_batch_prepare)
    pl.geo[s].pix_a = pl.geo[s].n == 8 ? 1 : 0;
    pl.tune[s] = resolve_tune(pl.geo[s], FIC_METHOD_MFMA);
    if (slices[s].bit_depth != slices[0].bit_depth ||
        slices[s].range_size != slices[0].range_size ||
        slices[s].s_bits != slices[0].s_bits ||
        slices[s].o_bits != slices[0].o_bits)
      return abi_fail(FIC_E_INVALID,
                        "slices must share bit depth, range size and bits");
  }
  if (slices[0].bit_depth != 8)
    return abi_fail(FIC_E_UNSUPPORTED, "batched search takes 8-bit slices");
  if (slices[0].range_size == 16 || slices[0].method != FIC_METHOD_MFMA)
    return abi_fail(FIC_E_UNSUPPORTED,
                    "batched search takes 4x4 or 8x8 ranges, matrix cores");

  // work list: slices largest first; within a slice, column chunks outer
  // and row groups inner so that workgroups running together share domains
  std::vector<long long> cost(n);
  for (int s = 0; s < n; ++s)
    cost[s] = (long long)(pl.geo[s].R_pad / kMfmaRangesPerWG) * pl.geo[s].NCB;
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<int4> search;
  pl.items_per_slice.assign(n, 0);
  std::vector<int> last(n, 0);  // position of each slice's last search item
  for (int s : order) {
    const Geo &g = pl.geo[s];
    const Tune &t = pl.tune[s];
    const int rg = g.R_pad / kMfmaRangesPerWG;
    for (int c0 = 0; c0 < g.NCB; c0 += t.item_blocks)
      for (int r = 0; r < rg; ++r) {
        last[s] = (int)search.size();
        search.push_back(int4{s, r, c0, std::min(c0 + t.item_blocks, g.NCB)});
        ++pl.items_per_slice[s];
      }
  }
  // A slice's code-extraction items follow its last search item by one grid
  // of items, so that the workgroup taking one rarely waits for the search
  // items still running; they run while later slices are searched.
  std::vector<std::pair<long long, int4>> ents;
  for (size_t i = 0; i < search.size(); ++i)
    ents.push_back({2ll * (long long)i, search[i]});
  pl.fin_per_slice.assign(n, 0);
  for (int s = 0; s < n; ++s) {
    const Geo &g = pl.geo[s];
    const int passes = (int)(((long long)g.R_pad * g.n + 255) / 256);
    for (int f = 0; f < passes; f += kFinPasses) {
      ents.push_back({2ll * (last[s] + kBatchSearchGrid) + 1,
                      int4{s, -1, f, std::min(kFinPasses, passes - f)}});
      ++pl.fin_per_slice[s];
    }
  }
  std::stable_sort(ents.begin(), ents.end(),
                   [](const std::pair<long long, int4> &a,
                      const std::pair<long long, int4> &b) {
                     return a.first < b.first;
                   });
  pl.items.clear();
  for (const auto &e : ents) pl.items.push_back(e.second);

  pl.wg_map.clear();
  for (int ph = 0; ph < 4; ++ph) {
    pl.phase_base[ph] = (int)pl.wg_map.size();
    int acc = 0;
    for (int s = 0; s < n; ++s) {
      const Geo &g = pl.geo[s];
      long long wg = 0;
      if (ph == 0) wg = g.n_dwg;
      if (ph == 1) wg = ((long long)g.R_pad * g.n + 255) / 256;
      if (ph == 2) wg = g.R_pad / 8;
      // phase 3 (code extraction) runs inside the search launch
      for (int i = 0; i < (int)wg; ++i) pl.wg_map.push_back(int2{s, i});
      acc += (int)wg;
    }
    pl.phase_total[ph] = acc;
  }

  size_t o = 0;
  pl.off_tab = o;     o = a256(o + sizeof(SliceDesc) * n);
  pl.off_items = o;   o = a256(o + sizeof(int4) * pl.items.size());
  pl.off_map = o;     o = a256(o + sizeof(int2) * pl.wg_map.size());
  pl.off_ips = o;     o = a256(o + sizeof(int) * n);
  pl.off_fps = o;     o = a256(o + sizeof(int) * n);
  pl.off_rem = o;     o = a256(o + sizeof(int) * n);
  pl.off_frem = o;    o = a256(o + sizeof(int) * n);
  pl.off_counter = o; o = a256(o + sizeof(int));
  pl.off_ticks = o;   o = a256(o + sizeof(unsigned long long) * (n + 1));
  pl.slice_off.resize(n);
  for (int s = 0; s < n; ++s) {
    pl.slice_off[s] = o;
    o = a256(o + enc_workspace_bytes(pl.geo[s]));
  }
  pl.total = o;
  return FIC_OK;
}

BatchDev batch_dev(const BatchPlan &pl, void *ws, int n) {
  char *w = (char *)ws;
  BatchDev bd;
  bd.tab = (SliceDesc *)(w + pl.off_tab);
  bd.items = (int4 *)(w + pl.off_items);
  bd.wg_map = (int2 *)(w + pl.off_map);
  bd.items_per_slice = (int *)(w + pl.off_ips);
  bd.fin_per_slice = (int *)(w + pl.off_fps);
  bd.remaining = (int *)(w + pl.off_rem);
  bd.fin_remaining = (int *)(w + pl.off_frem);
  bd.counter = (int *)(w + pl.off_counter);
  bd.ticks = (unsigned long long *)(w + pl.off_ticks);
  bd.n = n;
  bd.n_items = (int)pl.items.size();
  for (int i = 0; i < 4; ++i) {
    bd.phase_total[i] = pl.phase_total[i];
    bd.phase_base[i] = pl.phase_base[i];
  }
  bd.bits = pl.geo[0].bits;
  bd.rsize = pl.geo[0].n;
  return bd;
}

}  // namespace
}  // namespace fic

using namespace fic;

extern "C" {

int fic_batch_query(const fic_params *slices, int32_t n_slices,
                    size_t *ws_bytes) {
  BatchPlan pl;
  const int st = plan_batch(slices, n_slices, pl);
  if (st) return st;
  if (ws_bytes) *ws_bytes = pl.total;
  return abi_ok();
}

int fic_batch_prepare(const fic_params *slices, int32_t n_slices,
                      const void *const *images, const fic_codes *out,
                      void *workspace, size_t ws_bytes) {
  BatchPlan pl;
  int st = plan_batch(slices, n_slices, pl);
  if (st) return st;
  if (!images || !out || !workspace)
    return abi_fail(FIC_E_INVALID, "null images, codes or workspace");
  if (((uintptr_t)workspace) & 255)
    return abi_fail(FIC_E_INVALID, "workspace is not 256-byte aligned");
  if (ws_bytes < pl.total)
    return abi_fail(FIC_E_WORKSPACE, "workspace too small for the batch");
  std::vector<SliceDesc> tab(n_slices);
  for (int s = 0; s < n_slices; ++s) {
    if (!images[s] || !out[s].domain || !out[s].iso || !out[s].s_idx ||
        !out[s].o_idx || !out[s].err)
      return abi_fail(FIC_E_INVALID, "null image or code pointer in slice");
    tab[s].g = pl.geo[s];
    tab[s].g.pix_a = pl.geo[s].pix_a && ((uintptr_t)images[s] & 7) == 0;
    tab[s].b = enc_workspace_bufs(pl.geo[s],
                                  (char *)workspace + pl.slice_off[s]);
    tab[s].image = images[s];
    tab[s].out = out[s];
    tab[s].seed_blocks = pl.tune[s].seed_blocks;
  }
  char *w = (char *)workspace;
  hipError_t e = hipMemcpy(w + pl.off_tab, tab.data(),
                           sizeof(SliceDesc) * n_slices, hipMemcpyHostToDevice);
  if (e == hipSuccess && !pl.items.empty())
    e = hipMemcpy(w + pl.off_items, pl.items.data(),
                  sizeof(int4) * pl.items.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(w + pl.off_map, pl.wg_map.data(),
                  sizeof(int2) * pl.wg_map.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(w + pl.off_ips, pl.items_per_slice.data(),
                  sizeof(int) * n_slices, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(w + pl.off_fps, pl.fin_per_slice.data(),
                  sizeof(int) * n_slices, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    char msg[256];
    snprintf(msg, sizeof msg, "batch table upload: %s", hipGetErrorString(e));
    return abi_fail(FIC_E_HIP, msg);
  }
  return abi_ok();
}

int fic_encode_batch(const fic_params *slices, int32_t n_slices,
                     void *workspace, size_t ws_bytes, uint64_t *ticks,
                     void *stream) {
  BatchPlan pl;
  int st = plan_batch(slices, n_slices, pl);
  if (st) return st;
  if (!workspace) return abi_fail(FIC_E_INVALID, "null workspace");
  if (((uintptr_t)workspace) & 255)
    return abi_fail(FIC_E_INVALID, "workspace is not 256-byte aligned");
  if (ws_bytes < pl.total)
    return abi_fail(FIC_E_WORKSPACE, "workspace too small for the batch");
  BatchDev bd = batch_dev(pl, workspace, n_slices);
  if (ticks) bd.ticks = (unsigned long long *)ticks;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_prep_batch(bd, s);
  if (e == hipSuccess) e = launch_compact_batch(bd, s);
  int max_seed = 0;
  for (const Tune &t : pl.tune) max_seed = std::max(max_seed, t.seed_blocks);
  if (e == hipSuccess) e = launch_seed_batch(bd, max_seed, s);
  if (e == hipSuccess) e = launch_search_batch(bd, s);
  if (e != hipSuccess) {
    char msg[256];
    snprintf(msg, sizeof msg, "batch launch: %s", hipGetErrorString(e));
    return abi_fail(FIC_E_HIP, msg);
  }
  return abi_ok();
}

}  // extern "C"
