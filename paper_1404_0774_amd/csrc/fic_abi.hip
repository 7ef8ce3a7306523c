// fic_abi.hip -- host side of the libfic C ABI: argument validation,
// workspace layout and launch sequencing.  Validation is plain host code
// (no HIP call), so every error path can be exercised without a GPU.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>

#include "fic_internal.h"

namespace fic {
namespace {

thread_local std::string g_last_error;

int fail(int status, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

int ok() {
  g_last_error.clear();
  return FIC_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }


long long gcd_ll(long long a, long long b) {
  while (b) {
    long long t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// Bits needed for the largest possible residual scaled to an integer.  For
// any candidate |s_q| <= 1, pixels and contracted values lie in [0, P-1] and
// the fitted offset overshoots the grid by at most P + delta_o - 2, so the
// residual of eq. (8) is at most K (2P + delta_o - 3)^2.
int residual_bits(const Geo &g) {
  const double emax = (double)g.K * pow(2.0 * g.P + g.dlt - 3.0, 2.0);
  const double v = emax * g.escale;
  return (int)ceil(log2(v + 1.0));
}

// Validate the geometry and fill in Geo.  Host only.
int make_geo(const fic_params *p, Geo &g, bool for_encode) {
  if (!p) return fail(FIC_E_INVALID, "params is NULL");
  const int n = p->range_size;
  if (p->height <= 0 || p->width <= 0)
    return fail(FIC_E_INVALID, "image size %dx%d is empty", p->height,
                p->width);
  if (n <= 0) return fail(FIC_E_INVALID, "range_size %d < 1", n);
  if (p->height % n || p->width % n)
    return fail(FIC_E_INVALID, "image %dx%d is not a multiple of range_size %d",
                p->height, p->width, n);
  if (2 * n > p->height || 2 * n > p->width)
    return fail(FIC_E_INVALID, "domain side 2n = %d exceeds the image", 2 * n);
  if (p->domain_step < 1)
    return fail(FIC_E_INVALID, "domain_step %d < 1", p->domain_step);
  if (p->bit_depth != 8 && p->bit_depth != 12)
    return fail(FIC_E_UNSUPPORTED, "bit_depth %d (8 or 12)", p->bit_depth);
  if (n != 4 && n != 8 && n != 16)
    return fail(FIC_E_UNSUPPORTED, "range_size %d (4, 8 or 16)", n);
  // 16x16 ranges: the matrix-core search on 8-bit images (centred operands)
  if (for_encode && n == 16 &&
      (p->bit_depth != 8 || p->method != FIC_METHOD_MFMA))
    return fail(FIC_E_UNSUPPORTED,
                "16x16 ranges take 8-bit images and the matrix-core method");
  if (p->s_bits < 1 || p->s_bits > 8)
    return fail(FIC_E_UNSUPPORTED, "s_bits %d (1..8)", p->s_bits);
  // the code arrays hold one byte per index
  if (p->o_bits < 1 || p->o_bits > p->bit_depth + 1 || p->o_bits > 8)
    return fail(FIC_E_UNSUPPORTED, "o_bits %d (1..min(8, bit_depth+1))",
                p->o_bits);
  if (p->full_search != 0 && p->full_search != 1)
    return fail(FIC_E_INVALID, "full_search %d (0 or 1)", p->full_search);
  if (for_encode && p->method != FIC_METHOD_MFMA &&
      p->method != FIC_METHOD_DIRECT && p->method != FIC_METHOD_MFMA_I8)
    return fail(FIC_E_INVALID, "method %d", p->method);
  if (for_encode && p->method == FIC_METHOD_MFMA_I8 &&
      (p->bit_depth != 12 || p->range_size != 8))
    return fail(FIC_E_UNSUPPORTED,
                "the int8 matrix-core search takes 12-bit images with 8x8 "
                "ranges");
  if ((long long)p->height * p->width > (1ll << 30))
    return fail(FIC_E_UNSUPPORTED, "image larger than 2^30 pixels");

  g.H = p->height;
  g.W = p->width;
  g.bits = p->bit_depth;
  g.n = n;
  g.K = n * n;
  g.step = p->domain_step;
  g.sb = p->s_bits;
  g.ob = p->o_bits;
  g.RW = g.W / n;
  g.RH = g.H / n;
  g.R = g.RW * g.RH;
  g.NX = (g.W - 2 * n) / g.step + 1;
  g.NY = (g.H - 2 * n) / g.step + 1;
  g.ND = g.NX * g.NY;
  g.R_pad = (g.R + kMfmaRangesPerWG - 1) / kMfmaRangesPerWG * kMfmaRangesPerWG;
  g.NCB = (g.ND + 31) / 32;
  g.NC_pad = g.NCB * 32;
  g.n_dwg = (int)(((long long)g.NC_pad * n + 255) / 256);
  g.P = ldexp(1.0, g.bits);
  g.dlt = 2.0 * g.P / ldexp(1.0, g.ob);
  g.S = ldexp(1.0, g.sb - 1);
  g.escale = ldexp(1.0, 2 * g.sb + 2);
  g.invK = 1.0 / g.K;
  g.invS = 1.0 / g.S;
  g.invDlt = 1.0 / g.dlt;
  g.invEscale = 1.0 / g.escale;
  const int ebits = residual_bits(g);
  g.cbits = 64 - ebits;
  const long long ncand = 8ll * g.ND;
  if (g.cbits < 1 || g.cbits > 62 || ncand > (1ll << g.cbits))
    return fail(FIC_E_UNSUPPORTED,
                "%lld candidates exceed the %d index bits of the search key",
                ncand, g.cbits);
  // sweep order: a golden-ratio stride through the domain grid, coprime to ND
  long long st = llround(0.6180339887498949 * g.ND);
  if (st < 1) st = 1;
  while (gcd_ll(st, g.ND) != 1) ++st;
  g.dom_stride = (int)st;
  // range slots: the same stride through the ranges, so that every search
  // row group samples the whole image and the work per workgroup evens out
  long long rs = llround(0.6180339887498949 * g.R_pad);
  if (rs < 1) rs = 1;
  while (gcd_ll(rs, g.R_pad) != 1) ++rs;
  g.rng_stride = (int)rs;
  g.pix_a = 0;
  g.full = p->full_search;
  g.i8 = p->method == FIC_METHOD_MFMA_I8 && g.bits == 12;
  g.ident = 0;
  g.ctr = p->method == FIC_METHOD_MFMA && g.bits == 8 && n != 16;
  g.frag = (g.ctr && g.full) ||
           (g.bits == 8 && n == 16 && p->method == FIC_METHOD_MFMA) ||
           (g.bits == 12 && (p->method == FIC_METHOD_MFMA || g.i8));
  return FIC_OK;
}

EncLayout enc_layout(const Geo &g) {
  EncLayout L;
  const size_t planes = g.bits == 12 ? 2 : 1;
  size_t o = 0;
  L.off_bop = o;      o = align256(o + planes * (size_t)g.NC_pad * g.K * 2);
  L.off_aop = o;      o = align256(o + planes * (size_t)g.R_pad * 8 * g.K * 2);
  L.off_col_dom = o;  o = align256(o + (size_t)g.NC_pad * 4);
  L.off_col_sadp = o; o = align256(o + (size_t)g.NC_pad * 8);
  L.off_col_saa = o;  o = align256(o + (size_t)g.NC_pad * 8);
  L.off_col_rec = o;  o = align256(o + (size_t)g.NC_pad * 16);
  L.off_rng_sb = o;   o = align256(o + (size_t)g.R_pad * 8);
  L.off_rng_sbb = o;  o = align256(o + (size_t)g.R_pad * 8);
  L.off_best = o;     o = align256(o + (size_t)g.R_pad * 8);
  L.off_flat = o;     o = align256(o + (size_t)g.n_dwg * 4);
  L.off_act_slot = o; o = align256(o + (size_t)g.R_pad * 4);
  L.off_act_col = o;  o = align256(o + (size_t)g.NC_pad * 4);
  L.off_n_act = o;    o = align256(o + 2 * 4);
  L.off_rng_flag = o; o = align256(o + (size_t)g.R_pad);
  L.off_col_flag = o; o = align256(o + (size_t)g.NC_pad);
  const size_t i8 = g.i8 ? 1 : 0;
  L.off_bop8 = o;     o = align256(o + i8 * 2 * (size_t)g.NC_pad * g.K);
  L.off_aop8 = o;     o = align256(o + i8 * 2 * (size_t)g.R_pad * 8 * g.K);
  L.total = o;
  return L;
}

EncBufs enc_bufs(const EncLayout &L, void *ws) {
  char *w = (char *)ws;
  EncBufs b;
  b.bop = (_Float16 *)(w + L.off_bop);
  b.aop = (_Float16 *)(w + L.off_aop);
  b.col_dom = (int32_t *)(w + L.off_col_dom);
  b.col_sadp = (float2 *)(w + L.off_col_sadp);
  b.col_saa = (double *)(w + L.off_col_saa);
  b.col_rec = (ColRec *)(w + L.off_col_rec);
  b.rng_sb = (double *)(w + L.off_rng_sb);
  b.rng_sbb = (double *)(w + L.off_rng_sbb);
  b.best = (unsigned long long *)(w + L.off_best);
  b.flat_min = (int32_t *)(w + L.off_flat);
  b.act_slot = (int32_t *)(w + L.off_act_slot);
  b.act_col = (int32_t *)(w + L.off_act_col);
  b.n_act = (int32_t *)(w + L.off_n_act);
  b.rng_flag = (uint8_t *)(w + L.off_rng_flag);
  b.col_flag = (uint8_t *)(w + L.off_col_flag);
  b.rmask = nullptr;
  b.bop8 = (int8_t *)(w + L.off_bop8);
  b.aop8 = (int8_t *)(w + L.off_aop8);
  return b;
}

// Layout and header of the code stream of an encode with geometry g.
StreamGeo stream_geo(const Geo &g) {
  StreamGeo sg;
  sg.D = 0;
  while ((1ll << sg.D) < (long long)g.ND) ++sg.D;
  sg.sb = g.sb;
  sg.ob = g.ob;
  sg.B = sg.D + 3 + g.sb + g.ob;
  sg.R = g.R;
  sg.words = (sg.R * sg.B + 31) / 32;
  sg.header[0] = 0x53464950u;  // "PIFS" in little-endian byte order
  sg.header[1] = (uint32_t)g.H;
  sg.header[2] = (uint32_t)g.W;
  sg.header[3] = (uint32_t)g.bits | (uint32_t)g.n << 8 | (uint32_t)g.sb << 16 |
                 (uint32_t)g.ob << 24;
  sg.header[4] = (uint32_t)g.step;
  sg.header[5] = (uint32_t)sg.D;
  sg.header[6] = (uint32_t)((unsigned long long)sg.R & 0xffffffffu);
  sg.header[7] = (uint32_t)((unsigned long long)sg.R >> 32);
  return sg;
}

size_t stream_total_bytes(const StreamGeo &sg) {
  return 32 + 4 * (size_t)sg.words;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(FIC_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Phase timing for benchmarks: a pool of events, kMarks per timed call
// (before prep, seed, search and finalize, and at the end).
constexpr int kTimedCalls = 256;
constexpr int kMarks = 5;
struct Timing {
  bool on = false;
  bool created = false;
  int calls = 0;
  hipEvent_t ev[kMarks * kTimedCalls];
} g_timing;

void timing_mark(int phase, hipStream_t s) {
  if (!g_timing.on) return;
  const int slot = g_timing.calls % kTimedCalls;
  hipEventRecord(g_timing.ev[kMarks * slot + phase], s);
}

int encode_launch(const fic_params *p, Geo g, const void *image,
                  fic_codes out, void *workspace, void *stream,
                  const uint8_t *rmask = nullptr);

}  // namespace

// Shared with the batch front end (fic_batch.hip).
int make_geo_for_batch(const fic_params *p, Geo &g) {
  return make_geo(p, g, /*for_encode=*/true);
}
size_t enc_workspace_bytes(const Geo &g) { return enc_layout(g).total; }
EncBufs enc_workspace_bufs(const Geo &g, void *ws) {
  return enc_bufs(enc_layout(g), ws);
}
int abi_fail(int status, const char *msg) { return fail(status, "%s", msg); }
int abi_ok() { return ok(); }

}  // namespace fic

using namespace fic;

extern "C" {

int fic_query(const fic_params *p, int64_t *n_ranges, int64_t *n_domains,
              size_t *encode_ws_bytes, size_t *backward_ws_bytes) {
  Geo g;
  int st = make_geo(p, g, /*for_encode=*/false);
  if (st) return st;
  if (n_ranges) *n_ranges = g.R;
  if (n_domains) *n_domains = g.ND;
  if (encode_ws_bytes) *encode_ws_bytes = enc_layout(g).total;
  if (backward_ws_bytes) *backward_ws_bytes = decode_backward_ws_bytes(g);
  return ok();
}

int fic_encode(const fic_params *p, const void *image, fic_codes out,
               void *workspace, size_t ws_bytes, void *stream) {
  Geo g;
  int st = make_geo(p, g, /*for_encode=*/true);
  if (st) return st;
  if (!image || !workspace || !out.domain || !out.iso || !out.s_idx ||
      !out.o_idx || !out.err)
    return fail(FIC_E_INVALID, "null image, workspace or code pointer");
  if (((uintptr_t)workspace) & 255)
    return fail(FIC_E_INVALID, "workspace is not 256-byte aligned");
  const EncLayout L = enc_layout(g);
  if (ws_bytes < L.total)
    return fail(FIC_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes,
                L.total);
  return encode_launch(p, g, image, out, workspace, stream);
}

}  // extern "C"

namespace fic {
namespace {

// The launches of one encode on a validated workspace of at least
// enc_layout(g).total bytes.
int encode_launch(const fic_params *p, Geo g, const void *image,
                  fic_codes out, void *workspace, void *stream,
                  const uint8_t *rmask) {
  EncBufs b = enc_bufs(enc_layout(g), workspace);
  b.rmask = rmask;
  hipStream_t s = (hipStream_t)stream;
  // 8x8 ranges on the matrix cores take their range fragments straight from
  // the (8-byte aligned) image
  g.pix_a = p->method == FIC_METHOD_MFMA && g.bits == 8 && g.n == 8 &&
            ((uintptr_t)image & 7) == 0;
  // every range against every domain with no padding slots: the work lists
  // are the identity, written by the preparation
  g.ident = g.full && !rmask && g.R == g.R_pad ? 1 : 0;
  timing_mark(0, s);
  hipError_t e = launch_prep(g, image, b, s);
  if (e != hipSuccess) return hip_fail(e, "prep");
  timing_mark(1, s);
  // the seed pass ranks the leading column blocks to give every range a
  // starting bound; the search still covers every column block
  const Tune t = resolve_tune(g, p->method);
  // both searches walk the lists of range slots and domain columns they
  // visit (all of them, or those with variance), built here in order
  if (!g.ident) {
    e = launch_compact(g, b, s);
    if (e != hipSuccess) return hip_fail(e, "compact");
  }
  e = launch_seed_dense(g, b, t.seed_blocks, s);
  if (e != hipSuccess) return hip_fail(e, "seed");
  timing_mark(2, s);
  if (p->method == FIC_METHOD_DIRECT)
    e = launch_search_direct(g, b, t.chunks, s);
  else if (g.n == 16)
    e = launch_search_mfma16(
        g, b, t.chunks * (g.R_pad / kMfma12RangesPerWG), s);
  else if (p->method == FIC_METHOD_MFMA_I8)
    e = launch_search_mfma12_i8(
        g, b, t.chunks * (g.R_pad / kMfma12RangesPerWG), s);
  else if (g.bits == 12)
    e = launch_search_mfma12(
        g, b, t.chunks * (g.R_pad / kMfma12RangesPerWG), s);
  else
    e = launch_search_mfma(g, b, image, t.chunks * (g.R_pad / kMfmaRangesPerWG),
                           s);
  if (e != hipSuccess) return hip_fail(e, "search");
  timing_mark(3, s);
  e = launch_finalize(g, image, b, out, s);
  if (e != hipSuccess) return hip_fail(e, "finalize");
  timing_mark(4, s);
  if (g_timing.on) ++g_timing.calls;
  return ok();
}

// --- encode without allocation: scratch in a static device array ----------

// Encode workspace of fic_encode_noalloc.  Each device the library runs on
// holds its own copy from module load until the process ends.  In host code
// this name is a host-side stand-in, never a device address: kernels get the
// address that hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = 32ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices];

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
int scratch_address(void **ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kScratchDevices)
    return fail(FIC_E_UNSUPPORTED, "device %d beyond the %d the static scratch "
                "table covers", dev, kScratchDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *a = nullptr;
    e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!a || ((uintptr_t)a & 255))
      return fail(FIC_E_HIP, "static scratch address %p is not 256-byte "
                  "aligned", a);
    g_scratch_ptr[dev] = a;
  }
  *ptr = g_scratch_ptr[dev];
  return FIC_OK;
}

}  // namespace
}  // namespace fic

extern "C" {

int fic_encode_noalloc(const fic_params *p, const void *image, fic_codes out,
                       void *stream) {
  Geo g;
  int st = make_geo(p, g, /*for_encode=*/true);
  if (st) return st;
  if (!image || !out.domain || !out.iso || !out.s_idx || !out.o_idx ||
      !out.err)
    return fail(FIC_E_INVALID, "null image or code pointer");
  const EncLayout L = enc_layout(g);
  if (L.total > kScratchBytes)
    return fail(FIC_E_WORKSPACE, "encode needs %zu bytes, the static scratch "
                "array holds %zu", L.total, kScratchBytes);
  void *ws = nullptr;
  st = scratch_address(&ws);
  if (st) return st;
  // every buffer the launches read is written earlier in the same encode,
  // so the previous call's bytes need no clearing
  return encode_launch(p, g, image, out, ws, stream);
}

int fic_search_counts(const fic_params *p, const void *workspace,
                      size_t ws_bytes, int64_t *n_ranges, int64_t *n_domains) {
  Geo g;
  int st = make_geo(p, g, /*for_encode=*/true);
  if (st) return st;
  if (!workspace || !n_ranges || !n_domains)
    return fail(FIC_E_INVALID, "null workspace or output pointer");
  const EncLayout L = enc_layout(g);
  if (ws_bytes < L.total)
    return fail(FIC_E_INVALID, "workspace %zu bytes < %zu", ws_bytes, L.total);
  int32_t n[2];
  const hipError_t e = hipMemcpy(n, (const char *)workspace + L.off_n_act,
                                 sizeof n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  *n_ranges = n[0];
  *n_domains = n[1];
  return ok();
}

int fic_decode(const fic_params *p, const int32_t *domain, const uint8_t *iso,
               const float *s, const float *o, int32_t iters, float x0,
               float *traj, void *stream) {
  Geo g;
  int st = make_geo(p, g, /*for_encode=*/false);
  if (st) return st;
  if (!domain || !iso || !s || !o || !traj)
    return fail(FIC_E_INVALID, "null code or trajectory pointer");
  if (iters < 0) return fail(FIC_E_INVALID, "iters %d < 0", iters);
  hipError_t e = launch_decode(g, domain, iso, s, o, iters, x0, traj,
                               (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "decode");
  return ok();
}

int fic_decode_batch(const fic_params *p, int32_t n_images,
                     const int32_t *domain, const uint8_t *iso,
                     const float *s, const float *o, int32_t iters, float x0,
                     float *traj, void *stream) {
  Geo g;
  int st = make_geo(p, g, /*for_encode=*/false);
  if (st) return st;
  if (!domain || !iso || !s || !o || !traj)
    return fail(FIC_E_INVALID, "null code or trajectory pointer");
  if (iters < 0) return fail(FIC_E_INVALID, "iters %d < 0", iters);
  if (n_images < 1) return fail(FIC_E_INVALID, "n_images %d < 1", n_images);
  if (n_images > 65535)
    return fail(FIC_E_UNSUPPORTED, "n_images %d > 65535", n_images);
  if (g.n == 16)
    return fail(FIC_E_UNSUPPORTED, "the batched decode takes 4x4 or 8x8 ranges");
  if ((long long)g.H * g.W * n_images > (1ll << 31))
    return fail(FIC_E_UNSUPPORTED, "%d images of %dx%d exceed 2^31 pixels",
                n_images, g.H, g.W);
  hipError_t e = launch_decode_batch(g, n_images, domain, iso, s, o, iters, x0,
                                     traj, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "decode_batch");
  return ok();
}

int fic_decode_scaled(const fic_params *p, int32_t scale_num,
                      int32_t scale_den, const int32_t *domain,
                      const uint8_t *iso, const float *s, const float *o,
                      int32_t iters, float x0, float *traj, void *stream) {
  Geo g;
  int st = make_geo(p, g, /*for_encode=*/false);
  if (st) return st;
  if (!domain || !iso || !s || !o || !traj)
    return fail(FIC_E_INVALID, "null code or trajectory pointer");
  if (iters < 0) return fail(FIC_E_INVALID, "iters %d < 0", iters);
  if (scale_num < 1 || scale_den < 1)
    return fail(FIC_E_INVALID, "scale %d/%d is not positive", scale_num,
                scale_den);
  const long long nz = (long long)g.n * scale_num, sz = (long long)g.step * scale_num;
  if (nz % scale_den || sz % scale_den)
    return fail(FIC_E_INVALID,
                "scale %d/%d leaves ranges (%d) or the domain grid (%d) "
                "without whole pixels",
                scale_num, scale_den, g.n, g.step);
  DecGeo d;
  d.n = (int)(nz / scale_den);
  d.step = (int)(sz / scale_den);
  const long long Hz = (long long)g.RH * d.n, Wz = (long long)g.RW * d.n;
  if (Hz * Wz > (1ll << 30))
    return fail(FIC_E_UNSUPPORTED, "scaled image %lldx%lld larger than 2^30 "
                "pixels", Hz, Wz);
  d.H = (int)Hz;
  d.W = (int)Wz;
  d.RW = g.RW;
  d.NX = g.NX;
  d.ND = g.ND;
  // the domain grid keeps its shape: (W z - 2 n z) / (STEP z) = (W - 2n) / STEP
  if ((d.W - 2 * d.n) / d.step + 1 != g.NX || (d.H - 2 * d.n) / d.step + 1 != g.NY)
    return fail(FIC_E_INVALID, "scale %d/%d changes the domain grid",
                scale_num, scale_den);
  hipError_t e = launch_decode_scaled(d, domain, iso, s, o, iters, x0, traj,
                                      (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "decode_scaled");
  return ok();
}

int fic_decode_backward(const fic_params *p, const int32_t *domain,
                        const uint8_t *iso, const float *s, const float *o,
                        int32_t iters, const float *traj, const float *grad_xT,
                        float *grad_s, float *grad_o, void *workspace,
                        size_t ws_bytes, void *stream) {
  Geo g;
  int st = make_geo(p, g, /*for_encode=*/false);
  if (st) return st;
  if (g.n == 16)
    return fail(FIC_E_UNSUPPORTED, "the adjoint takes 4x4 or 8x8 ranges");
  if ((long long)g.H * g.W > (1ll << 28))
    return fail(FIC_E_UNSUPPORTED, "the adjoint takes at most 2^28 pixels");
  if (!domain || !iso || !s || !o || !traj || !grad_xT || !grad_s || !grad_o ||
      !workspace)
    return fail(FIC_E_INVALID, "null pointer argument");
  if (iters < 0) return fail(FIC_E_INVALID, "iters %d < 0", iters);
  if (((uintptr_t)workspace) & 255)
    return fail(FIC_E_INVALID, "workspace is not 256-byte aligned");
  const size_t need = decode_backward_ws_bytes(g);
  if (ws_bytes < need)
    return fail(FIC_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes,
                need);
  hipError_t e = launch_decode_backward(g, domain, iso, s, o, iters, traj,
                                        grad_xT, grad_s, grad_o, workspace,
                                        (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "decode_backward");
  return ok();
}

int fic_decode_backward_batch_workspace(const fic_params *p,
                                        int32_t n_images, size_t *bytes) {
  Geo g;
  int st = make_geo(p, g, /*for_encode=*/false);
  if (st) return st;
  if (!bytes) return fail(FIC_E_INVALID, "bytes is NULL");
  if (n_images < 1) return fail(FIC_E_INVALID, "n_images %d < 1", n_images);
  *bytes = decode_backward_batch_ws_bytes(g, n_images);
  return ok();
}

int fic_decode_backward_batch(const fic_params *p, int32_t n_images,
                              const int32_t *domain, const uint8_t *iso,
                              const float *s, const float *o, int32_t iters,
                              const float *traj, const float *grad_xT,
                              float *grad_s, float *grad_o, void *workspace,
                              size_t ws_bytes, void *stream) {
  Geo g;
  int st = make_geo(p, g, /*for_encode=*/false);
  if (st) return st;
  if (!domain || !iso || !s || !o || !traj || !grad_xT || !grad_s || !grad_o ||
      !workspace)
    return fail(FIC_E_INVALID, "null pointer argument");
  if (iters < 0) return fail(FIC_E_INVALID, "iters %d < 0", iters);
  if (n_images < 1) return fail(FIC_E_INVALID, "n_images %d < 1", n_images);
  if (((uintptr_t)workspace) & 255)
    return fail(FIC_E_INVALID, "workspace is not 256-byte aligned");
  if (n_images > 65535)
    return fail(FIC_E_UNSUPPORTED, "n_images %d > 65535", n_images);
  if (g.n == 16)
    return fail(FIC_E_UNSUPPORTED, "the adjoint takes 4x4 or 8x8 ranges");
  if ((long long)g.H * g.W * n_images > (1ll << 31))
    return fail(FIC_E_UNSUPPORTED, "%d images of %dx%d exceed 2^31 pixels",
                n_images, g.H, g.W);
  if (!decode_backward_batch_ok(g))
    return fail(FIC_E_UNSUPPORTED,
                "the batched adjoint takes up to 8192 ranges and 16384 "
                "domains per image");
  const size_t need = decode_backward_batch_ws_bytes(g, n_images);
  if (ws_bytes < need)
    return fail(FIC_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes,
                need);
  (void)o;
  hipError_t e = launch_decode_backward_batch(
      g, n_images, domain, iso, s, iters, traj, grad_xT, grad_s, grad_o,
      workspace, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "decode_backward_batch");
  return ok();
}

int fic_refine_workspace(const fic_params *p, int32_t iters, size_t *bytes) {
  Geo g;
  int st = make_geo(p, g, /*for_encode=*/false);
  if (st) return st;
  if (iters < 0) return fail(FIC_E_INVALID, "iters %d < 0", iters);
  if (!bytes) return fail(FIC_E_INVALID, "bytes is NULL");
  *bytes = refine_ws_bytes(g, iters);
  return ok();
}

int fic_refine(const fic_params *p, const int32_t *domain, const uint8_t *iso,
               float *s, float *o, const void *image, int32_t iters, float x0,
               int32_t steps, float lr_s, float lr_o, double *loss,
               void *workspace, size_t ws_bytes, void *stream) {
  Geo g;
  int st = make_geo(p, g, /*for_encode=*/false);
  if (st) return st;
  if (g.n == 16)
    return fail(FIC_E_UNSUPPORTED, "refinement takes 4x4 or 8x8 ranges");
  if ((long long)g.H * g.W > (1ll << 28))
    return fail(FIC_E_UNSUPPORTED, "refinement takes at most 2^28 pixels");
  if (!domain || !iso || !s || !o || !image || !loss || !workspace)
    return fail(FIC_E_INVALID, "null pointer argument");
  if (iters < 0 || steps < 0)
    return fail(FIC_E_INVALID, "iters %d or steps %d < 0", iters, steps);
  if (!(lr_s >= 0.0f) || !(lr_o >= 0.0f))
    return fail(FIC_E_INVALID, "learning rates must be >= 0");
  if (((uintptr_t)workspace) & 255)
    return fail(FIC_E_INVALID, "workspace is not 256-byte aligned");
  const size_t need = refine_ws_bytes(g, iters);
  if (ws_bytes < need)
    return fail(FIC_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes,
                need);
  hipError_t e = launch_refine(g, domain, iso, s, o, image, iters, x0, steps,
                               lr_s, lr_o, loss, workspace, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "refine");
  return ok();
}

}  // extern "C"

namespace fic {
namespace {

// Levels and workspace of a quadtree encode.
struct QtPlan {
  int L;
  fic_params lp[3];
  Geo g[3];
  size_t off_enc, off_codes[3], off_split[3], off_mask[3], off_cnt[3], off_off,
      total;
};

int qt_plan(const fic_params *p, int n_min, QtPlan &q) {
  Geo g0;
  int st = make_geo(p, g0, /*for_encode=*/true);
  if (st) return st;
  if (n_min != 4 && n_min != 8 && n_min != 16)
    return fail(FIC_E_UNSUPPORTED, "min_range_size %d (4, 8 or 16)", n_min);
  if (n_min > p->range_size)
    return fail(FIC_E_INVALID, "min_range_size %d above range_size %d", n_min,
                p->range_size);
  q.L = 0;
  size_t enc = 0;
  for (int n = p->range_size; n >= n_min; n /= 2) {
    q.lp[q.L] = *p;
    q.lp[q.L].range_size = n;
    st = make_geo(&q.lp[q.L], q.g[q.L], /*for_encode=*/true);
    if (st) return st;
    enc = enc > enc_layout(q.g[q.L]).total ? enc : enc_layout(q.g[q.L]).total;
    ++q.L;
  }
  size_t o = 0;
  q.off_enc = o;
  o = align256(o + enc);
  for (int l = 0; l < q.L; ++l) {
    const size_t R = (size_t)q.g[l].R;
    q.off_codes[l] = o;
    o = align256(o + R * (4 + 1 + 1 + 1));
    o = align256(o + R * 8);  // residuals (8-byte aligned after the bytes)
    q.off_split[l] = o;
    o = align256(o + R);
    q.off_mask[l] = o;
    o = align256(o + R);
    q.off_cnt[l] = o;
    o = align256(o + R * 4);
  }
  q.off_off = o;
  o = align256(o + ((size_t)q.g[0].R + 1) * 4);
  q.total = o;
  return FIC_OK;
}

fic_codes qt_codes(const QtPlan &q, int l, char *w) {
  const size_t R = (size_t)q.g[l].R;
  char *c = w + q.off_codes[l];
  fic_codes k;
  k.domain = (int32_t *)c;
  k.iso = (uint8_t *)(c + 4 * R);
  k.s_idx = (uint8_t *)(c + 5 * R);
  k.o_idx = (uint8_t *)(c + 6 * R);
  k.err = (double *)(c + align256(7 * R));
  return k;
}

}  // namespace
}  // namespace fic

extern "C" {

int fic_quadtree_query(const fic_params *p, int32_t min_range_size,
                       size_t *ws_bytes, int64_t *max_leaves) {
  QtPlan q;
  const int st = qt_plan(p, min_range_size, q);
  if (st) return st;
  if (ws_bytes) *ws_bytes = q.total;
  if (max_leaves) *max_leaves = q.g[q.L - 1].R;
  return ok();
}

int fic_encode_quadtree(const fic_params *p, int32_t min_range_size,
                        double tau, const void *image, fic_quadtree_out out,
                        void *workspace, size_t ws_bytes, void *stream) {
  QtPlan q;
  int st = qt_plan(p, min_range_size, q);
  if (st) return st;
  if (tau != tau) return fail(FIC_E_INVALID, "tau is NaN");
  if (!image || !workspace || !out.y || !out.x || !out.size ||
      !out.n_leaves || !out.codes.domain || !out.codes.iso ||
      !out.codes.s_idx || !out.codes.o_idx || !out.codes.err)
    return fail(FIC_E_INVALID, "null image, workspace or output pointer");
  if (((uintptr_t)workspace) & 255)
    return fail(FIC_E_INVALID, "workspace is not 256-byte aligned");
  if (ws_bytes < q.total)
    return fail(FIC_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes,
                q.total);
  char *w = (char *)workspace;
  hipStream_t s = (hipStream_t)stream;
  QtLevels lv;
  lv.L = q.L;
  lv.R0 = q.g[0].R;
  for (int l = 0; l < q.L; ++l) {
    const fic_codes c = qt_codes(q, l, w);
    const uint8_t *mask = l ? (const uint8_t *)(w + q.off_mask[l]) : nullptr;
    st = encode_launch(&q.lp[l], q.g[l], image, c, w + q.off_enc, stream, mask);
    if (st) return st;
    uint8_t *split = (uint8_t *)(w + q.off_split[l]);
    if (l + 1 < q.L) {
      const double lim = tau * (double)q.g[l].K;
      const hipError_t e =
          launch_qt_split(q.g[l].RW, q.g[l].R, mask, c.err, lim, split,
                          (uint8_t *)(w + q.off_mask[l + 1]), s);
      if (e != hipSuccess) return hip_fail(e, "quadtree split");
    }
    lv.lv[l].codes = c;
    lv.lv[l].split = split;
    lv.lv[l].RW = q.g[l].RW;
    lv.lv[l].n = q.g[l].n;
  }
  // leaves under each top-level range: counted from the finest level that
  // can split upwards (a level with one level below it has one leaf per
  // quadrant); a single level has one leaf per range
  int32_t *cnt0 = (int32_t *)(w + q.off_cnt[0]);
  for (int l = q.L > 1 ? q.L - 2 : 0; l >= 0; --l) {
    const bool splits = l + 1 < q.L;
    const bool deeper = l + 2 < q.L;
    const hipError_t e = launch_qt_count(
        q.g[l].RW, q.g[l].R, splits ? lv.lv[l].split : nullptr,
        deeper ? (const int32_t *)(w + q.off_cnt[l + 1]) : nullptr,
        (int32_t *)(w + q.off_cnt[l]), s);
    if (e != hipSuccess) return hip_fail(e, "quadtree count");
  }
  const hipError_t e =
      launch_qt_leaves(lv, cnt0, (int32_t *)(w + q.off_off), out, s);
  if (e != hipSuccess) return hip_fail(e, "quadtree leaves");
  return ok();
}

int fic_stream_query(const fic_params *p, size_t *bytes,
                     int32_t *record_bits) {
  Geo g;
  const int st = make_geo(p, g, /*for_encode=*/false);
  if (st) return st;
  const StreamGeo sg = stream_geo(g);
  if (bytes) *bytes = stream_total_bytes(sg);
  if (record_bits) *record_bits = sg.B;
  return ok();
}

int fic_stream_pack(const fic_params *p, const int32_t *domain,
                    const uint8_t *iso, const uint8_t *s_idx,
                    const uint8_t *o_idx, void *out, size_t out_bytes,
                    void *stream) {
  Geo g;
  const int st = make_geo(p, g, /*for_encode=*/false);
  if (st) return st;
  if (!domain || !iso || !s_idx || !o_idx || !out)
    return fail(FIC_E_INVALID, "null code or stream pointer");
  if ((uintptr_t)out & 3)
    return fail(FIC_E_INVALID, "stream buffer is not 4-byte aligned");
  const StreamGeo sg = stream_geo(g);
  if (out_bytes < stream_total_bytes(sg))
    return fail(FIC_E_WORKSPACE, "stream buffer %zu bytes < %zu needed",
                out_bytes, stream_total_bytes(sg));
  const hipError_t e = launch_stream_pack(sg, domain, iso, s_idx, o_idx, out,
                                          (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "stream_pack");
  return ok();
}

int fic_stream_header(const void *header, size_t bytes, fic_params *p) {
  if (!header || !p) return fail(FIC_E_INVALID, "null header or params");
  if (bytes < 32) return fail(FIC_E_INVALID, "a stream header is 32 bytes");
  uint32_t h[8];
  memcpy(h, header, sizeof h);
  if (h[0] != 0x53464950u) return fail(FIC_E_INVALID, "not a PIFS code stream");
  fic_params q;
  memset(&q, 0, sizeof q);
  q.height = (int32_t)h[1];
  q.width = (int32_t)h[2];
  q.bit_depth = (int32_t)(h[3] & 255u);
  q.range_size = (int32_t)((h[3] >> 8) & 255u);
  q.s_bits = (int32_t)((h[3] >> 16) & 255u);
  q.o_bits = (int32_t)(h[3] >> 24);
  q.domain_step = (int32_t)h[4];
  q.method = FIC_METHOD_MFMA;
  Geo g;
  if (h[1] > 0x7fffffffu || h[2] > 0x7fffffffu || h[4] > 0x7fffffffu ||
      make_geo(&q, g, /*for_encode=*/false) != FIC_OK)
    return fail(FIC_E_INVALID, "stream header holds invalid parameters");
  const StreamGeo sg = stream_geo(g);
  if (h[5] != (uint32_t)sg.D || h[6] != sg.header[6] || h[7] != sg.header[7])
    return fail(FIC_E_INVALID,
                "stream header's domain bits or range count disagree with "
                "its geometry");
  *p = q;
  return ok();
}

int fic_stream_unpack(const fic_params *p, const void *in, size_t in_bytes,
                      int32_t *domain, uint8_t *iso, uint8_t *s_idx,
                      uint8_t *o_idx, void *stream) {
  Geo g;
  const int st = make_geo(p, g, /*for_encode=*/false);
  if (st) return st;
  if (!in || !domain || !iso || !s_idx || !o_idx)
    return fail(FIC_E_INVALID, "null stream or code pointer");
  if ((uintptr_t)in & 3)
    return fail(FIC_E_INVALID, "stream is not 4-byte aligned");
  const StreamGeo sg = stream_geo(g);
  if (in_bytes < stream_total_bytes(sg))
    return fail(FIC_E_INVALID, "stream %zu bytes < %zu for these parameters",
                in_bytes, stream_total_bytes(sg));
  const hipError_t e = launch_stream_unpack(sg, in, domain, iso, s_idx, o_idx,
                                            (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "stream_unpack");
  return ok();
}

int fic_timing_begin(void) {
  if (!g_timing.created) {
    for (int i = 0; i < kMarks * kTimedCalls; ++i) {
      hipError_t e = hipEventCreate(&g_timing.ev[i]);
      if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    g_timing.created = true;
  }
  g_timing.on = true;
  g_timing.calls = 0;
  return ok();
}

int fic_timing_end(int32_t *n_calls, double *ms_prep, double *ms_seed,
                   double *ms_search, double *ms_finalize) {
  if (!g_timing.on) return fail(FIC_E_INVALID, "timing was not begun");
  g_timing.on = false;
  const int n = g_timing.calls < kTimedCalls ? g_timing.calls : kTimedCalls;
  double acc[kMarks - 1] = {0, 0, 0, 0};
  for (int c = 0; c < n; ++c) {
    hipError_t e = hipEventSynchronize(g_timing.ev[kMarks * c + kMarks - 1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    for (int ph = 0; ph < kMarks - 1; ++ph) {
      float ms = 0.0f;
      e = hipEventElapsedTime(&ms, g_timing.ev[kMarks * c + ph],
                              g_timing.ev[kMarks * c + ph + 1]);
      if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
      acc[ph] += ms;
    }
  }
  if (n_calls) *n_calls = n;
  if (ms_prep) *ms_prep = acc[0];
  if (ms_seed) *ms_seed = acc[1];
  if (ms_search) *ms_search = acc[2];
  if (ms_finalize) *ms_finalize = acc[3];
  return ok();
}

const char *fic_status_string(int status) {
  switch (status) {
    case FIC_OK: return "ok";
    case FIC_E_INVALID: return "invalid argument";
    case FIC_E_UNSUPPORTED: return "unsupported parameters";
    case FIC_E_WORKSPACE: return "workspace too small";
    case FIC_E_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char *fic_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
