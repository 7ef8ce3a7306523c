// fic_internal.h -- host/device shared definitions of libfic (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fic.h"

namespace fic {

// Geometry and quantisation constants of one encode, passed by value to
// every kernel.
struct Geo {
  int H, W;          // image size
  int bits;          // 8 or 12
  int n, K;          // range side, pixels per range (n*n)
  int step;          // domain grid spacing
  int sb, ob;        // contrast / offset bits
  int RW, RH, R;     // ranges per row, per column, total
  int NX, NY, ND;    // domain grid
  int R_pad;         // ranges rounded up to the search tile
  int NCB;           // column blocks of 32 domains
  int n_dwg;         // workgroups of the domain preparation
  int NC_pad;        // NCB * 32
  int cbits;         // low bits of the search key that hold the candidate
  int dom_stride;    // sweep order: column c holds domain (c * dom_stride) % ND
  int rng_stride;    // range slots: slot i holds range (i * rng_stride) % R_pad
                     //   (slots of ranges >= R are padding)
  int pix_a;         // 1: the 8-bit n = 8 matrix-core search builds its range
                     //   fragments from the image; no range operand is written
  int full;          // 1: ranges and domains without variance are searched
                     //   too (0: they are left out; their outcome is fixed)
  int i8;            // 1: 12-bit operands also as int8 hi/lo planes (the
                     //   int8 matrix-core search)
  int ident;         // 1: the searched range slots and domain columns are
                     //   all of them, in order (a full search of every range
                     //   with no padding slots): the preparation writes the
                     //   lists and their lengths, with no compaction pass
  int ctr;           // 1: 8-bit matrix-core operands (4x4, 8x8 ranges) are
                     //   centred on each block's rounded mean:
                     //   A - round(SA/K) and b - round(Sb/K), exact FP16
  int frag;          // 1: the domain operand planes are stored in MFMA
                     //   fragment order (full matrix-core searches of 8-bit
                     //   centred images, the 16x16 and the 12-bit
                     //   matrix-core searches; bop_index and bop8_index give
                     //   the layout)
  double escale;     // 2^(2 sb + 2): residual * escale is an integer
  double P;          // 2^bits
  double dlt;        // offset step
  double S;          // 2^(sb - 1)
  // exact reciprocals of the powers of two above (K, S, dlt, escale): a
  // product by them equals the quotient bit for bit, at a fraction of the cost
  double invK, invS, invDlt, invEscale;
};

// Device buffers carved out of the caller's workspace.
// One column's statistics in a single 16-byte record (8-bit search): SA,
// sqrt(D') rounded down (+inf for flat domains and padding), the domain
// index and the sum of squared cell sums, exact in 32 bits for 8-bit images
// (<= 64 * 1020^2).
struct __attribute__((aligned(16))) ColRec {
  float sa, sc;
  int dom;
  unsigned saa;
};

struct EncBufs {
  _Float16 *bop;     // [NC_pad][K] contracted domain cell sums, sweep order
                     //   (12-bit: two planes, hi then lo, each [NC_pad][K])
  _Float16 *aop;     // [R_pad * 8][K] range pixels permuted per transform,
                     //   row 8 i + k for range slot i (12-bit: two planes);
                     //   every per-range array below is indexed by slot
  int32_t *col_dom;  // [NC_pad] domain index of a column, -1 for padding
  float2 *col_sadp;  // [NC_pad] (sum of the column's cell sums SA,
                     //   prune denominator D' rounded down; +inf for flat
                     //   domains and padding)
  double *col_saa;   // [NC_pad] sum of squared cell sums
  ColRec *col_rec;   // [NC_pad] the three above in one record (saa = 0
                     //   for 12-bit images)
  double *rng_sb;    // [R_pad] sum of range pixels
  double *rng_sbb;   // [R_pad] sum of squared range pixels
  unsigned long long *best; // [R_pad] packed (residual, candidate) keys
  int32_t *flat_min;  // [domain-prep workgroups] smallest flat domain index
                      //   seen by each workgroup (INT_MAX if none)
  // The candidates the search has to visit: range slots holding a range with
  // variance and domain columns holding a domain with variance, each in
  // order (flat ranges keep candidate 0, flat domains tie with the first
  // one; code extraction handles both).
  int32_t *act_slot;  // [R_pad] searched range slots, first n_act[0] valid
  int32_t *act_col;   // [NC_pad] searched domain columns, first n_act[1]
  int32_t *n_act;     // [2] counts of the two lists
  uint8_t *rng_flag;  // [R_pad] 1: slot holds a range with variance
  uint8_t *col_flag;  // [NC_pad] 1: column holds a domain with variance
  int8_t *bop8;      // 12-bit int8 search only: [2][NC_pad][K] A_hi, A_lo
  int8_t *aop8;      // 12-bit int8 search only: [2][R_pad * 8][K] b_hi, b_lo
  // Optional, per image range (not slot): 0 leaves the range out of the
  // search (its code is then candidate 0's); null searches every range.
  // The quadtree encode searches only the quadrants of split ranges.
  const uint8_t *rmask;
};

// Byte layout of the encode workspace.
struct EncLayout {
  size_t off_bop, off_aop, off_col_dom, off_col_sadp, off_col_saa, off_col_rec;
  size_t off_rng_sb, off_rng_sbb, off_best, off_flat, off_act_slot,
      off_act_col, off_n_act, off_rng_flag, off_col_flag, off_bop8, off_aop8;
  size_t total;
};

// One slice of a batch, as the batched kernels see it (device table).
struct SliceDesc {
  Geo g;
  EncBufs b;
  const void *image;
  fic_codes out;
  int seed_blocks;  // column blocks the dense seed pass fits
};

// Device side of a batch (all pointers into the caller's workspace).
struct BatchDev {
  SliceDesc *tab;             // [n]
  int4 *items;                // [n_items] work list of the persistent search:
                              //   search item (slice, row group, first
                              //   block, end block) or code-extraction item
                              //   (slice, -1, first workgroup, workgroups)
  int2 *wg_map;               // per phase (domain prep, range prep, seed)
                              //   and workgroup: slice and the workgroup's
                              //   index within the slice
  int *items_per_slice;       // [n] search items per slice
  int *fin_per_slice;         // [n] code-extraction items per slice
  int *remaining;             // [n] unfinished search items per slice
  int *fin_remaining;         // [n] unfinished code-extraction items
  int *counter;               // [1] next work item
  unsigned long long *ticks;  // [n + 1] start tick, codes-ready tick per slice
  int n, n_items;
  int phase_total[4];         // workgroups per phase
  int phase_base[4];          // first entry of each phase in wg_map
  int bits, rsize;            // common to every slice
};

// Geometry of a decode at any range size (the encoded geometry scaled):
// image H x W, ranges n x n (RW per row), domains 2n x 2n on a grid of
// spacing step with NX per row and ND in all.
struct DecGeo {
  int H, W, n, step, RW, NX, ND;
};

// Layout of a code stream: R records of B bits (D of them the domain index)
// in `words` payload words after the 8-word header.
struct StreamGeo {
  long long R, words;
  int B, D, sb, ob;
  uint32_t header[8];
};

// One level of a quadtree encode: its codes (every range of its grid),
// split flags, ranges per row and range side.
struct QtLevel {
  fic_codes codes;
  const uint8_t *split;
  int RW, n;
};
struct QtLevels {
  QtLevel lv[3];
  int L;   // levels (1..3)
  int R0;  // ranges of the top level
};

// Launchers (one per kernel file).  All return hipError_t of the launch.
hipError_t launch_prep(const Geo &g, const void *image, const EncBufs &b,
                       hipStream_t st);
hipError_t launch_seed_dense(const Geo &g, const EncBufs &b, int nblocks,
                             hipStream_t st);
hipError_t launch_search_mfma(const Geo &g, const EncBufs &b,
                              const void *image, int workgroups,
                              hipStream_t st);
hipError_t launch_search_mfma12(const Geo &g, const EncBufs &b,
                                int workgroups, hipStream_t st);
hipError_t launch_search_mfma16(const Geo &g, const EncBufs &b,
                                int workgroups, hipStream_t st);
hipError_t launch_search_mfma12_i8(const Geo &g, const EncBufs &b,
                                   int workgroups, hipStream_t st);
hipError_t launch_search_direct(const Geo &g, const EncBufs &b, int chunks,
                                hipStream_t st);
hipError_t launch_finalize(const Geo &g, const void *image, const EncBufs &b,
                           fic_codes out, hipStream_t st);
hipError_t launch_decode(const Geo &g, const int32_t *domain,
                         const uint8_t *iso, const float *s, const float *o,
                         int iters, float x0, float *traj, hipStream_t st);
hipError_t launch_decode_backward(const Geo &g, const int32_t *domain,
                                  const uint8_t *iso, const float *s,
                                  const float *o, int iters, const float *traj,
                                  const float *grad_xT, float *grad_s,
                                  float *grad_o, void *ws, hipStream_t st);
hipError_t launch_decode_batch(const Geo &g, int n_images,
                               const int32_t *domain, const uint8_t *iso,
                               const float *s, const float *o, int iters,
                               float x0, float *traj, hipStream_t st);
hipError_t launch_decode_scaled(const DecGeo &d, const int32_t *domain,
                                const uint8_t *iso, const float *s,
                                const float *o, int iters, float x0,
                                float *traj, hipStream_t st);
size_t decode_backward_ws_bytes(const Geo &g);
size_t decode_backward_batch_ws_bytes(const Geo &g, int n_images);
bool decode_backward_batch_ok(const Geo &g);
hipError_t launch_decode_backward_batch(const Geo &g, int n_images,
                                        const int32_t *domain,
                                        const uint8_t *iso, const float *s,
                                        int iters, const float *traj,
                                        const float *grad_xT, float *grad_s,
                                        float *grad_o, void *ws,
                                        hipStream_t st);
hipError_t launch_qt_split(int RW, int R, const uint8_t *mask,
                           const double *err, double lim, uint8_t *split,
                           uint8_t *mask_next, hipStream_t st);
hipError_t launch_qt_count(int RW, int R, const uint8_t *split,
                           const int32_t *cnt_next, int32_t *cnt,
                           hipStream_t st);
hipError_t launch_qt_leaves(const QtLevels &q, const int32_t *cnt0,
                            int32_t *off, const fic_quadtree_out &out,
                            hipStream_t st);
hipError_t launch_stream_pack(const StreamGeo &sg, const int32_t *domain,
                              const uint8_t *iso, const uint8_t *s_idx,
                              const uint8_t *o_idx, void *out,
                              hipStream_t st);
hipError_t launch_stream_unpack(const StreamGeo &sg, const void *in,
                                int32_t *domain, uint8_t *iso, uint8_t *s_idx,
                                uint8_t *o_idx, hipStream_t st);
hipError_t launch_prep_batch(const BatchDev &bd, hipStream_t st);
hipError_t launch_compact(const Geo &g, const EncBufs &b, hipStream_t st);
hipError_t launch_compact_batch(const BatchDev &bd, hipStream_t st);
hipError_t launch_seed_batch(const BatchDev &bd, int nblocks, hipStream_t st);
hipError_t launch_search_batch(const BatchDev &bd, hipStream_t st);
size_t refine_ws_bytes(const Geo &g, int iters);
hipError_t launch_refine(const Geo &g, const int32_t *domain, const uint8_t *iso,
                         float *s, float *o, const void *image, int iters,
                         float x0, int steps, float lr_s, float lr_o,
                         double *loss, void *ws, hipStream_t st);

// Search tile: ranges per workgroup of the matrix-core search.
constexpr int kMfmaRangesPerWG = 64;  // 4 waves x 4 row blocks x 4 ranges
constexpr int kMfma12RangesPerWG = 16;
constexpr int kDirectRangesPerWG = 32;
// Workgroups of the batched search's persistent grid (about two per compute
// unit); the work list places code extraction one grid of items behind.
constexpr int kBatchSearchGrid = 512;

// Launch shape of one encode, resolved from the tuning table (fic_tuning.hip)
// with the library defaults for anything the table leaves open.  Always
// 1 <= chunks <= NCB and 0 <= seed_blocks <= NCB.
struct Tune {
  int chunks;       // column chunks per row group of the search grid
  int seed_blocks;  // leading column blocks ranked by the seed pass
  int item_blocks;  // batched search: column blocks per work item
};
Tune resolve_tune(const Geo &g, int method);

// Shared by the host files (defined in fic_abi.hip, which owns the
// thread-local error state).
int abi_fail(int status, const char *msg);
int abi_ok();
int make_geo_for_batch(const fic_params *p, Geo &g);  // encode validation
size_t enc_workspace_bytes(const Geo &g);
EncBufs enc_workspace_bufs(const Geo &g, void *ws);

}  // namespace fic
