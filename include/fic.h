/*
 * fic.h -- C ABI of libfic.so: fractal (PIFS) image encoding and decoding on
 * AMD Instinct MI355X (gfx950).
 *
 * The operations follow the problem statement of "GPU Accelerated Fractal
 * Image Compression for Medical Imaging in Parallel Computing Platform"
 * (arXiv 1404.0774):
 *   - the image is split into n x n non-overlapping range blocks and 2n x 2n
 *     domain blocks on a grid of spacing STEP, each domain contracted 2x2 and
 *     taken under eight square symmetries (Section V, Alg. 1);
 *   - every range is compared with every transformed domain by least squares
 *     and the pair with the smallest residual is kept (eqs. 8-12, Alg. 2-3);
 *   - the code of a range is {domain, transform, s, o} (Alg. 2), decoded by
 *     iterating the partitioned IFS map (eq. 6) towards its attractor
 *     (Section III).
 *
 * Conventions shared by every entry point:
 *   - Every data pointer is a DEVICE pointer owned by the caller (for example
 *     the data_ptr() of a torch tensor).  The library allocates nothing and
 *     frees nothing.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls validate their arguments on the host, enqueue work on `stream`
 *     and return without synchronising; outputs are valid once the stream
 *     has reached the call.
 *   - Return value: FIC_OK (0) or one of the FIC_E_* codes below.  On error
 *     nothing has been enqueued, except for FIC_E_HIP, which reports a failed
 *     launch.  fic_last_error() gives a message for the calling thread.
 *   - Images are row-major, height x width, uint8 (bit_depth 8) or uint16
 *     (bit_depth 12, values 0..4095).
 *   - Ranges are numbered row-major: r = ry * (width / n) + rx.  Domains are
 *     numbered row-major over their grid: d = dy * NX + dx with top-left
 *     corner (dy * STEP, dx * STEP), NX = (width - 2n) / STEP + 1.
 *   - Transform k in 0..7 maps the contracted domain T to the block
 *     B[i][j] = T[sigma_k(i, j)], with m = n - 1:
 *       0 (i, j)      identity            4 (i, m-j)    mirror left-right
 *       1 (j, m-i)    rotate 90 ccw       5 (j, i)      transpose
 *       2 (m-i, m-j)  rotate 180          6 (m-i, j)    mirror top-bottom
 *       3 (m-j, i)    rotate 270 ccw      7 (m-j, m-i)  anti-transpose
 *     The candidate index is c = 8 d + k.
 *   - Quantisation: s = s_idx / 2^(s_bits-1) - 1;
 *     o = o_idx * delta_o - 2^bit_depth with delta_o = 2^(bit_depth+1-o_bits).
 */
#ifndef FIC_H
#define FIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum fic_status {
  FIC_OK = 0,
  FIC_E_INVALID = 1,     /* null pointer, bad geometry, bad count */
  FIC_E_UNSUPPORTED = 2, /* valid request outside what the kernels handle */
  FIC_E_WORKSPACE = 3,   /* workspace smaller than fic_query reported */
  FIC_E_HIP = 4          /* a HIP launch or runtime call failed */
};

enum fic_method {
  FIC_METHOD_MFMA = 0,    /* search as an FP16 matrix-core contraction */
  FIC_METHOD_DIRECT = 1,  /* plain method: LDS-tiled per-candidate sums */
  FIC_METHOD_MFMA_I8 = 2  /* 12-bit images with 8x8 ranges only: the same
                             contraction on the int8 matrix cores (hi/lo
                             pieces of 7 and 6 bits, exact int32 partial
                             products) */
};

typedef struct {
  int32_t height, width; /* pixels; multiples of range_size */
  int32_t bit_depth;     /* 8 or 12 */
  int32_t range_size;    /* n: 4, 8 or 16 (16: 8-bit images, matrix-core
                            method; no adjoint, refinement or batch) */
  int32_t domain_step;   /* STEP >= 1 */
  int32_t s_bits;        /* contrast bits, 1..8 (5 in the reference setup) */
  int32_t o_bits;        /* offset bits, 1..min(8, bit_depth+1) (7) */
  int32_t method;        /* enum fic_method (FIC_METHOD_MFMA_I8: 12-bit) */
  int32_t full_search;   /* 0: skip the candidates whose outcome is fixed
                            (below); 1: every range meets every domain in
                            the contraction.  The codes are identical. */
} fic_params;

/*
 * Shadow blocks.  A range without variance (all pixels equal) ties on every
 * candidate and keeps candidate 0 (Section V: such blocks need no search).
 * A domain without variance fits every range with s = 0 and the range mean
 * (eqs. 11-12), so all such domains tie and only the first can win.  With
 * full_search = 0 the search leaves both kinds out of the contraction and
 * code extraction compares the first flat domain; with full_search = 1 they
 * go through the contraction and the least-squares test like every other
 * candidate (the test rejects them).  Both give the same codes.
 */

/* Codes, one entry per range (structure of arrays, device memory). */
typedef struct {
  int32_t *domain; /* d */
  uint8_t *iso;    /* k */
  uint8_t *s_idx;  /* contrast index */
  uint8_t *o_idx;  /* offset index */
  double *err;     /* residual of eq. (8) with the quantised s and o */
} fic_codes;

/*
 * fic_query -- host only, no GPU work.  Validates `p` and reports the range
 * and domain counts of the partition (Section V: non-overlapping n x n
 * ranges, 2n x 2n domains on a grid of spacing STEP) and the workspace bytes
 * that fic_encode and fic_decode_backward need for these parameters.  Any output pointer may be
 * NULL.  Errors: FIC_E_INVALID (null p, height or width not a multiple of n,
 * 2n larger than a side, STEP < 1, full_search not 0 or 1),
 * FIC_E_UNSUPPORTED (bit_depth not 8 or 12,
 * n not 4, 8 or 16, s_bits/o_bits out of range, more candidates than the
 * packed 64-bit search key can index).
 */
int fic_query(const fic_params *p, int64_t *n_ranges, int64_t *n_domains,
              size_t *encode_ws_bytes, size_t *backward_ws_bytes);

/*
 * fic_encode -- exhaustive range-domain search (Alg. 2 / Alg. 3, eqs. 8-12).
 * For every range, among all candidates c = 8 d + k, keeps the one with the
 * smallest residual after the fit s = eq. (9) (eq. (11) when the domain has
 * no variance), s quantised (round half up, clamped), o = eq. (10) with the
 * quantised s, o quantised the same way.  Ties keep the smallest c.
 *   image      device, height*width pixels (uint8 or uint16, see above)
 *   out        device arrays of n_ranges entries each, written
 *   workspace  device, >= encode_ws_bytes from fic_query, 256-byte aligned;
 *              contents on entry are ignored and on return are undefined
 * The result does not depend on `method`.
 */
int fic_encode(const fic_params *p, const void *image, fic_codes out,
               void *workspace, size_t ws_bytes, void *stream);

/*
 * fic_encode_noalloc -- fic_encode for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid allocation).  Same search, same codes; the workspace is a static
 * 32 MiB device array inside the library (one per device, held from module
 * load until the process ends) instead of a caller buffer.
 *   image, out  as for fic_encode
 * The first call on a device looks up that device's copy of the array
 * (hipGetSymbolAddress); no call allocates or frees memory.  Every call on
 * one device shares its array, which keeps the last call's contents: calls
 * that overlap on one device (two streams, two threads) race and must be
 * serialised by the caller.  fic_search_counts does not apply.
 * Errors: those of fic_encode's validation; FIC_E_WORKSPACE when
 * fic_query's encode_ws_bytes exceeds 32 MiB (nothing is enqueued);
 * FIC_E_HIP.
 */
int fic_encode_noalloc(const fic_params *p, const void *image, fic_codes out,
                       void *stream);

/*
 * fic_search_counts -- host, synchronous.  After an fic_encode of `p` has
 * completed on `workspace`, reports how many ranges and how many domains the
 * search kernel visited (either method): with full_search = 0 those with
 * variance, with full_search = 1 all of them.  The search evaluated
 * 8 * n_ranges * n_domains candidates.
 * Errors: FIC_E_INVALID (null pointers, workspace smaller than fic_query
 * reports), FIC_E_HIP.
 */
/*
 * fic_search_counts -- host, synchronous (waits for the device): how many
 * ranges and domains the last fic_encode into this workspace put through
 * the search.  With full_search = 0 the ranges and domains without variance
 * are left out (their outcome is fixed, eqs. 11-12 and the shadow-block rule
 * of Section V); with full_search = 1 every one is searched.  8 n_ranges
 * n_domains is then the number of candidates evaluated.  `workspace` is the
 * one the encode used.  Errors: FIC_E_INVALID (null pointers, a workspace
 * smaller than fic_query's encode_ws_bytes), FIC_E_HIP.
 */
int fic_search_counts(const fic_params *p, const void *workspace,
                      size_t ws_bytes, int64_t *n_ranges, int64_t *n_domains);

/*
 * Batched encode of many slices of uneven size (each slice an independent
 * fic_encode problem, Alg. 2 / Alg. 3 per slice; the paper encodes one image
 * per kernel launch, Section V).
 * All slices must share bit_depth (8), range_size, s_bits and o_bits; size
 * and domain_step may differ.
 *
 * fic_batch_query -- host only: workspace bytes for the batch.
 * fic_batch_prepare -- host, synchronous: validates the slices, lays out the
 *   workspace (every slice's encode buffers, a slice table and a work list
 *   ordered largest slice first) and copies the table and work list to the
 *   device.  images[s] and out[s] are the slice's device image and device
 *   code arrays, as in fic_encode.  Call it whenever the slice shapes or
 *   pointers change, outside any stream capture.
 * fic_encode_batch -- enqueues the batch on `stream`: one launch per phase
 *   for all slices (operand preparation, list compaction, seed pass,
 *   search); the search runs as a persistent grid that takes work items
 *   from a device counter, and extracts each slice's codes as soon as that
 *   slice's search is complete, while later slices are still searched.  It
 *   performs no allocation and no host-device copy, so a stream capture of
 *   it can be replayed as a graph.  `ticks` (device, n_slices + 1 entries,
 *   may be NULL) receives the GPU's 100 MHz clock at the start of the search
 *   ([0]) and when each slice's codes were written ([1 + s]).  Codes equal
 *   those of fic_encode per slice.
 * Errors: FIC_E_INVALID, FIC_E_UNSUPPORTED (not 8-bit; slice geometry as in
 * fic_query), FIC_E_WORKSPACE, FIC_E_HIP.
 */
int fic_batch_query(const fic_params *slices, int32_t n_slices,
                    size_t *ws_bytes);
int fic_batch_prepare(const fic_params *slices, int32_t n_slices,
                      const void *const *images, const fic_codes *out,
                      void *workspace, size_t ws_bytes);
int fic_encode_batch(const fic_params *slices, int32_t n_slices,
                     void *workspace, size_t ws_bytes, uint64_t *ticks,
                     void *stream);

/*
 * fic_decode -- iterate the partitioned IFS map (eq. 6) `iters` times from
 * the constant image x0 (Section III: the attractor of a contractive map):
 *   x_{t+1}[range r, pixel (i,j)] = s_r * mean2x2(x_t, cell sigma_k(i,j) of
 *                                   domain d_r) + o_r
 * in FP32.  traj receives (iters + 1) images of height*width floats,
 * traj[0] = x0.  domain/iso/s/o hold one entry per range (device).
 * Errors: FIC_E_INVALID (null pointers, iters < 0).
 */
int fic_decode(const fic_params *p, const int32_t *domain, const uint8_t *iso,
               const float *s, const float *o, int32_t iters, float x0,
               float *traj, void *stream);

/*
 * fic_decode_batch -- fic_decode of n_images images that share `p` (size,
 * range size, domain grid), each with its own codes, one launch per
 * iteration for the whole batch.  Codes are packed image after image
 * (domain[b * n_ranges + r], likewise iso, s, o); traj receives image b's
 * trajectory at traj + b * (iters + 1) * height * width, laid out as
 * fic_decode's.  Errors: FIC_E_INVALID (null pointers, iters < 0,
 * n_images < 1), FIC_E_UNSUPPORTED (more than 2^31 pixels in one iterate,
 * more than 65535 images, 16x16 ranges).
 */
int fic_decode_batch(const fic_params *p, int32_t n_images,
                     const int32_t *domain, const uint8_t *iso,
                     const float *s, const float *o, int32_t iters, float x0,
                     float *traj, void *stream);

/*
 * fic_decode_scaled -- fic_decode at another resolution.  A range's code
 * names its domain by grid position, not by pixels, so the codes of a
 * height x width image decode at any size (Section I; Section VI decodes at
 * four times the original size).  At scale z = scale_num / scale_den every
 * length of the partition scales by z: the output is (height z) x (width z),
 * ranges are n z pixels on a side, domains 2 n z, the domain grid spacing
 * STEP z; each range keeps its domain index, transform, s and o, and the map
 * keeps its definition (the transform of the 2x2-mean contraction, times s,
 * plus o).  `p` describes the encoded image (its range and domain counts
 * index the codes).  traj receives (iters + 1) images of
 * (height z) x (width z) floats, traj[0] = x0.  z = 1 is fic_decode.
 * Errors: FIC_E_INVALID (null pointers, iters < 0, scale_num or scale_den
 * < 1, n z or STEP z not a whole number), FIC_E_UNSUPPORTED (an output
 * larger than 2^30 pixels).
 */
int fic_decode_scaled(const fic_params *p, int32_t scale_num,
                      int32_t scale_den, const int32_t *domain,
                      const uint8_t *iso, const float *s, const float *o,
                      int32_t iters, float x0, float *traj, void *stream);

/*
 * fic_decode_backward -- reverse pass of fic_decode with respect to s and o.
 * Given traj from fic_decode (same codes, same iters) and grad_xT = dL/dx_T
 * (height*width floats), writes dL/ds and dL/do (n_ranges floats each,
 * overwritten).  Deterministic: repeated calls give identical bits.
 *   workspace  device, >= backward_ws_bytes from fic_query
 * Errors: FIC_E_INVALID (null pointers, iters < 0, workspace not 256-byte
 * aligned), FIC_E_UNSUPPORTED (16x16 ranges, more than 2^28 pixels),
 * FIC_E_WORKSPACE.
 */
int fic_decode_backward(const fic_params *p, const int32_t *domain,
                        const uint8_t *iso, const float *s, const float *o,
                        int32_t iters, const float *traj, const float *grad_xT,
                        float *grad_s, float *grad_o, void *workspace,
                        size_t ws_bytes, void *stream);

/*
 * fic_decode_backward_batch -- fic_decode_backward of n_images images that
 * share `p`, each with its own codes, one launch per reverse step for the
 * whole batch.  Codes, dL/ds and dL/do are packed image after image
 * (b * n_ranges + r); traj is fic_decode_batch's output (image b at
 * traj + b * (iters + 1) * height * width); grad_xT holds image b's dL/dx_T
 * at grad_xT + b * height * width.  Each image's result is bitwise the
 * single call's.
 *   workspace  device, >= fic_decode_backward_batch_workspace bytes,
 *              256-byte aligned
 * Errors: FIC_E_INVALID (null pointers, iters < 0, n_images < 1, workspace
 * not 256-byte aligned), FIC_E_UNSUPPORTED (more than 65535 images or 2^31
 * pixels in all, 16x16 ranges, more than 8192 ranges or 16384 domains per
 * image), FIC_E_WORKSPACE.
 */
int fic_decode_backward_batch(const fic_params *p, int32_t n_images,
                              const int32_t *domain, const uint8_t *iso,
                              const float *s, const float *o, int32_t iters,
                              const float *traj, const float *grad_xT,
                              float *grad_s, float *grad_o, void *workspace,
                              size_t ws_bytes, void *stream);

/* Workspace bytes fic_decode_backward_batch needs (host only). */
int fic_decode_backward_batch_workspace(const fic_params *p,
                                        int32_t n_images, size_t *bytes);

/*
 * fic_refine -- adjust s and o of fixed codes to lower the error of their
 * decoded attractor against the image (the collage theorem of Section III
 * bounds that error; here it is minimised directly).  Domain and transform
 * indices are held exact.  Runs `steps` Adam steps (beta1 0.9, beta2 0.999,
 * eps 1e-8, learning rates lr_s and lr_o) on
 *     L = mean((x_T - I)^2),   x_T = fic_decode(iters, x0),
 * with gradients from fic_decode_backward; s is kept in [-0.999, 0.999].
 *   s, o      device, n_ranges floats each, updated in place
 *   image     device, the original image (uint8 / uint16 as in fic_encode)
 *   loss      device, steps + 1 doubles: L before each step and after the last
 *   workspace device, >= fic_refine_workspace bytes, 256-byte aligned
 * Errors: FIC_E_INVALID (null pointers, negative iters/steps/rates),
 * FIC_E_UNSUPPORTED (16x16 ranges, more than 2^28 pixels), FIC_E_WORKSPACE.
 */
int fic_refine(const fic_params *p, const int32_t *domain, const uint8_t *iso,
               float *s, float *o, const void *image, int32_t iters, float x0,
               int32_t steps, float lr_s, float lr_o, double *loss,
               void *workspace, size_t ws_bytes, void *stream);

/* Workspace bytes fic_refine needs for these parameters and iters (host). */
int fic_refine_workspace(const fic_params *p, int32_t iters, size_t *bytes);

/*
 * Quadtree (adaptive) ranges (Section V's quadtree method; Section II's
 * adaptive fractal coding).  Every range of side p->range_size (the largest
 * side, n_max) is encoded as by fic_encode; a range whose residual exceeds
 * tau * n^2 (tau: a squared error per pixel) and whose side n is above
 * min_range_size is split into its four quadrants, which are encoded the
 * same way at side n / 2 (2n x 2n domains on the same STEP grid).  Sides
 * are 16 (8-bit images), 8 and 4: up to three levels.  The leaves are
 * written top-level range by top-level range (row-major), each one's leaves
 * in Z order (top-left, top-right, bottom-left, bottom-right, recursively).
 * A leaf's domain index refers to the domain grid of its own side.
 *
 * fic_quadtree_query -- host only: workspace bytes and the largest leaf
 *   count, (height / min_range_size) (width / min_range_size), which the
 *   output arrays must hold.
 * fic_encode_quadtree -- enqueues the levels' searches and the leaf layout
 *   on `stream`.  out: device arrays of at least the largest leaf count
 *   (y, x: the leaf's top-left pixel; size: its side; codes as fic_encode);
 *   *out.n_leaves (device) receives the leaf count.
 * Errors: FIC_E_INVALID (null pointers, tau NaN, min_range_size not a
 * power-of-two fraction of range_size, workspace misaligned),
 * FIC_E_UNSUPPORTED (sides other than 4, 8 and 16, parameters as fic_query),
 * FIC_E_WORKSPACE, FIC_E_HIP.
 */
typedef struct {
  int32_t *y, *x;     /* top-left pixel of each leaf */
  uint8_t *size;      /* side of each leaf */
  fic_codes codes;    /* the leaf's code (domain index on its side's grid) */
  int32_t *n_leaves;  /* [1]: number of leaves written */
} fic_quadtree_out;

int fic_quadtree_query(const fic_params *p, int32_t min_range_size,
                       size_t *ws_bytes, int64_t *max_leaves);
int fic_encode_quadtree(const fic_params *p, int32_t min_range_size,
                        double tau, const void *image, fic_quadtree_out out,
                        void *workspace, size_t ws_bytes, void *stream);

/*
 * Code stream: the codes written compactly for the encoding file (Section
 * IV saves the codes; Table III reports the size reduction).  The paper
 * gives no format; this library's is a 32-byte header and one fixed-width
 * record per range:
 *   header, little-endian: bytes 0-3 "PIFS"; 4-7 height; 8-11 width;
 *     12 bit_depth; 13 range_size; 14 s_bits; 15 o_bits; 16-19 domain_step;
 *     20 D; 21-23 zero; 24-31 number of ranges R.
 *   payload: range r occupies bits [r B, (r + 1) B), B = D + 3 + s_bits +
 *     o_bits, D the smallest number of bits that indexes the N_d domains
 *     (2^D >= N_d); from a record's first bit: domain index (D bits),
 *     transform (3), contrast index (s_bits), offset index (o_bits), each
 *     least significant bit first.  Payload bit i is bit (i mod 8) of payload
 *     byte i / 8, zero-padded to a multiple of 32 bits.
 * Size: 32 + 4 ceil(R B / 32) bytes.  The codes' residuals are not stored.
 *
 * fic_stream_query -- host only: stream bytes and B for `p`.
 * fic_stream_pack -- writes the stream of the codes (device arrays of R
 *   entries) into `out` (device, >= the queried bytes, 4-byte aligned).
 *   Each field is masked to its width, so codes outside their ranges (not
 *   produced by fic_encode) do not spill into neighbouring fields.
 * fic_stream_header -- host only: reads the 32-byte header (host memory)
 *   into `p` (method 0, full_search 0) after checking the magic, the
 *   parameters and that D and R agree with them.
 * fic_stream_unpack -- reads the R records of a stream (device, 4-byte
 *   aligned, >= the queried bytes for `p`) into the code arrays (device);
 *   the header is not read (pass the parameters fic_stream_header returned).
 * Errors: FIC_E_INVALID (null pointers, misalignment, a short or foreign
 * stream), FIC_E_UNSUPPORTED (parameters as fic_query), FIC_E_WORKSPACE
 * (output buffer too small), FIC_E_HIP.
 */
int fic_stream_query(const fic_params *p, size_t *bytes, int32_t *record_bits);
int fic_stream_pack(const fic_params *p, const int32_t *domain,
                    const uint8_t *iso, const uint8_t *s_idx,
                    const uint8_t *o_idx, void *out, size_t out_bytes,
                    void *stream);
int fic_stream_header(const void *header, size_t bytes, fic_params *p);
int fic_stream_unpack(const fic_params *p, const void *in, size_t in_bytes,
                      int32_t *domain, uint8_t *iso, uint8_t *s_idx,
                      uint8_t *o_idx, void *stream);

/*
 * Launch-shape tuning (host only; no GPU work).  The search grid splits the
 * candidate table of eq. (8) into row groups of ranges and column chunks of
 * domains; these entries choose how many chunks (the matrix-core searches
 * launch col_chunks workgroups per row group of all ranges; the 8-bit ones
 * spread them over the row groups of the ranges they search, the 12-bit ones
 * give each searched row group col_chunks chunks and leave the rest idle),
 * how many leading 32-column
 * blocks a seed pass ranks first to give each range a starting bound (the
 * search still covers every block; the 8-bit, n = 8 matrix-core search seeds
 * itself and always resolves this to 0), and how many
 * column blocks one work item of the batched search covers.  Any choice
 * yields the same codes; only speed changes.  An entry applies to encodes
 * with equal bit_depth, range_size and method and at least `min_domains`
 * domains; among those the largest min_domains wins.  A field of 0 (-1 for
 * seed_blocks) keeps the built-in default.  Values are clamped to the
 * problem (at least one chunk; at most every column block).
 *
 * fic_set_tuning -- replaces the table with n_entries entries (0 clears it).
 *   Errors: FIC_E_INVALID (NULL entries with n > 0, a field out of range:
 *   bit_depth 8|12, range_size 4|8|16, method, min_domains >= 0,
 *   col_chunks 0..4096, seed_blocks -1..64, item_blocks 0..4096).
 * fic_load_tuning -- replaces the table with the entries of a JSON file:
 *   every object holding a "bit_depth" key is one entry, read from the
 *   integer keys named like the fields below; other keys are ignored.
 *   Errors: FIC_E_INVALID (unreadable file, malformed JSON, a bad entry);
 *   on error the table is unchanged.
 * fic_get_tuning -- the resolved shape fic_encode would use for `p`
 *   (min_domains reports the domain count of `p`).  Errors as fic_query.
 * The table is process-wide and guarded by a lock; calls may come from any
 * thread, but changing it while another thread encodes gives that encode
 * either the old or the new shape.
 */
typedef struct {
  int32_t bit_depth, range_size, method; /* key */
  int32_t min_domains;                   /* applies from this domain count */
  int32_t col_chunks;  /* column chunks per row group of the search grid */
  int32_t seed_blocks; /* 32-column blocks ranked by the seed; -1 default */
  int32_t item_blocks; /* batched search: column blocks per work item */
} fic_tuning;

int fic_set_tuning(const fic_tuning *entries, int32_t n_entries);
int fic_load_tuning(const char *json_path);
int fic_get_tuning(const fic_params *p, fic_tuning *out);

/*
 * Benchmark support (not needed to encode; the per-phase times set beside
 * the encode times of Table III).  fic_timing_begin enables and
 * resets phase timing: while enabled, every fic_encode records HIP events on
 * its own stream before operand preparation, before the list compaction and
 * seeding pass, before the search, before code extraction and at its end
 * (the most recent 256 calls are kept).  fic_timing_end waits for those
 * events, returns the number of timed calls and the summed milliseconds of
 * each phase (the search phase is the one search kernel launch), and
 * disables timing.  Not thread-safe: meant for a single benchmarking
 * thread.  Errors: FIC_E_HIP
 * (event creation or query failed), FIC_E_INVALID (end without begin).
 */
int fic_timing_begin(void);
int fic_timing_end(int32_t *n_calls, double *ms_prep, double *ms_seed,
                   double *ms_search, double *ms_finalize);

/* Message for a status code; never NULL. */
const char *fic_status_string(int status);

/* Message of the calling thread's last failed call ("" if none). */
const char *fic_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FIC_H */
