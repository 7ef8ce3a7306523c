/*
 * fic_oracle.c -- CPU reference (test infrastructure only).
 *
 * This file is the slow, obviously-correct oracle that the GPU encoder,
 * decoder and adjoint are checked against.  It is NOT part of the product
 * path: only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no code, header or table with the HIP
 * library.
 *
 * Everything is plain double precision.  All quantities the encoder produces
 * are dyadic rationals with few significant bits (pixels are integers, the
 * contracted domain values are quarter-integers, the contrast grid has step
 * 2^-(s_bits-1), the offset grid is integral), so every sum and residual below
 * is exact in double; the only rounding is the one division of eq. (9).
 *
 * Readings of the paper that this file fixes (the paper leaves them open):
 *  - the contraction tau (Section V, Alg. 1) is the 2x2 mean of the domain;
 *  - the eight transforms (Section V: rotations by 90/180/270 degrees and
 *    mirroring) are: k = 0..3 rotate k quarter turns counter-clockwise,
 *    k = 4..7 mirror left-right first, then rotate (k - 4) quarter turns;
 *  - eq. (9)'s denominator is n*sum(a^2) - (sum a)^2 (the form printed next to
 *    eqs. (11)-(12)); "n" in eqs. (8)-(12) is the pixel count K of a block;
 *  - s and o are quantised: s is fitted (eq. 9, or eq. 11 when the domain has
 *    no variance), rounded half-up onto a 2^s_bits grid over [-1, 1) and
 *    clamped; o is then fitted with that s (eq. 10, eq. 12 when s = 0), rounded
 *    half-up onto a 2^o_bits grid over [-2^bits, 2^bits) and clamped; the
 *    residual (eq. 8) uses the quantised pair;
 *  - domains start on a grid of spacing STEP (Alg. 1), row-major, and must lie
 *    inside the image; the candidate index is c = 8 d + k;
 *  - ties keep the first candidate met in Alg. 2's loop order (strict "<").
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL 1

/* ---------------------------------------------------------------------------
 * Block geometry.
 * ------------------------------------------------------------------------- */

/* Number of range blocks: the image is split into n x n non-overlapping
 * blocks, row-major (Section V; Section VI). */
int64_t oracle_n_ranges(int height, int width, int n) {
  if (n <= 0 || height % n || width % n) return -1;
  return (int64_t)(height / n) * (width / n);
}

/* Domain grid (Alg. 1): top-left corners at multiples of STEP such that the
 * 2n x 2n domain lies inside the image. */
static int domain_axis(int len, int n, int step) {
  if (len < 2 * n) return 0;
  return (len - 2 * n) / step + 1;
}

int64_t oracle_n_domains(int height, int width, int n, int step) {
  if (n <= 0 || step <= 0) return -1;
  return (int64_t)domain_axis(height, n, step) * domain_axis(width, n, step);
}

/* ---------------------------------------------------------------------------
 * Alg. 1: contraction tau of a domain block and the eight transforms S_k.
 * ------------------------------------------------------------------------- */

/* tau: the 2n x 2n block at (Y, X) averaged over 2x2 cells -> n x n. */
void oracle_contract(const uint16_t *img, int width, int Y, int X, int n,
                     double *out) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const uint16_t *p = img + (size_t)(Y + 2 * i) * width + (X + 2 * j);
      double s = (double)p[0] + (double)p[1] + (double)p[width] +
                 (double)p[width + 1];
      out[i * n + j] = s / 4.0;
    }
}

/* One quarter turn counter-clockwise of an n x n block: the new row i is the
 * old column n-1-i, read top to bottom. */
static void rotate_ccw(const double *in, int n, double *out) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[i * n + j] = in[j * n + (n - 1 - i)];
}

/* Mirror left-right. */
static void mirror_lr(const double *in, int n, double *out) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[i * n + j] = in[i * n + (n - 1 - j)];
}

/* S_k: k in 0..7; k >= 4 mirrors first, then (k mod 4) quarter turns.
 * Blocks are at most ORACLE_MAX_N x ORACLE_MAX_N. */
#define ORACLE_MAX_N 32
void oracle_isometry(const double *in, int n, int k, double *out) {
  double a[ORACLE_MAX_N * ORACLE_MAX_N], t[ORACLE_MAX_N * ORACLE_MAX_N];
  if (n <= 0 || n > ORACLE_MAX_N) return;
  if (k >= 4)
    mirror_lr(in, n, a);
  else
    memcpy(a, in, sizeof(double) * n * n);
  for (int q = 0; q < (k & 3); ++q) {
    rotate_ccw(a, n, t);
    memcpy(a, t, sizeof(double) * n * n);
  }
  memcpy(out, a, sizeof(double) * n * n);
}

/* ---------------------------------------------------------------------------
 * Least squares (eqs. 9-12), quantisation, residual (eq. 8).
 * ------------------------------------------------------------------------- */

typedef struct {
  int j;      /* contrast index, s_q = j / 2^(s_bits-1) - 1 */
  int m;      /* offset index,  o_q = m * delta_o - 2^bits */
  double s;   /* s_q */
  double o;   /* o_q */
  double err; /* eq. (8) with (s_q, o_q) */
} fit_t;

static double clampd(double v, double lo, double hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

/* Fit s and o of the map a -> s a + o onto b (K pixels), quantise, and
 * return the residual. */
static fit_t fit_block(const double *a, const double *b, int K, int bits,
                       int s_bits, int o_bits) {
  double sa = 0, saa = 0, sab = 0, sb = 0;
  for (int i = 0; i < K; ++i) {
    sa += a[i];
    saa += a[i] * a[i];
    sab += a[i] * b[i];
    sb += b[i];
  }
  const double nK = (double)K;
  const double var = nK * saa - sa * sa; /* domain variance term */
  double s;
  if (var == 0.0)
    s = 0.0;                                /* eq. (11) */
  else
    s = (nK * sab - sa * sb) / var;         /* eq. (9) */

  const double s_levels = ldexp(1.0, s_bits - 1);
  const double j = clampd(floor((s + 1.0) * s_levels + 0.5), 0.0,
                          ldexp(1.0, s_bits) - 1.0);
  const double s_q = j / s_levels - 1.0;

  const double o = (sb - s_q * sa) / nK;    /* eq. (10); eq. (12) if s_q = 0 */
  const double P = ldexp(1.0, bits);
  const double delta_o = 2.0 * P / ldexp(1.0, o_bits);
  const double m = clampd(floor((o + P) / delta_o + 0.5), 0.0,
                          ldexp(1.0, o_bits) - 1.0);
  const double o_q = m * delta_o - P;

  double r = 0;                             /* eq. (8) */
  for (int i = 0; i < K; ++i) {
    const double e = s_q * a[i] + o_q - b[i];
    r += e * e;
  }
  fit_t f = {(int)j, (int)m, s_q, o_q, r};
  return f;
}

/* Exposed for the unit tests: fit one pair of K-pixel blocks. */
void oracle_fit(const double *a, const double *b, int K, int bits, int s_bits,
                int o_bits, int32_t *j, int32_t *m, double *s, double *o,
                double *err) {
  fit_t f = fit_block(a, b, K, bits, s_bits, o_bits);
  *j = f.j;
  *m = f.m;
  *s = f.s;
  *o = f.o;
  *err = f.err;
}

/* ---------------------------------------------------------------------------
 * Alg. 2 / Alg. 3: the full search.
 * ------------------------------------------------------------------------- */

static int check_params(int height, int width, int bits, int n, int step,
                        int s_bits, int o_bits) {
  if (height <= 0 || width <= 0 || n <= 0 || step <= 0) return OR_EINVAL;
  if (n > ORACLE_MAX_N) return OR_EINVAL;
  if (height % n || width % n) return OR_EINVAL;
  if (2 * n > height || 2 * n > width) return OR_EINVAL;
  if (bits < 1 || bits > 16) return OR_EINVAL;
  /* the code arrays hold one byte per index */
  if (s_bits < 1 || s_bits > 8 || o_bits < 1 || o_bits > bits + 1 ||
      o_bits > 8)
    return OR_EINVAL;
  return OR_OK;
}

/* Alg. 3 for one range: all domains d in row-major order, all eight
 * transforms, least squares, residual; keep the strictly smaller residual. */
static void search_range(int width, int n, const uint16_t *img,
                         const double *pool, int64_t ND, int bits, int s_bits,
                         int o_bits, int64_t r, int32_t *out_domain,
                         uint8_t *out_iso, uint8_t *out_sidx, uint8_t *out_oidx,
                         double *out_err) {
  const int K = n * n;
  const int rw = width / n;
  double b[ORACLE_MAX_N * ORACLE_MAX_N], a[ORACLE_MAX_N * ORACLE_MAX_N];
  const int ry = (int)(r / rw), rx = (int)(r % rw);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      b[i * n + j] = (double)img[(size_t)(ry * n + i) * width + rx * n + j];

  double best = INFINITY;
  int64_t best_d = 0;
  int best_k = 0;
  fit_t best_f = {0, 0, 0, 0, INFINITY};
  for (int64_t d = 0; d < ND; ++d) {
    for (int k = 0; k < 8; ++k) {
      oracle_isometry(pool + (size_t)d * K, n, k, a);
      fit_t f = fit_block(a, b, K, bits, s_bits, o_bits);
      if (f.err < best) {
        best = f.err;
        best_d = d;
        best_k = k;
        best_f = f;
      }
    }
  }
  *out_domain = (int32_t)best_d;
  *out_iso = (uint8_t)best_k;
  *out_sidx = (uint8_t)best_f.j;
  *out_oidx = (uint8_t)best_f.m;
  *out_err = best_f.err;
}

/* Alg. 1: the contracted domains of the grid, row-major. */
static double *build_pool(int height, int width, int n, int step,
                          const uint16_t *img, int64_t *ND) {
  const int K = n * n;
  const int ny = domain_axis(height, n, step), nx = domain_axis(width, n, step);
  *ND = (int64_t)ny * nx;
  double *pool = (double *)malloc(sizeof(double) * (size_t)(*ND) * K);
  for (int dy = 0; dy < ny; ++dy)
    for (int dx = 0; dx < nx; ++dx)
      oracle_contract(img, width, dy * step, dx * step, n,
                      pool + ((size_t)dy * nx + dx) * K);
  return pool;
}

/*
 * Encode the ranges listed in `ranges` (row-major range indices); outputs
 * are indexed by position in the list.  n_threads <= 0 uses OpenMP's
 * default.
 */
int oracle_encode_list(int height, int width, int bits, int n, int step,
                       int s_bits, int o_bits, const uint16_t *img,
                       const int64_t *ranges, int64_t count, int n_threads,
                       int32_t *out_domain, uint8_t *out_iso,
                       uint8_t *out_sidx, uint8_t *out_oidx, double *out_err) {
  if (check_params(height, width, bits, n, step, s_bits, o_bits))
    return OR_EINVAL;
  const int64_t R = oracle_n_ranges(height, width, n);
  for (int64_t i = 0; i < count; ++i)
    if (ranges[i] < 0 || ranges[i] >= R) return OR_EINVAL;
  int64_t ND;
  double *pool = build_pool(height, width, n, step, img, &ND);
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t i = 0; i < count; ++i)
    search_range(width, n, img, pool, ND, bits, s_bits, o_bits, ranges[i],
                 out_domain + i, out_iso + i, out_sidx + i, out_oidx + i,
                 out_err + i);
  free(pool);
  return OR_OK;
}

/* Encode the contiguous ranges [r_begin, r_end). */
int oracle_encode(int height, int width, int bits, int n, int step, int s_bits,
                  int o_bits, const uint16_t *img, int64_t r_begin,
                  int64_t r_end, int n_threads, int32_t *out_domain,
                  uint8_t *out_iso, uint8_t *out_sidx, uint8_t *out_oidx,
                  double *out_err) {
  if (check_params(height, width, bits, n, step, s_bits, o_bits))
    return OR_EINVAL;
  const int64_t R = oracle_n_ranges(height, width, n);
  if (r_begin < 0 || r_end > R || r_begin > r_end) return OR_EINVAL;
  const int64_t count = r_end - r_begin;
  int64_t *ranges = (int64_t *)malloc(sizeof(int64_t) * (size_t)(count + 1));
  for (int64_t i = 0; i < count; ++i) ranges[i] = r_begin + i;
  const int rc = oracle_encode_list(height, width, bits, n, step, s_bits,
                                    o_bits, img, ranges, count, n_threads,
                                    out_domain, out_iso, out_sidx, out_oidx,
                                    out_err);
  free(ranges);
  return rc;
}

/* ---------------------------------------------------------------------------
 * Decoder: iterate the PIFS map (eq. 6) from a constant image.
 * ------------------------------------------------------------------------- */

/* One application of the PIFS map: every range r becomes
 * s_r * S_k(tau(domain d_r of x)) + o_r. */
static void pifs_apply(int height, int width, int n, int step,
                       const int32_t *domain, const uint8_t *iso,
                       const double *s, const double *o, const double *x,
                       double *y) {
  const int K = n * n;
  const int nx = domain_axis(width, n, step);
  const int rw = width / n, rh = height / n;
  double *a = (double *)malloc(sizeof(double) * K);
  double *cell = (double *)malloc(sizeof(double) * K);
  for (int ry = 0; ry < rh; ++ry)
    for (int rx = 0; rx < rw; ++rx) {
      const int r = ry * rw + rx;
      const int Y = (domain[r] / nx) * step, X = (domain[r] % nx) * step;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          const double *p = x + (size_t)(Y + 2 * i) * width + X + 2 * j;
          cell[i * n + j] = (p[0] + p[1] + p[width] + p[width + 1]) / 4.0;
        }
      oracle_isometry(cell, n, iso[r], a);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
          y[(size_t)(ry * n + i) * width + rx * n + j] =
              s[r] * a[i * n + j] + o[r];
    }
  free(a);
  free(cell);
}

/* One application of the map to an arbitrary image x (for the tests). */
int oracle_pifs_apply(int height, int width, int n, int step,
                      const int32_t *domain, const uint8_t *iso,
                      const double *s, const double *o, const double *x,
                      double *y) {
  if (n <= 0 || n > ORACLE_MAX_N || height % n || width % n) return OR_EINVAL;
  pifs_apply(height, width, n, step, domain, iso, s, o, x, y);
  return OR_OK;
}

/* traj holds (iters + 1) images; traj[0] = x0 everywhere. */
int oracle_decode(int height, int width, int n, int step, const int32_t *domain,
                  const uint8_t *iso, const double *s, const double *o,
                  int iters, double x0, double *traj) {
  if (n <= 0 || n > ORACLE_MAX_N || height % n || width % n || iters < 0)
    return OR_EINVAL;
  const size_t HW = (size_t)height * width;
  for (size_t p = 0; p < HW; ++p) traj[p] = x0;
  for (int t = 0; t < iters; ++t)
    pifs_apply(height, width, n, step, domain, iso, s, o, traj + t * HW,
               traj + (t + 1) * HW);
  return OR_OK;
}

/*
 * Decoding at another resolution.  The code of a range refers to a domain by
 * its grid position, not by pixels, so it can be decoded at any size
 * (Section I; Section VI decodes at four times the original size).  Reading
 * used here: at scale z = num / den every length of the partition scales by
 * z -- the image becomes (H z) x (W z), a range n z pixels on a side, a
 * domain 2 n z, the domain grid spacing STEP z -- while the map keeps its
 * definition (each range becomes s S_k(tau(domain)) + o, tau the 2x2 mean)
 * and every range keeps its domain index, transform, s and o.  Needs n z and
 * STEP z to be whole numbers; the domain grid then has the same shape at
 * every scale.  traj holds (iters + 1) images of (H z) x (W z).
 */
int oracle_decode_scaled(int height, int width, int n, int step, int num,
                         int den, const int32_t *domain, const uint8_t *iso,
                         const double *s, const double *o, int iters,
                         double x0, double *traj) {
  if (num <= 0 || den <= 0 || n <= 0 || step <= 0 || height % n || width % n)
    return OR_EINVAL;
  if ((n * num) % den || (step * num) % den) return OR_EINVAL;
  const int nz = n * num / den, sz = step * num / den;
  const int hz = height / n * nz, wz = width / n * nz;
  if (nz < 1 || nz > ORACLE_MAX_N) return OR_EINVAL;
  if (domain_axis(hz, nz, sz) != domain_axis(height, n, step) ||
      domain_axis(wz, nz, sz) != domain_axis(width, n, step))
    return OR_EINVAL;
  return oracle_decode(hz, wz, nz, sz, domain, iso, s, o, iters, x0, traj);
}

/*
 * Reverse-mode derivative of the unrolled decoder.  Given g = dL/dx_T it
 * returns dL/ds and dL/do.  The PIFS map is affine in (s, o) for a fixed
 * x_t (eq. 6), so with u_t = S_k(tau(x_t)) on every range:
 *   dL/ds_r += sum_{p in r} g_{t+1}(p) u_t(p),  dL/do_r += sum_{p in r} g_{t+1}(p),
 *   g_t = (d x_{t+1} / d x_t)^T g_{t+1}: each range pixel sends s_r/4 of its
 *   gradient to each of the four image pixels of the cell it was averaged from.
 */
int oracle_decode_backward(int height, int width, int n, int step,
                           const int32_t *domain, const uint8_t *iso,
                           const double *s, const double *o, int iters,
                           const double *traj, const double *grad_xT,
                           double *grad_s, double *grad_o) {
  if (n <= 0 || n > ORACLE_MAX_N || height % n || width % n || iters < 0)
    return OR_EINVAL;
  (void)o;
  const int K = n * n;
  const int nx = domain_axis(width, n, step);
  const int rw = width / n, rh = height / n;
  const int64_t R = (int64_t)rw * rh;
  const size_t HW = (size_t)height * width;
  double *g = (double *)malloc(sizeof(double) * HW);
  double *gp = (double *)malloc(sizeof(double) * HW);
  double *cell = (double *)malloc(sizeof(double) * K);
  double *u = (double *)malloc(sizeof(double) * K);
  /* where the pixel (i, j) of range r was read from: index map of S_k */
  double *idx = (double *)malloc(sizeof(double) * K);
  double *idxk = (double *)malloc(sizeof(double) * K);
  memcpy(g, grad_xT, sizeof(double) * HW);
  for (int64_t r = 0; r < R; ++r) grad_s[r] = grad_o[r] = 0.0;

  for (int t = iters - 1; t >= 0; --t) {
    const double *x = traj + (size_t)t * HW;
    for (size_t p = 0; p < HW; ++p) gp[p] = 0.0;
    for (int ry = 0; ry < rh; ++ry)
      for (int rx = 0; rx < rw; ++rx) {
        const int r = ry * rw + rx;
        const int Y = (domain[r] / nx) * step, X = (domain[r] % nx) * step;
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j) {
            const double *p = x + (size_t)(Y + 2 * i) * width + X + 2 * j;
            cell[i * n + j] = (p[0] + p[1] + p[width] + p[width + 1]) / 4.0;
            idx[i * n + j] = (double)(i * n + j);
          }
        oracle_isometry(cell, n, iso[r], u);
        oracle_isometry(idx, n, iso[r], idxk); /* source cell of each pixel */
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j) {
            const double gv = g[(size_t)(ry * n + i) * width + rx * n + j];
            grad_s[r] += gv * u[i * n + j];
            grad_o[r] += gv;
            const int c = (int)idxk[i * n + j];
            const int ci = c / n, cj = c % n;
            double *q = gp + (size_t)(Y + 2 * ci) * width + X + 2 * cj;
            const double w = gv * s[r] / 4.0;
            q[0] += w;
            q[1] += w;
            q[width] += w;
            q[width + 1] += w;
          }
      }
    double *tmp = g;
    g = gp;
    gp = tmp;
  }
  free(g);
  free(gp);
  free(cell);
  free(u);
  free(idx);
  free(idxk);
  return OR_OK;
}

/* ---------------------------------------------------------------------------
 * Code stream (Section IV: the codes are saved to the encoding file; Table III
 * reports the size reduction).  The paper gives no file format; this build's
 * format is a 32-byte header followed by one fixed-width record per range.
 *   header (little-endian): bytes 0-3 "PIFS"; 4-7 height; 8-11 width;
 *     12 bit depth; 13 range size n; 14 s_bits; 15 o_bits; 16-19 domain
 *     step; 20 domain bits D; 21-23 zero; 24-31 number of ranges R.
 *   records: range r occupies stream bits [r B, (r + 1) B) of the payload,
 *     B = D + 3 + s_bits + o_bits, D = the bits that index N_d domains
 *     (the smallest D with 2^D >= N_d); within a record, from its first bit:
 *     domain index (D bits), transform (3), contrast index (s_bits), offset
 *     index (o_bits), each field least significant bit first.  Stream bit i
 *     is bit (i mod 8) of payload byte i / 8; the payload is padded with
 *     zero bits to a multiple of 32 bits.
 * The oracle writes and reads the stream one bit at a time.
 * ------------------------------------------------------------------------- */

int oracle_stream_domain_bits(int64_t n_domains) {
  int D = 0;
  while (((int64_t)1 << D) < n_domains) ++D;
  return D;
}

int64_t oracle_stream_bytes(int height, int width, int n, int step,
                            int s_bits, int o_bits) {
  const int64_t R = oracle_n_ranges(height, width, n);
  const int64_t ND = oracle_n_domains(height, width, n, step);
  if (R < 0 || ND <= 0) return -1;
  const int64_t B = oracle_stream_domain_bits(ND) + 3 + s_bits + o_bits;
  return 32 + 4 * ((R * B + 31) / 32);
}

static void put_bits(uint8_t *pay, int64_t *pos, uint64_t v, int nbits) {
  for (int b = 0; b < nbits; ++b, ++*pos)
    if ((v >> b) & 1u) pay[*pos / 8] |= (uint8_t)(1u << (*pos % 8));
}

static uint64_t get_bits(const uint8_t *pay, int64_t *pos, int nbits) {
  uint64_t v = 0;
  for (int b = 0; b < nbits; ++b, ++*pos)
    v |= (uint64_t)((pay[*pos / 8] >> (*pos % 8)) & 1u) << b;
  return v;
}

static void put_le(uint8_t *p, uint64_t v, int nbytes) {
  for (int i = 0; i < nbytes; ++i) p[i] = (uint8_t)(v >> (8 * i));
}

/* Writes the whole stream (header and records) into out (bytes long). */
int oracle_stream_pack(int height, int width, int bits, int n, int step,
                       int s_bits, int o_bits, const int32_t *domain,
                       const uint8_t *iso, const uint8_t *s_idx,
                       const uint8_t *o_idx, uint8_t *out, int64_t bytes) {
  const int64_t need =
      oracle_stream_bytes(height, width, n, step, s_bits, o_bits);
  if (need < 0 || bytes < need) return OR_EINVAL;
  const int64_t R = oracle_n_ranges(height, width, n);
  const int64_t ND = oracle_n_domains(height, width, n, step);
  const int D = oracle_stream_domain_bits(ND);
  memset(out, 0, (size_t)need);
  memcpy(out, "PIFS", 4);
  put_le(out + 4, (uint64_t)height, 4);
  put_le(out + 8, (uint64_t)width, 4);
  out[12] = (uint8_t)bits;
  out[13] = (uint8_t)n;
  out[14] = (uint8_t)s_bits;
  out[15] = (uint8_t)o_bits;
  put_le(out + 16, (uint64_t)step, 4);
  out[20] = (uint8_t)D;
  put_le(out + 24, (uint64_t)R, 8);
  uint8_t *pay = out + 32;
  int64_t pos = 0;
  for (int64_t r = 0; r < R; ++r) {
    if (domain[r] < 0 || domain[r] >= ND || iso[r] > 7 ||
        s_idx[r] >= (1u << s_bits) || o_idx[r] >= (1u << o_bits))
      return OR_EINVAL;
    put_bits(pay, &pos, (uint64_t)domain[r], D);
    put_bits(pay, &pos, iso[r], 3);
    put_bits(pay, &pos, s_idx[r], s_bits);
    put_bits(pay, &pos, o_idx[r], o_bits);
  }
  return OR_OK;
}

/* Reads the R records of a stream whose header matches the geometry. */
int oracle_stream_unpack(int height, int width, int n, int step, int s_bits,
                         int o_bits, const uint8_t *in, int64_t bytes,
                         int32_t *domain, uint8_t *iso, uint8_t *s_idx,
                         uint8_t *o_idx) {
  const int64_t need =
      oracle_stream_bytes(height, width, n, step, s_bits, o_bits);
  if (need < 0 || bytes < need || memcmp(in, "PIFS", 4) != 0) return OR_EINVAL;
  const int64_t R = oracle_n_ranges(height, width, n);
  const int D = oracle_stream_domain_bits(oracle_n_domains(height, width, n, step));
  const uint8_t *pay = in + 32;
  int64_t pos = 0;
  for (int64_t r = 0; r < R; ++r) {
    domain[r] = (int32_t)get_bits(pay, &pos, D);
    iso[r] = (uint8_t)get_bits(pay, &pos, 3);
    s_idx[r] = (uint8_t)get_bits(pay, &pos, s_bits);
    o_idx[r] = (uint8_t)get_bits(pay, &pos, o_bits);
  }
  return OR_OK;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
