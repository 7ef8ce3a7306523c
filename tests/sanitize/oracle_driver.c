/* Drives the oracle's entry points on small and edge-case inputs, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).
 * Exit status 0 when every call returns what the oracle documents. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t oracle_n_ranges(int, int, int);
int64_t oracle_n_domains(int, int, int, int);
int oracle_encode(int, int, int, int, int, int, int, const uint16_t *, int64_t,
                  int64_t, int, int32_t *, uint8_t *, uint8_t *, uint8_t *,
                  double *);
int oracle_decode(int, int, int, int, const int32_t *, const uint8_t *,
                  const double *, const double *, int, double, double *);
int oracle_decode_scaled(int, int, int, int, int, int, const int32_t *,
                         const uint8_t *, const double *, const double *, int,
                         double, double *);
int oracle_decode_backward(int, int, int, int, const int32_t *,
                           const uint8_t *, const double *, const double *,
                           int, const double *, const double *, double *,
                           double *);
int64_t oracle_stream_bytes(int, int, int, int, int, int);
int oracle_stream_pack(int, int, int, int, int, int, int, const int32_t *,
                       const uint8_t *, const uint8_t *, const uint8_t *,
                       uint8_t *, int64_t);
int oracle_stream_unpack(int, int, int, int, int, int, const uint8_t *,
                         int64_t, int32_t *, uint8_t *, uint8_t *, uint8_t *);

static int fails = 0;
#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); ++fails; } } while (0)

static void run(int H, int W, int bits, int n, int step, unsigned seed) {
  const int64_t R = oracle_n_ranges(H, W, n);
  uint16_t *img = malloc(sizeof(uint16_t) * H * W);
  for (int i = 0; i < H * W; ++i) {
    seed = seed * 1103515245u + 12345u;
    img[i] = (uint16_t)((seed >> 16) % (1u << bits));
  }
  int32_t *d = malloc(sizeof(int32_t) * R);
  uint8_t *k = malloc(R), *j = malloc(R), *m = malloc(R);
  double *e = malloc(sizeof(double) * R);
  CHECK(oracle_encode(H, W, bits, n, step, 5, 7, img, 0, R, 1, d, k, j, m, e) == 0);
  double *s = malloc(sizeof(double) * R), *o = malloc(sizeof(double) * R);
  for (int64_t r = 0; r < R; ++r) {
    s[r] = j[r] / 16.0 - 1.0;
    o[r] = m[r] * (2.0 * (1 << bits) / 128) - (1 << bits);
  }
  const int T = 3;
  double *traj = malloc(sizeof(double) * (T + 1) * H * W);
  CHECK(oracle_decode(H, W, n, step, d, k, s, o, T, 128.0, traj) == 0);
  double *gs = malloc(sizeof(double) * R), *go = malloc(sizeof(double) * R);
  CHECK(oracle_decode_backward(H, W, n, step, d, k, s, o, T, traj, traj + T * H * W, gs, go) == 0);
  double *traj2 = malloc(sizeof(double) * (T + 1) * 4 * H * W);
  CHECK(oracle_decode_scaled(H, W, n, step, 2, 1, d, k, s, o, T, 128.0, traj2) == 0);
  CHECK(oracle_decode_scaled(H, W, n, step, 1, 3, d, k, s, o, T, 128.0, traj2) != 0);
  const int64_t nb = oracle_stream_bytes(H, W, n, step, 5, 7);
  uint8_t *st = malloc(nb);
  CHECK(oracle_stream_pack(H, W, bits, n, step, 5, 7, d, k, j, m, st, nb) == 0);
  CHECK(oracle_stream_pack(H, W, bits, n, step, 5, 7, d, k, j, m, st, nb - 1) != 0);
  int32_t *d2 = malloc(sizeof(int32_t) * R);
  uint8_t *k2 = malloc(R), *j2 = malloc(R), *m2 = malloc(R);
  CHECK(oracle_stream_unpack(H, W, n, step, 5, 7, st, nb, d2, k2, j2, m2) == 0);
  CHECK(memcmp(d, d2, sizeof(int32_t) * R) == 0 && memcmp(k, k2, R) == 0 &&
        memcmp(j, j2, R) == 0 && memcmp(m, m2, R) == 0);
  st[0] = 'X';
  CHECK(oracle_stream_unpack(H, W, n, step, 5, 7, st, nb, d2, k2, j2, m2) != 0);
  free(img); free(d); free(k); free(j); free(m); free(e); free(s); free(o);
  free(traj); free(gs); free(go); free(traj2); free(st); free(d2); free(k2);
  free(j2); free(m2);
}

int main(void) {
  run(16, 16, 8, 4, 4, 1u);
  run(24, 40, 12, 4, 3, 2u);
  run(32, 32, 8, 8, 2, 3u);
  run(8, 8, 8, 4, 1, 4u);
  /* invalid geometry is refused, not read */
  CHECK(oracle_encode(10, 16, 8, 4, 4, 5, 7, NULL, 0, 0, 1, NULL, NULL, NULL, NULL, NULL) != 0);
  CHECK(oracle_encode(16, 16, 8, 4, 0, 5, 7, NULL, 0, 0, 1, NULL, NULL, NULL, NULL, NULL) != 0);
  CHECK(oracle_encode(16, 16, 8, 4, 4, 9, 7, NULL, 0, 0, 1, NULL, NULL, NULL, NULL, NULL) != 0);
  if (fails) return 1;
  printf("oracle driver ok\n");
  return 0;
}
