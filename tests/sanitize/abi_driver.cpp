// Drives the host side of libfic's C ABI (argument validation, the JSON
// reader of the tuning table, the code-stream header) with malformed and
// edge-case inputs, for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host pass.  Never calls into the GPU:
// every call here fails validation or is host-only.  argv[1]: a scratch
// directory for the JSON files.
#include <stdio.h>
#include <string.h>

#include <string>

#include "../../include/fic.h"

static int fails = 0;
#define CHECK(c)                                                       \
  do {                                                                 \
    if (!(c)) {                                                        \
      fprintf(stderr, "check failed: %s (line %d): %s\n", #c, __LINE__, \
              fic_last_error());                                       \
      ++fails;                                                         \
    }                                                                  \
  } while (0)

static fic_params params(int H, int W, int bits, int n, int step) {
  fic_params p;
  memset(&p, 0, sizeof p);
  p.height = H;
  p.width = W;
  p.bit_depth = bits;
  p.range_size = n;
  p.domain_step = step;
  p.s_bits = 5;
  p.o_bits = 7;
  return p;
}

static int load_json(const std::string &dir, const char *name,
                     const std::string &text) {
  const std::string path = dir + "/" + name;
  FILE *f = fopen(path.c_str(), "wb");
  if (!f) return -1;
  fwrite(text.data(), 1, text.size(), f);
  fclose(f);
  return fic_load_tuning(path.c_str());
}

int main(int argc, char **argv) {
  const std::string dir = argc > 1 ? argv[1] : "/tmp";
  // geometry validation
  int64_t nr, nd;
  size_t ew, bw;
  fic_params p = params(512, 512, 8, 8, 4);
  CHECK(fic_query(&p, &nr, &nd, &ew, &bw) == FIC_OK && nr == 4096 && nd == 15625);
  const int bad[][5] = {{500, 512, 8, 8, 4}, {512, 512, 10, 8, 4}, {512, 512, 8, 6, 4},
                        {512, 512, 8, 8, 0}, {8, 8, 8, 8, 4}, {0, 0, 8, 4, 4},
                        {-4, 16, 8, 4, 4}, {1 << 16, 1 << 16, 8, 8, 4},
                        {2048, 2048, 12, 8, 1}};
  for (const auto &b : bad) {
    fic_params q = params(b[0], b[1], b[2], b[3], b[4]);
    CHECK(fic_query(&q, &nr, &nd, &ew, &bw) != FIC_OK);
  }
  fic_params q = p;
  q.full_search = 7;
  CHECK(fic_query(&q, nullptr, nullptr, nullptr, nullptr) == FIC_E_INVALID);
  q = p;
  q.o_bits = 9;
  CHECK(fic_query(&q, nullptr, nullptr, nullptr, nullptr) == FIC_E_UNSUPPORTED);
  CHECK(fic_query(nullptr, nullptr, nullptr, nullptr, nullptr) == FIC_E_INVALID);
  // entry points refuse before any device work
  fic_codes none;
  memset(&none, 0, sizeof none);
  CHECK(fic_encode(&p, nullptr, none, nullptr, 0, nullptr) == FIC_E_INVALID);
  CHECK(fic_decode(&p, nullptr, nullptr, nullptr, nullptr, 12, 128.f, nullptr,
                   nullptr) == FIC_E_INVALID);
  CHECK(fic_decode_scaled(&p, 1, 3, nullptr, nullptr, nullptr, nullptr, 12,
                          128.f, nullptr, nullptr) == FIC_E_INVALID);
  CHECK(fic_decode_batch(&p, 0, nullptr, nullptr, nullptr, nullptr, 12, 128.f,
                         nullptr, nullptr) == FIC_E_INVALID);
  size_t sb;
  int32_t rb;
  CHECK(fic_stream_query(&p, &sb, &rb) == FIC_OK && rb == 29);
  // batch planning (host only)
  fic_params sl[3] = {params(64, 64, 8, 8, 8), params(128, 96, 8, 8, 4),
                      params(256, 256, 8, 8, 8)};
  size_t bb = 0;
  CHECK(fic_batch_query(sl, 3, &bb) == FIC_OK && bb > 0);
  sl[1].range_size = 4;
  CHECK(fic_batch_query(sl, 3, &bb) == FIC_E_INVALID);
  CHECK(fic_batch_query(sl, 0, &bb) == FIC_E_INVALID);
  // stream header: a good one, then corruptions
  unsigned char h[32];
  memset(h, 0, sizeof h);
  memcpy(h, "PIFS", 4);
  const unsigned v[] = {512, 512};
  memcpy(h + 4, &v[0], 4);
  memcpy(h + 8, &v[1], 4);
  h[12] = 8; h[13] = 8; h[14] = 5; h[15] = 7;
  const unsigned step = 4;
  memcpy(h + 16, &step, 4);
  h[20] = 14;
  const unsigned long long R = 4096;
  memcpy(h + 24, &R, 8);
  fic_params got;
  CHECK(fic_stream_header(h, 32, &got) == FIC_OK && got.height == 512 &&
        got.domain_step == 4);
  for (int at = 0; at < 32; ++at) {
    unsigned char c[32];
    memcpy(c, h, 32);
    c[at] ^= 0xA5;
    fic_stream_header(c, 32, &got);  // any status; must not misbehave
  }
  unsigned char huge[32];
  memcpy(huge, h, 32);
  memset(huge + 4, 0xFF, 8);  // 4 billion pixels a side
  CHECK(fic_stream_header(huge, 32, &got) != FIC_OK);
  CHECK(fic_stream_header(h, 31, &got) == FIC_E_INVALID);
  // the tuning table's JSON reader
  CHECK(load_json(dir, "ok.json",
                  "{\"entries\": [{\"bit_depth\": 8, \"range_size\": 8, \"method\": 0, "
                  "\"col_chunks\": 6, \"sweep\": [1, 2.5, \"x\", null, true]}]}") == FIC_OK);
  fic_tuning t;
  CHECK(fic_get_tuning(&p, &t) == FIC_OK && t.col_chunks == 6);
  const char *malformed[] = {
      "", "{", "[", "{\"entries\": [", "{\"a\": }", "{\"a\" 1}", "[1, 2,]",
      "{\"bit_depth\": 8.5, \"range_size\": 8, \"method\": 0}",
      "{\"bit_depth\": 1e300, \"range_size\": 8, \"method\": 0}",
      "{\"bit_depth\": -1e300, \"range_size\": 8, \"method\": 0}",
      "{\"bit_depth\": nan, \"range_size\": 8, \"method\": 0}",
      "{\"bit_depth\": 8, \"range_size\": 8, \"method\": 0, \"col_chunks\": 99999}",
      "\"unterminated", "{\"k\\", "tru", "nul", "[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[1]]]]",
      "{\"bit_depth\": 8} trailing"};
  int i = 0;
  for (const char *m : malformed) {
    const std::string name = "bad" + std::to_string(i++) + ".json";
    CHECK(load_json(dir, name.c_str(), m) == FIC_E_INVALID);
  }
  CHECK(fic_get_tuning(&p, &t) == FIC_OK && t.col_chunks == 6);  // unchanged
  CHECK(fic_load_tuning((dir + "/missing.json").c_str()) == FIC_E_INVALID);
  CHECK(fic_set_tuning(nullptr, 0) == FIC_OK);
  CHECK(fic_status_string(12345) != nullptr);
  if (fails) return 1;
  printf("abi driver ok\n");
  return 0;
}
