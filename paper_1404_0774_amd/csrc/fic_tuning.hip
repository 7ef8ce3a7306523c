// fic_tuning.hip -- host-only table of launch shapes for the search.
//
// The search grid is split into row groups (ranges) and column chunks
// (domains); how many chunks, how many leading column blocks the dense seed
// pass fits, and how long a work item of the batched search is are choices
// that depend on the device and on the problem size.  They change speed
// only: every choice gives the same codes.  The table maps
// (bit depth, range size, method, lower bound on the domain count) to such
// a choice; anything it leaves open takes the built-in default.
#include <ctype.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "fic_internal.h"

namespace fic {
namespace {

std::mutex g_mu;
std::vector<fic_tuning> g_table;

constexpr int kMaxChunks = 4096;
constexpr int kMaxSeedBlocks = 64;
constexpr int kMaxItemBlocks = 4096;

// Built-in defaults: about two workgroups per compute unit (256 CUs) in the
// search launch (the 12-bit matrix-core searches about 24, which the compute
// units take in turn, so the launch ends evenly), one seed block (ranked for
// a starting bound) once there are 16 or more column blocks, 16 column
// blocks per batched work item.
Tune default_tune(const Geo &g, int method) {
  const int per_wg =
      ((g.bits == 12 && method != FIC_METHOD_DIRECT) || g.n == 16)
          ? kMfma12RangesPerWG
          : kMfmaRangesPerWG;
  const int row_groups = std::max(1, g.R_pad / per_wg);
  Tune t;
  t.seed_blocks = g.NCB >= 16 ? 1 : 0;
  const int target = g.bits == 12 && method != FIC_METHOD_DIRECT ? 6144 : 512;
  t.chunks = (target + row_groups - 1) / row_groups;
  t.item_blocks = 16;
  return t;
}

bool valid_entry(const fic_tuning &e, char *msg, size_t len) {
  if (e.bit_depth != 8 && e.bit_depth != 12) {
    snprintf(msg, len, "tuning entry: bit_depth %d (8 or 12)", e.bit_depth);
    return false;
  }
  if (e.range_size != 4 && e.range_size != 8 && e.range_size != 16) {
    snprintf(msg, len, "tuning entry: range_size %d (4, 8 or 16)",
             e.range_size);
    return false;
  }
  if (e.method != FIC_METHOD_MFMA && e.method != FIC_METHOD_DIRECT &&
      e.method != FIC_METHOD_MFMA_I8) {
    snprintf(msg, len, "tuning entry: method %d", e.method);
    return false;
  }
  if (e.min_domains < 0) {
    snprintf(msg, len, "tuning entry: min_domains %d < 0", e.min_domains);
    return false;
  }
  if (e.col_chunks < 0 || e.col_chunks > kMaxChunks) {
    snprintf(msg, len, "tuning entry: col_chunks %d outside 0..%d",
             e.col_chunks, kMaxChunks);
    return false;
  }
  if (e.seed_blocks < -1 || e.seed_blocks > kMaxSeedBlocks) {
    snprintf(msg, len, "tuning entry: seed_blocks %d outside -1..%d",
             e.seed_blocks, kMaxSeedBlocks);
    return false;
  }
  if (e.item_blocks < 0 || e.item_blocks > kMaxItemBlocks) {
    snprintf(msg, len, "tuning entry: item_blocks %d outside 0..%d",
             e.item_blocks, kMaxItemBlocks);
    return false;
  }
  return true;
}

int set_table(const fic_tuning *entries, int n) {
  if (n < 0) return abi_fail(FIC_E_INVALID, "tuning: n_entries < 0");
  if (n > 0 && !entries) return abi_fail(FIC_E_INVALID, "tuning: entries NULL");
  char msg[160];
  for (int i = 0; i < n; ++i)
    if (!valid_entry(entries[i], msg, sizeof msg))
      return abi_fail(FIC_E_INVALID, msg);
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.assign(entries, entries + n);
  return abi_ok();
}

// ---- a reader for the one JSON shape the autotuner writes -----------------
// {"entries": [{"bit_depth": 8, "range_size": 8, ...}, ...], ...}: every
// object that holds a "bit_depth" key is an entry; integer fields only,
// other keys (timings, device names) are skipped.

struct Reader {
  const char *p, *end;
  std::string err;

  void ws() {
    while (p < end && isspace((unsigned char)*p)) ++p;
  }
  bool fail(const char *m) {
    if (err.empty()) err = m;
    return false;
  }
  bool string(std::string &out) {
    ws();
    if (p >= end || *p != '"') return fail("expected a string");
    ++p;
    out.clear();
    while (p < end && *p != '"') {
      if (*p == '\\') {
        if (++p >= end) break;
      }
      out.push_back(*p++);
    }
    if (p >= end) return fail("unterminated string");
    ++p;
    return true;
  }
  bool number(double &v) {
    ws();
    char *q = nullptr;
    v = strtod(p, &q);
    if (q == p) return fail("expected a number");
    p = q;
    return true;
  }
  bool literal(const char *w) {
    const size_t n = strlen(w);
    if ((size_t)(end - p) < n || strncmp(p, w, n) != 0)
      return fail("unexpected token");
    p += n;
    return true;
  }
  // any value; objects holding "bit_depth" are appended to `out`
  bool value(std::vector<fic_tuning> &out, int depth) {
    if (depth > 32) return fail("nesting too deep");
    ws();
    if (p >= end) return fail("unexpected end of input");
    if (*p == '{') return object(out, depth);
    if (*p == '[') {
      ++p;
      ws();
      if (p < end && *p == ']') {
        ++p;
        return true;
      }
      for (;;) {
        if (!value(out, depth + 1)) return false;
        ws();
        if (p < end && *p == ',') {
          ++p;
          continue;
        }
        if (p < end && *p == ']') {
          ++p;
          return true;
        }
        return fail("expected , or ] in array");
      }
    }
    if (*p == '"') {
      std::string s;
      return string(s);
    }
    if (*p == 't') return literal("true");
    if (*p == 'f') return literal("false");
    if (*p == 'n') return literal("null");
    double v;
    return number(v);
  }
  bool object(std::vector<fic_tuning> &out, int depth) {
    ++p;  // '{'
    fic_tuning e;
    e.bit_depth = e.range_size = e.method = -1;
    e.min_domains = 0;
    e.col_chunks = 0;
    e.seed_blocks = -1;
    e.item_blocks = 0;
    bool is_entry = false;
    ws();
    if (p < end && *p == '}') {
      ++p;
      return true;
    }
    for (;;) {
      std::string key;
      if (!string(key)) return false;
      ws();
      if (p >= end || *p != ':') return fail("expected : after key");
      ++p;
      int32_t *field = nullptr;
      if (key == "bit_depth") field = &e.bit_depth, is_entry = true;
      else if (key == "range_size") field = &e.range_size;
      else if (key == "method") field = &e.method;
      else if (key == "min_domains") field = &e.min_domains;
      else if (key == "col_chunks") field = &e.col_chunks;
      else if (key == "seed_blocks") field = &e.seed_blocks;
      else if (key == "item_blocks") field = &e.item_blocks;
      if (field) {
        double v;
        if (!number(v)) return false;
        // range first: converting an out-of-range double to int is undefined
        if (!(v >= -2147483648.0 && v <= 2147483647.0) || v != floor(v))
          return fail("tuning field is not a 32-bit integer");
        *field = (int32_t)v;
      } else if (!value(out, depth + 1)) {
        return false;
      }
      ws();
      if (p < end && *p == ',') {
        ++p;
        continue;
      }
      if (p < end && *p == '}') {
        ++p;
        break;
      }
      return fail("expected , or } in object");
    }
    if (is_entry) out.push_back(e);
    return true;
  }
};

}  // namespace

Tune resolve_tune(const Geo &g, int method) {
  Tune t = default_tune(g, method);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    const fic_tuning *pick = nullptr;
    for (const fic_tuning &e : g_table) {
      if (e.bit_depth != g.bits || e.range_size != g.n || e.method != method ||
          e.min_domains > g.ND)
        continue;
      if (!pick || e.min_domains >= pick->min_domains) pick = &e;
    }
    if (pick) {
      if (pick->col_chunks > 0) t.chunks = pick->col_chunks;
      if (pick->seed_blocks >= 0) t.seed_blocks = pick->seed_blocks;
      if (pick->item_blocks > 0) t.item_blocks = pick->item_blocks;
    }
  }
  t.seed_blocks = std::max(0, std::min(t.seed_blocks, g.NCB));
  // the 8-bit, n = 8 matrix-core search seeds itself and has no range
  // operand for the seed pass to read
  if (method == FIC_METHOD_MFMA && g.bits == 8 && g.n == 8) t.seed_blocks = 0;
  // 16x16 ranges keep centred operands, which the seed pass does not read
  if (g.n == 16) t.seed_blocks = 0;
  t.chunks = std::max(1, std::min(t.chunks, g.NCB));
  t.item_blocks = std::max(1, t.item_blocks);
  return t;
}

}  // namespace fic

using namespace fic;

extern "C" {

int fic_set_tuning(const fic_tuning *entries, int32_t n_entries) {
  return set_table(entries, n_entries);
}

int fic_load_tuning(const char *json_path) {
  if (!json_path) return abi_fail(FIC_E_INVALID, "tuning: path is NULL");
  FILE *f = fopen(json_path, "rb");
  if (!f) {
    std::string m = std::string("tuning: cannot open ") + json_path;
    return abi_fail(FIC_E_INVALID, m.c_str());
  }
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof buf, f)) > 0) {
    text.append(buf, got);
    if (text.size() > (16u << 20)) break;
  }
  fclose(f);
  if (text.size() > (16u << 20))
    return abi_fail(FIC_E_INVALID, "tuning: file larger than 16 MiB");
  Reader rd{text.data(), text.data() + text.size(), {}};
  std::vector<fic_tuning> entries;
  if (!rd.value(entries, 0)) {
    std::string m = "tuning: " + rd.err + " at byte " +
                    std::to_string(rd.p - text.data());
    return abi_fail(FIC_E_INVALID, m.c_str());
  }
  rd.ws();
  if (rd.p != rd.end) return abi_fail(FIC_E_INVALID, "tuning: trailing text");
  return set_table(entries.data(), (int)entries.size());
}

int fic_get_tuning(const fic_params *p, fic_tuning *out) {
  if (!out) return abi_fail(FIC_E_INVALID, "tuning: out is NULL");
  Geo g;
  const int st = make_geo_for_batch(p, g);
  if (st) return st;
  const Tune t = resolve_tune(g, p->method);
  out->bit_depth = p->bit_depth;
  out->range_size = p->range_size;
  out->method = p->method;
  out->min_domains = g.ND;
  out->col_chunks = t.chunks;
  out->seed_blocks = t.seed_blocks;
  out->item_blocks = t.item_blocks;
  return abi_ok();
}

}  // extern "C"
