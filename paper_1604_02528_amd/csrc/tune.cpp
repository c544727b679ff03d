// Tune table of the selected-inversion library: per (GPU target, ROCm
// version, dtype, node-size bucket) choices of how a supernode's GEMM-1 runs,
// written by the autotuner (paper_1604_02528_amd/tune.py) and read by
// selinv_analyze when selinv_opts.tune_cache names a file.
//
// File format (JSON):
//   {"format": "selinv-tune-1",
//    "entries": [{"arch": "gfx950", "rocm": "7.2.0", "dtype": "c128",
//                 "s_max": 256, "c_max": 4096,
//                 "dense": 1, "ydense": 1, "split_min_k": 320}, ...]}
// A node of width s and |C(K)| = c takes the entry of its dtype with the
// smallest (s_max, c_max) bucket that holds it (s <= s_max, c <= c_max);
// nodes no entry holds keep the library defaults.  Fields:
//   dense        1: X_{C,C} gathered once into a dense buffer; 0: gathered by
//                the GEMM-1 tiles on the fly
//   ydense       1: a dense node's GEMM-1 tiles run in the dense-loader kernel
//                (level schedule; GEMM-2 shares fused on 64 x 64 tiles, in
//                separate items on 128 x 128 ones); 0: in the general kernel,
//                GEMM-2 fused
//   split_min_k  shortest contraction part of a split GEMM-1 (0: library
//                default, < 0: never split)
//   tile         64 or 128: the GEMM-1 tile of a node whose tiles run in the
//                dense-loader kernel (128 x 128 for FP64 plans only; absent: 64)
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include <rocm-core/rocm_version.h>

#include "internal.hpp"

namespace selinv {

namespace {

[[noreturn]] void bad(const std::string &path, const std::string &what) {
  Failure f;
  f.status = SELINV_EINVAL;
  f.msg = "tune table " + path + ": " + what;
  throw f;
}

// A small recursive-descent reader for the subset of JSON the table uses:
// objects, arrays, strings without escapes other than \" and \\, numbers.
struct Reader {
  const std::string &s;
  const std::string &path;
  size_t i = 0;
  void ws() {
    while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
  }
  bool peek(char c) {
    ws();
    return i < s.size() && s[i] == c;
  }
  void expect(char c) {
    ws();
    if (i >= s.size() || s[i] != c) bad(path, std::string("expected '") + c + "' at byte " + std::to_string(i));
    ++i;
  }
  std::string str() {
    expect('"');
    std::string out;
    while (i < s.size() && s[i] != '"') {
      if (s[i] == '\\' && i + 1 < s.size()) ++i;
      out.push_back(s[i++]);
    }
    expect('"');
    return out;
  }
  double num() {
    ws();
    const char *b = s.c_str() + i;
    char *e = nullptr;
    const double v = std::strtod(b, &e);
    if (e == b) bad(path, "expected a number at byte " + std::to_string(i));
    i += (size_t)(e - b);
    return v;
  }
  // Skip any value (for fields the reader does not use).
  void skip() {
    ws();
    if (peek('"')) {
      str();
    } else if (peek('{')) {
      expect('{');
      if (!peek('}'))
        do {
          str();
          expect(':');
          skip();
        } while (peek(',') && (expect(','), true));
      expect('}');
    } else if (peek('[')) {
      expect('[');
      if (!peek(']'))
        do skip();
        while (peek(',') && (expect(','), true));
      expect(']');
    } else if (s.compare(i, 4, "true") == 0 || s.compare(i, 4, "null") == 0) {
      i += 4;
    } else if (s.compare(i, 5, "false") == 0) {
      i += 5;
    } else {
      num();
    }
  }
};

TuneEntry read_entry(Reader &r) {
  TuneEntry e;
  r.expect('{');
  if (!r.peek('}')) {
    do {
      const std::string k = r.str();
      r.expect(':');
      if (k == "arch") e.arch = r.str();
      else if (k == "rocm") e.rocm = r.str();
      else if (k == "dtype") e.dtype = r.str();
      else if (k == "s_max") e.s_max = (int64_t)r.num();
      else if (k == "c_max") e.c_max = (int64_t)r.num();
      else if (k == "dense") e.dense = (int)r.num();
      else if (k == "ydense") e.ydense = (int)r.num();
      else if (k == "split_min_k") e.split_min_k = (int)r.num();
      else if (k == "tile") {
        e.tile = (int)r.num();
        if (e.tile != 64 && e.tile != 128) bad(r.path, "\"tile\" must be 64 or 128");
      } else r.skip();
    } while (r.peek(',') && (r.expect(','), true));
  }
  r.expect('}');
  return e;
}

}  // namespace

const char *tune_arch() { return "gfx950"; }

std::string tune_rocm() {
  return std::to_string(ROCM_VERSION_MAJOR) + "." + std::to_string(ROCM_VERSION_MINOR) + "." +
         std::to_string(ROCM_VERSION_PATCH);
}

TuneTable load_tune_table(const std::string &path, const std::string &dtype) {
  FILE *f = std::fopen(path.c_str(), "rb");
  if (!f) bad(path, "cannot open");
  std::string text;
  char buf[65536];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
  std::fclose(f);
  Reader r{text, path};
  TuneTable t;
  bool format_ok = false;
  r.expect('{');
  if (!r.peek('}')) {
    do {
      const std::string k = r.str();
      r.expect(':');
      if (k == "format") {
        format_ok = r.str() == "selinv-tune-1";
      } else if (k == "entries") {
        r.expect('[');
        if (!r.peek(']')) {
          do {
            TuneEntry e = read_entry(r);
            if (e.arch == tune_arch() && e.rocm == tune_rocm() && e.dtype == dtype && e.s_max > 0 && e.c_max >= 0)
              t.entries.push_back(e);
          } while (r.peek(',') && (r.expect(','), true));
        }
        r.expect(']');
      } else {
        r.skip();
      }
    } while (r.peek(',') && (r.expect(','), true));
  }
  r.expect('}');
  if (!format_ok) bad(path, "missing or unknown \"format\" (want \"selinv-tune-1\")");
  return t;
}

const TuneEntry *TuneTable::find(int64_t s, int64_t c) const {
  const TuneEntry *best = nullptr;
  for (const TuneEntry &e : entries)
    if (s <= e.s_max && c <= e.c_max &&
        (!best || e.s_max < best->s_max || (e.s_max == best->s_max && e.c_max < best->c_max)))
      best = &e;
  return best;
}

}  // namespace selinv
