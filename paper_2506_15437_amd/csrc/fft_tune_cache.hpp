// The batched path's tuning cache: plain host C++ (no HIP), so that its
// parsing can be checked without a GPU.
//
// One line per tuned shape set:
//   <key> <grid_mult> <order> <group_kib> <variants>
// key       : 16 hex digits (hash of the shape set and the kernel table version)
// grid_mult : persistent workgroups per CU, 1 ... 3 (the values the plan's XCC
//             probe checks)
// order     : 0 (all row items, then all column items) or 1 (chunked)
// group_kib : data per item group, 64, 256 or 1024
// variants  : 2 x kVariantSlots characters '0' / '1', the radix/tile variant
//             of every row length 2^j (first half) and column length 2^j
//             (second half), j = 0 ... kVariantSlots - 1
// A line that does not match this format is ignored; when several valid
// lines carry the key, the last one wins (a re-tune appends).
#pragma once

#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>

namespace fft2d {
namespace tune {

constexpr int kVariantSlots = 15;  // lengths 2^0 ... 2^14

struct Choice {
  int grid_mult = 2;
  int order = 1;
  int group_kib = 256;
  unsigned char variant[2][kVariantSlots] = {};  // [0 row / 1 column][log2 length]
};

inline bool valid_group_kib(int g) { return g == 64 || g == 256 || g == 1024; }

inline std::string variants_string(const Choice& c) {
  std::string s;
  for (int m = 0; m < 2; ++m)
    for (int j = 0; j < kVariantSlots; ++j) s += c.variant[m][j] ? '1' : '0';
  return s;
}

// Parses one line; true (and *out set) only for a well-formed line with this key.
inline bool parse_line(const std::string& line, const std::string& key, Choice* out) {
  std::istringstream ls(line);
  std::string k, var, extra;
  int m = 0, o = -1, g = 0;
  if (!(ls >> k >> m >> o >> g >> var)) return false;
  if (ls >> extra) return false;
  if (k != key || m < 1 || m > 3 || (o != 0 && o != 1) || !valid_group_kib(g)) return false;
  if ((int)var.size() != 2 * kVariantSlots) return false;
  Choice c;
  c.grid_mult = m;
  c.order = o;
  c.group_kib = g;
  for (int i = 0; i < 2 * kVariantSlots; ++i) {
    if (var[(size_t)i] != '0' && var[(size_t)i] != '1') return false;
    c.variant[i / kVariantSlots][i % kVariantSlots] = var[(size_t)i] == '1';
  }
  *out = c;
  return true;
}

inline std::string format_line(const std::string& key, const Choice& c) {
  return key + " " + std::to_string(c.grid_mult) + " " + std::to_string(c.order) + " " +
         std::to_string(c.group_kib) + " " + variants_string(c);
}

// The last valid line for `key` in the file at `path`; false if the file is
// missing, unreadable, or has no such line.
inline bool lookup(const std::string& path, const std::string& key, Choice* out) {
  if (path.empty()) return false;
  std::ifstream in(path);
  if (!in) return false;
  std::string line;
  bool found = false;
  Choice c;
  while (std::getline(in, line)) {
    if (parse_line(line, key, &c)) {
      *out = c;
      found = true;
    }
  }
  return found;
}

}  // namespace tune
}  // namespace fft2d
