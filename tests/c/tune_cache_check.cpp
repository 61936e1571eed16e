// CPU check of the batched path's tuning-cache parsing
// (paper_2506_15437_amd/csrc/fft_tune_cache.hpp), built with g++ and run by
// tests/test_host.py with a scratch folder as its argument.
//
// A missing file, an empty file, a file of binary junk and every kind of
// malformed line yield no choice (the plan then tunes or keeps its defaults);
// a valid line is found among junk, the last valid line for a key wins, and a
// line written by format_line parses back to the same choice.
#include "../../paper_2506_15437_amd/csrc/fft_tune_cache.hpp"

#include <cstdio>
#include <cstring>
#include <fstream>
#include <string>

using namespace fft2d::tune;

namespace {

int failures = 0;

void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAIL %s\n", what);
    ++failures;
  }
}

void write(const std::string& path, const std::string& text) {
  std::ofstream out(path, std::ios::binary | std::ios::trunc);
  out << text;
}

bool same(const Choice& a, const Choice& b) {
  return a.grid_mult == b.grid_mult && a.order == b.order && a.group_kib == b.group_kib &&
         std::memcmp(a.variant, b.variant, sizeof(a.variant)) == 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  const std::string dir = argv[1];
  const std::string key = "0123456789abcdef";
  const std::string zeros(2 * kVariantSlots, '0');
  Choice c;
  c.grid_mult = 3;
  c.order = 0;
  c.group_kib = 1024;
  c.variant[0][8] = 1;
  c.variant[1][11] = 1;
  const std::string good = format_line(key, c);
  Choice got;

  expect(!lookup(dir + "/missing.txt", key, &got), "missing file");
  expect(!lookup("", key, &got), "empty path");
  write(dir + "/empty.txt", "");
  expect(!lookup(dir + "/empty.txt", key, &got), "empty file");
  std::string junk;
  for (int i = 0; i < 4096; ++i) junk += (char)((i * 7919) & 0xff);
  write(dir + "/junk.txt", junk);
  expect(!lookup(dir + "/junk.txt", key, &got), "binary junk");

  const char* bad[] = {
      "",                                                  // empty line
      "0123456789abcdef",                                  // key only
      "0123456789abcdef 2 1 256",                          // old format, no variants
      "0123456789abcdef 4 1 256 ZEROS",                    // grid multiplier the probe never checked
      "0123456789abcdef 0 1 256 ZEROS",                    // grid multiplier 0
      "0123456789abcdef 2 2 256 ZEROS",                    // order 2
      "0123456789abcdef 2 1 128 ZEROS",                    // group size not offered
      "0123456789abcdef 2 1 256 0101",                     // variants too short
      "0123456789abcdef 2 1 256 ZEROS0",                   // variants too long
      "0123456789abcdef 2 1 256 ZEROS extra",              // trailing field
      "0123456789abcdef two 1 256 ZEROS",                  // not a number
      "fedcba9876543210 2 1 256 ZEROS",                    // another key
  };
  for (const char* b : bad) {
    std::string line = b;
    const size_t z = line.find("ZEROS");
    if (z != std::string::npos) line.replace(z, 5, zeros);
    write(dir + "/bad.txt", line + "\n");
    if (lookup(dir + "/bad.txt", key, &got)) {
      std::printf("FAIL accepted malformed line: %s\n", b);
      ++failures;
    }
  }
  {
    std::string line = key + " 2 1 256 " + zeros;
    line[line.size() - 3] = '2';  // a variant digit other than 0 / 1
    write(dir + "/bad.txt", line + "\n");
    expect(!lookup(dir + "/bad.txt", key, &got), "variant digit 2");
  }

  // a valid line among junk is found and parses back to what was written
  write(dir + "/mixed.txt", junk.substr(0, 100) + "\n" + "garbage line\n" + good + "\n" + "0123 1 1\n");
  expect(lookup(dir + "/mixed.txt", key, &got) && same(got, c), "valid line among junk");
  // the last valid line wins
  Choice d = c;
  d.grid_mult = 1;
  d.variant[0][8] = 0;
  write(dir + "/two.txt", good + "\n" + format_line(key, d) + "\n" + key + " 9 9 9 x\n");
  expect(lookup(dir + "/two.txt", key, &got) && same(got, d), "last valid line wins");
  // defaults are untouched when nothing is found
  Choice def;
  Choice untouched = def;
  expect(!lookup(dir + "/junk.txt", key, &untouched) && same(untouched, def), "defaults kept");

  if (failures) return 1;
  std::printf("ok\n");
  return 0;
}
