// CPU check of the batched path's work schedule (paper_2506_15437_amd/csrc/
// fft_schedule.hpp, and its guided regrouping in fft_batched_guided.hpp),
// built with g++ and run by tests/test_host.py.
//
// For many random shape sets and every queue count, item order, group size and
// worker count (0: fixed groups) the library uses, it checks the properties
// the persistent kernel relies on:
//   * every row tile, column tile, whole-grid item and copy item of every
//     transform appears exactly once;
//   * all items of a transform sit in one queue, and there every row item of
//     the transform comes before every column item of it (so the lowest
//     unfinished item of a queue never waits);
//   * groups are non-empty, cover the item table in order, and never straddle
//     two queues; queue ranges are contiguous and in order;
//   * every item holds 1 ... 65535 tiles.
// Prints "ok <cases>" and exits 0, or prints the first violation and exits 1.
#include "../../paper_2506_15437_amd/csrc/fft_schedule.hpp"
#include "../../paper_2506_15437_amd/csrc/fft_batched_guided.hpp"

#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

using namespace fft2d::sched;

namespace {

int fail(const char* what, long a, long b) {
  std::printf("FAIL %s (%ld, %ld)\n", what, a, b);
  return 1;
}

int check(const std::vector<Shape>& f, int nq, int order, int gk, int workers) {
  const Schedule fixed = build_schedule(f, nq, order, gk);
  const Schedule sc = workers > 0 ? guided(fixed, f, nq, workers, (int64_t)gk * 1024 / 8) : fixed;
  if (workers > 0) {
    // regrouping keeps the order of the tiles within each queue and never makes more groups or items
    if (sc.groups.size() > fixed.groups.size()) return fail("guided groups", (long)sc.groups.size(), 0);
    if (sc.items.size() > fixed.items.size()) return fail("guided items", (long)sc.items.size(), 0);
    for (int x = 0; x <= kMaxQueues; ++x)
      if ((sc.qbeg[x] == sc.qbeg[kMaxQueues]) != (fixed.qbeg[x] == fixed.qbeg[kMaxQueues]))
        return fail("guided queue emptiness", x, sc.qbeg[x]);
  }
  const int ng = (int)sc.groups.size() - 1;
  const int ni = (int)sc.items.size();
  if (ng < 0) return fail("no group end", ng, 0);
  if (sc.groups.back() != (uint32_t)ni) return fail("groups end", sc.groups.back(), ni);
  if (ng > 0 && sc.groups[0] != 0) return fail("first group start", sc.groups[0], 0);
  for (int g = 0; g < ng; ++g)
    if (sc.groups[g] >= sc.groups[g + 1]) return fail("empty group", g, sc.groups[g]);
  const int eq = std::max(1, std::min(nq, kMaxQueues));
  if (sc.qbeg[0] != 0) return fail("first queue start", sc.qbeg[0], 0);
  for (int x = 0; x < kMaxQueues; ++x)
    if (sc.qbeg[x] > sc.qbeg[x + 1]) return fail("queue order", x, sc.qbeg[x]);
  for (int x = eq; x <= kMaxQueues; ++x)
    if (sc.qbeg[x] != ng) return fail("unused queue not empty", x, sc.qbeg[x]);
  // queue of every item, from the group ranges
  std::vector<int> qof((size_t)ni, -1);
  for (int x = 0; x < eq; ++x)
    for (int g = sc.qbeg[x]; g < sc.qbeg[x + 1]; ++g)
      for (uint32_t i = sc.groups[g]; i < sc.groups[g + 1]; ++i) qof[i] = x;
  for (int i = 0; i < ni; ++i)
    if (qof[(size_t)i] < 0) return fail("item outside every queue", i, 0);
  const size_t nf = f.size();
  std::vector<std::vector<int>> row_seen(nf), col_seen(nf);
  std::vector<int> whole_seen(nf, 0), queue(nf, -1), last_row(nf, -1), first_col(nf, 1 << 30);
  for (size_t k = 0; k < nf; ++k) {
    row_seen[k].assign((size_t)f[k].nrow, 0);
    col_seen[k].assign((size_t)f[k].ncol, 0);
  }
  for (int i = 0; i < ni; ++i) {
    const Item& it = sc.items[(size_t)i];
    const uint32_t k = item_fft(it), kind = item_kind(it), t0 = item_first(it), cnt = item_count(it);
    if (k >= nf) return fail("transform index", k, (long)nf);
    if (cnt < 1 || cnt > (uint32_t)kMaxRun) return fail("tile count", i, cnt);
    if (queue[k] < 0) queue[k] = qof[(size_t)i];
    if (queue[k] != qof[(size_t)i]) return fail("transform in two queues", k, i);
    const Shape& s = f[k];
    if (kind == kCopyItem || kind == kGridItem) {
      const bool ok = kind == kCopyItem ? (s.rows == 1 && s.cols == 1) : (s.grid && !(s.rows == 1 && s.cols == 1));
      if (!ok || t0 != 0 || cnt != 1) return fail("whole item of wrong transform", k, kind);
      ++whole_seen[k];
      last_row[k] = std::max(last_row[k], i);
    } else if (kind == kRowItem) {
      if (s.grid || (s.rows == 1 && s.cols == 1)) return fail("row item of a whole transform", k, i);
      for (uint32_t t = t0; t < t0 + cnt; ++t) {
        if (t >= (uint32_t)s.nrow) return fail("row tile out of range", k, t);
        ++row_seen[k][t];
      }
      last_row[k] = std::max(last_row[k], i);
    } else {
      if (s.grid) return fail("column item of a whole-grid transform", k, i);
      for (uint32_t t = t0; t < t0 + cnt; ++t) {
        if (t >= (uint32_t)s.ncol) return fail("column tile out of range", k, t);
        ++col_seen[k][t];
      }
      first_col[k] = std::min(first_col[k], i);
    }
  }
  for (size_t k = 0; k < nf; ++k) {
    const Shape& s = f[k];
    const bool whole = s.grid || (s.rows == 1 && s.cols == 1);
    if (whole_seen[k] != (whole ? 1 : 0)) return fail("whole items of a transform", (long)k, whole_seen[k]);
    for (size_t t = 0; t < row_seen[k].size(); ++t)
      if (row_seen[k][t] != (whole ? 0 : 1)) return fail("row tile count", (long)k, (long)t);
    for (size_t t = 0; t < col_seen[k].size(); ++t)
      if (col_seen[k][t] != (s.grid ? 0 : 1)) return fail("column tile count", (long)k, (long)t);
    if (first_col[k] < (1 << 30) && last_row[k] >= first_col[k])
      return fail("a column item before a row item of its transform", (long)k, first_col[k]);
  }
  return 0;
}

// A transform of 2^a x 2^b with tile sizes like the library's (C vectors of
// a tile, a power of two; split transforms with m1 rows per row tile).
Shape random_shape(std::mt19937_64& rng) {
  Shape s;
  const int a = (int)(rng() % 15), b = (int)(rng() % 15);
  s.rows = 1 << a;
  s.cols = 1 << b;
  s.m1 = 1;
  if (s.rows >= 1024 && s.cols >= 512 && s.cols <= 8192 && rng() % 2) s.m1 = std::max(2, 16384 / s.cols / 2);
  if (s.rows % s.m1 != 0 || s.rows / s.m1 < 2) s.m1 = 1;
  s.grid = (s.rows * (int64_t)s.cols <= 16384 && s.rows >= 64 && s.cols >= 64 && rng() % 2) ? 1 : 0;
  s.row_c = s.m1 > 1 ? s.m1 : std::max(1, 8192 / std::max(1, s.cols));
  s.col_c = std::max(1, 8192 / std::max(1, s.rows / s.m1));
  s.nrow = (s.grid || s.cols == 1) ? 0 : (s.m1 > 1 ? s.rows / s.m1 : (s.rows + s.row_c - 1) / s.row_c);
  s.ncol = (s.grid || s.rows == 1) ? 0 : (int)(((int64_t)s.m1 * s.cols + s.col_c - 1) / s.col_c);
  return s;
}

}  // namespace

int main(int argc, char** argv) {
  const int sets = argc > 1 ? std::atoi(argv[1]) : 200;
  std::mt19937_64 rng(12345);
  long cases = 0;
  for (int n = 0; n < sets; ++n) {
    const int count = 1 + (int)(rng() % (n % 4 == 0 ? 600 : 40));
    std::vector<Shape> f((size_t)count);
    for (Shape& s : f) s = random_shape(rng);
    if (n == 0) f.assign(3, Shape{});  // three 1 x 1 transforms
    for (int nq = 1; nq <= 9; ++nq)
      for (int order = 0; order < 2; ++order)
        for (int gk : {64, 256, 1024})
          for (int workers : {0, 1, 32, 96}) {
            if (check(f, nq, order, gk, workers)) {
              std::printf("set %d count %d nq %d order %d group_kib %d workers %d\n", n, count, nq, order, gk,
                          workers);
              return 1;
            }
            ++cases;
          }
  }
  std::printf("ok %ld\n", cases);
  return 0;
}
