// Work schedule of the batched path: plain host C++ (no HIP), so that the
// scheduling rules can be compiled and checked on a machine without a GPU.
//
// Every transform f is cut into items: row items (runs of consecutive row
// tiles, the row FFT of length N), column items (runs of column tiles, the
// column FFT of length M / m1), one whole-grid item for a small grid done by
// one workgroup, or one copy item for a 1 x 1 grid. Transforms are dealt to
// `nq` queues (one per XCD), largest first, each to the queue with the fewest
// points so far, so that all items of a transform share one XCD's L2. In every
// queue all row items of a transform precede all of its column items; the
// persistent kernel relies on this for its waits (a column item waits for its
// transform's row items, which were all popped earlier from the same queue).
// Consecutive items of a queue form groups of at least `group_kib` KiB of
// data; a workgroup pops one group at a time.
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

namespace fft2d {
namespace sched {

enum ItemKind : uint32_t { kRowItem = 0, kColItem = 1, kCopyItem = 2, kGridItem = 3 };

constexpr int kMaxQueues = 8;
constexpr int kMaxRun = 0xffff;  // tiles per item (16 bits of Item::y)

// One transform as the scheduler sees it.
struct Shape {
  int32_t rows = 1, cols = 1;  // M, N
  int32_t m1 = 1;              // split factor (1: plain); column vectors are m1 * N columns of M / m1 points
  int32_t grid = 0;            // 1: one whole-grid item
  int32_t nrow = 0, ncol = 0;  // row tiles, column tiles
  int32_t row_c = 1, col_c = 1;  // vectors per row tile, per column tile
};

// One item: x = transform << 2 | kind, y = first tile | tile count << 16.
// Same layout as the kernel's uint2.
struct Item {
  uint32_t x, y;
};
static_assert(sizeof(Item) == 8, "an item is two 32-bit words");

inline uint32_t item_fft(const Item& it) { return it.x >> 2; }
inline uint32_t item_kind(const Item& it) { return it.x & 3u; }
inline uint32_t item_first(const Item& it) { return it.y & 0xffffu; }
inline uint32_t item_count(const Item& it) { return it.y >> 16; }

struct Schedule {
  std::vector<Item> items;
  std::vector<uint32_t> groups;  // item index where each group starts, plus the end
  int qbeg[kMaxQueues + 1] = {};  // queue x owns groups [qbeg[x], qbeg[x + 1])
};

// Points one item moves (its data size / 8 bytes): tiles t0 .. t0 + cnt - 1.
inline int64_t item_points(const Shape& s, uint32_t kind, int64_t t0, int64_t cnt) {
  const int64_t M = s.rows, N = s.cols, m1 = s.m1;
  if (kind == kCopyItem) return 1;
  if (kind == kGridItem) return M * N;
  if (kind == kRowItem) return std::min<int64_t>(s.row_c * cnt, M - t0 * s.row_c) * N;
  return std::min<int64_t>(s.col_c * cnt, m1 * N - t0 * s.col_c) * (M / m1);
}

// order 0 lists every row item of a queue and then every column item
// (largest transforms first); order 1 works in chunks of about 16 MiB per
// queue: a chunk's row items, then the previous chunk's column items (which
// then mostly read data still in the MALL).
inline Schedule build_schedule(const std::vector<Shape>& f, int nq, int order, int group_kib) {
  nq = std::max(1, std::min(nq, kMaxQueues));
  const int64_t count = (int64_t)f.size();
  std::vector<int> idx((size_t)count);
  for (int64_t i = 0; i < count; ++i) idx[(size_t)i] = (int)i;
  auto pts = [&](int i) { return (int64_t)f[(size_t)i].rows * f[(size_t)i].cols; };
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return pts(a) > pts(b); });
  std::vector<std::vector<int>> q((size_t)nq);
  std::vector<int64_t> load((size_t)nq, 0);
  for (int i : idx) {
    const size_t x = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
    q[x].push_back(i);
    load[x] += pts(i);
  }
  Schedule sc;
  const int64_t target = (int64_t)group_kib * 1024 / 8;
  // runs of tiles: about `target` points each (at least one tile)
  auto runs = [&](int i, uint32_t kind, int ntiles, std::vector<Item>& out) {
    const int64_t per_tile = std::max<int64_t>(1, item_points(f[(size_t)i], kind, 0, 1));
    const int run = (int)std::max<int64_t>(1, std::min<int64_t>(target / per_tile, kMaxRun));
    for (int t = 0; t < ntiles; t += run)
      out.push_back(Item{(uint32_t)i << 2 | kind, (uint32_t)t | (uint32_t)std::min(run, ntiles - t) << 16});
  };
  auto rows_of = [&](int i, std::vector<Item>& out) {
    const Shape& s = f[(size_t)i];
    if (s.rows == 1 && s.cols == 1) {
      out.push_back(Item{(uint32_t)i << 2 | kCopyItem, 1u << 16});
    } else if (s.grid) {
      out.push_back(Item{(uint32_t)i << 2 | kGridItem, 1u << 16});
    } else {
      runs(i, kRowItem, s.nrow, out);
    }
  };
  auto cols_of = [&](int i, std::vector<Item>& out) { runs(i, kColItem, f[(size_t)i].ncol, out); };
  for (int x = 0; x < nq; ++x) {
    std::vector<Item> items;
    const std::vector<int>& qx = q[(size_t)x];
    if (order == 0) {
      for (int i : qx) rows_of(i, items);
      for (int i : qx) cols_of(i, items);
    } else {
      const int64_t chunk_points = (int64_t(16) << 20) / 8;
      std::vector<int> prev, cur;
      int64_t acc = 0;
      for (size_t k = 0; k < qx.size(); ++k) {
        rows_of(qx[k], items);
        cur.push_back(qx[k]);
        acc += pts(qx[k]);
        if (acc >= chunk_points || k + 1 == qx.size()) {
          for (int g : prev) cols_of(g, items);
          prev.swap(cur);
          cur.clear();
          acc = 0;
        }
      }
      for (int g : prev) cols_of(g, items);
    }
    sc.qbeg[x] = (int)sc.groups.size();
    int64_t acc = target;  // open a new group at the first item
    for (const Item& it : items) {
      if (acc >= target) {
        sc.groups.push_back((uint32_t)sc.items.size());
        acc = 0;
      }
      acc += item_points(f[item_fft(it)], item_kind(it), item_first(it), item_count(it));
      sc.items.push_back(it);
    }
  }
  for (int x = nq; x <= kMaxQueues; ++x) sc.qbeg[x] = (int)sc.groups.size();
  sc.groups.push_back((uint32_t)sc.items.size());
  return sc;
}

}  // namespace sched
}  // namespace fft2d
