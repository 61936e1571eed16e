// Guided grouping of the batched path's work schedule: plain host C++ (no
// HIP), checked on the CPU with the scheduler itself.
//
// A workgroup of the persistent kernel pops one group at a time and calls one
// tile function per item. Those functions hold up to 120 VGPRs, so each call
// saves and restores the callee-saved registers it uses (up to 57 per lane,
// through scratch memory): per call a fixed cost in memory traffic. Groups of
// a fixed small size keep the end of a queue balanced but make many calls.
// Guided grouping (large groups first, smaller ones as the queue drains, as
// in guided self-scheduling) keeps the balanced end and makes fewer calls:
// a group holds at least max(min_points, r / (2 * workers)) points, r being
// the points of the queue from that group on, and consecutive items of one
// transform and kind whose tiles follow each other are merged into one item.
// Order within a queue is unchanged, so every property the kernel relies on
// (each tile once, one queue per transform, its row items before its column
// items) carries over.
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

#include "fft_schedule.hpp"

namespace fft2d {
namespace sched {

inline Schedule guided(const Schedule& in, const std::vector<Shape>& f, int nq, int workers, int64_t min_points) {
  nq = std::max(1, std::min(nq, kMaxQueues));
  const int64_t div = 2 * (int64_t)std::max(1, workers);
  min_points = std::max<int64_t>(1, min_points);
  auto points = [&](const Item& it) {
    return item_points(f[item_fft(it)], item_kind(it), item_first(it), item_count(it));
  };
  Schedule out;
  for (int x = 0; x < nq; ++x) {
    const uint32_t i0 = in.groups[(size_t)in.qbeg[x]];
    const uint32_t i1 = in.groups[(size_t)in.qbeg[x + 1]];
    int64_t remaining = 0;
    for (uint32_t i = i0; i < i1; ++i) remaining += points(in.items[i]);
    out.qbeg[x] = (int)out.groups.size();
    uint32_t i = i0;
    while (i < i1) {
      const int64_t target = std::max(min_points, remaining / div);
      const size_t first = out.items.size();
      out.groups.push_back((uint32_t)first);
      int64_t acc = 0;
      while (i < i1 && acc < target) {
        const Item& it = in.items[i];
        const int64_t p = points(it);
        const uint32_t kind = item_kind(it);
        bool merged = false;
        if (out.items.size() > first && (kind == kRowItem || kind == kColItem)) {
          Item& last = out.items.back();
          const uint32_t cnt = item_count(last) + item_count(it);
          if (last.x == it.x && item_first(last) + item_count(last) == item_first(it) && cnt <= (uint32_t)kMaxRun) {
            last.y = item_first(last) | cnt << 16;
            merged = true;
          }
        }
        if (!merged) out.items.push_back(it);
        acc += p;
        remaining -= p;
        ++i;
      }
    }
  }
  for (int x = nq; x <= kMaxQueues; ++x) out.qbeg[x] = (int)out.groups.size();
  out.groups.push_back((uint32_t)out.items.size());
  return out;
}

}  // namespace sched
}  // namespace fft2d
