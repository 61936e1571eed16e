// Batched path: many 2D FFTs of different power-of-two shapes in ONE
// persistent kernel launch, replayed from a HIP graph.
//
// Work decomposition. Every transform f (rows M, cols N) becomes row items
// (tiles of C_row(N) rows; the row FFT of length N) and column items (tiles of
// C_col(M) columns; the column FFT of length M, in place on the output); an
// item is a run of consecutive tiles of one transform and kind. Tall grids
// are split as in the plain path: their row items are tiles of the row pass
// with an M1-point combine (into a plan work buffer) and their column items
// run columns of M / M1 points from it to the output. Small grids (at most 16384
// points, see batched_grid_item) are one whole-grid item each. A 1 x 1
// transform is one copy item.
//
// Queues. Each transform is assigned to one XCD (balanced by its point
// count), and each XCD has its own queue of item groups (consecutive items of
// at least a target size). A workgroup reads the XCD it runs on from the
// XCC_ID hardware register and only pops groups of that XCD's queue, so all
// items of one transform run on one XCD and share its L2. In every queue the
// row items of a transform precede its column items.
//
// Dependencies. A column item of f waits until f's row-item counter reaches
// its row-item count. Every row item of f sits earlier in the same queue and
// was popped by a running workgroup; row items never wait; a workgroup works
// through its group in order. So the lowest unfinished item can always
// proceed and every wait ends, whatever the number of resident workgroups.
// Publication stays inside the XCD: every wave waits until its stores are
// acknowledged (they are then in the XCD's L2), the workgroup synchronises,
// one lane increments the counter; the consumer's loads are device-scope
// loads, which the CU's L1 does not serve. No L2 writeback or invalidation
// is needed. The plan checks at creation, with a probe launch of the same
// grid, that the XCC_ID values are 0 .. nq-1 and that every queue has
// workgroups; if not, it falls back to one queue with agent-scope release /
// acquire around every counter (correct across XCDs, slower).
//
// Direction. The kernel always runs the forward sign; the inverse is
// conj(F(conj(x))) / (M N): row items conjugate on load, column items
// conjugate and scale on store (exact in floating point).
#include "fft_batched.h"
#include "fft_batched_guided.hpp"
#include "fft_pass.hpp"
#include "fft_schedule.hpp"
#include "fft_tune_cache.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include <sys/stat.h>

namespace fft2d {
namespace {

using namespace dev;

constexpr int kThreads = 512;
// id = variant * 48 + mode * 16 + log2(L); mode 0 = row, 1 = column, 2 = row
// with combine; variant 0 or 1 (a second radix schedule / tile shape for rows
// and columns of 32 ... 16384 points, chosen per length by the autotuner).
constexpr int kNumCfg = 96;
constexpr int kVariantStride = 48;
constexpr int kMinVariantLog2 = 5;  // lengths below 32 have one configuration

// Row configurations (512 threads each).
using BR2 = Cfg<2, 2, 512, 1, false, 2>;
using BR4 = Cfg<4, 4, 512, 1, false, 4>;
using BR8 = Cfg<8, 8, 512, 1, false, 8>;
using BR16 = Cfg<16, 16, 512, 1, false, 16>;
using BR32 = Cfg<32, 8, 128, 1, false, 8, 4>;
using BR64 = Cfg<64, 8, 64, 1, false, 8, 8>;
using BR128 = Cfg<128, 16, 64, 1, false, 16, 8>;
using BR256 = Cfg<256, 16, 32, 1, false, 16, 16>;
using BR512 = Cfg<512, 16, 16, 1, false, 16, 16, 2>;
using BR1024 = Cfg<1024, 16, 8, 1, false, 16, 16, 4>;
using BR2048 = Cfg<2048, 16, 4, 1, false, 16, 16, 8>;
using BR4096 = Cfg<4096, 16, 2, 1, false, 16, 16, 16>;
using BR8192 = Cfg<8192, 16, 1, 1, false, 16, 16, 16, 2>;
using BR16384 = Cfg<16384, 32, 1, 2, false, 16, 16, 16, 4>;
// Column configurations (512 threads each).
using BC2 = Cfg<2, 2, 512, 1, true, 2>;
using BC4 = Cfg<4, 4, 512, 1, true, 4>;
using BC8 = Cfg<8, 8, 512, 1, true, 8>;
using BC16 = Cfg<16, 16, 512, 1, true, 16>;
using BC32 = Cfg<32, 8, 128, 1, true, 8, 4>;
using BC64 = Cfg<64, 8, 64, 1, true, 8, 8>;
using BC128 = Cfg<128, 16, 64, 1, true, 16, 8>;
using BC256 = Cfg<256, 16, 32, 1, true, 16, 16>;
using BC512 = Cfg<512, 16, 16, 1, true, 16, 16, 2>;
using BC1024 = Cfg<1024, 32, 16, 2, true, 32, 32>;
using BC2048 = Cfg<2048, 32, 8, 2, true, 16, 16, 8>;
using BC4096 = Cfg<4096, 32, 4, 2, true, 16, 16, 16>;
using BC8192 = Cfg<8192, 32, 2, 2, true, 16, 16, 32>;
using BC16384 = Cfg<16384, 32, 1, 2, true, 16, 16, 16, 4>;
// Row-with-combine configurations of split transforms (512 threads each): M1
// rows of length L per tile, M1 = C.
using BRC512 = Cfg<512, 16, 16, 1, false, 16, 16, 2>;
// The last stage of the row FFT runs across the M1 rows (rowx_tile): its
// radix times M1 is the points per thread, and the combine needs no exchange
// of its own.
using BRC1024 = Cfg<1024, 32, 16, 2, false, 32, 16, 2>;
using BRC2048 = Cfg<2048, 32, 8, 2, false, 32, 16, 4>;
using BRC4096 = Cfg<4096, 32, 4, 2, false, 32, 16, 8>;
using BRC8192 = Cfg<8192, 32, 2, 2, false, 32, 16, 16>;

// Variant-1 configurations (512 threads each): the other points-per-thread
// count, hence the other tile size (4096 / 8192 / 16384 points) and, for
// columns, the other row-segment width, or another radix order.
using BR32v = Cfg<32, 16, 256, 1, false, 16, 2>;
using BR64v = Cfg<64, 16, 128, 1, false, 16, 4>;
using BR128v = Cfg<128, 8, 32, 1, false, 8, 8, 2>;
using BR256v = Cfg<256, 32, 64, 2, false, 8, 32>;
using BR512v = Cfg<512, 32, 32, 2, false, 16, 32>;
using BR1024v = Cfg<1024, 32, 16, 2, false, 16, 16, 4>;
using BR2048v = Cfg<2048, 32, 8, 2, false, 16, 16, 8>;
using BR4096v = Cfg<4096, 32, 4, 2, false, 16, 16, 16>;
using BR8192v = Cfg<8192, 32, 2, 2, false, 16, 16, 32>;
using BR16384v = Cfg<16384, 32, 1, 2, false, 16, 16, 4, 16>;
using BC32v = Cfg<32, 16, 256, 1, true, 16, 2>;
using BC64v = Cfg<64, 16, 128, 1, true, 16, 4>;
using BC128v = Cfg<128, 8, 32, 1, true, 8, 8, 2>;
using BC256v = Cfg<256, 32, 64, 2, true, 8, 32>;
using BC512v = Cfg<512, 32, 32, 2, true, 16, 32>;
using BC1024v = Cfg<1024, 16, 8, 1, true, 16, 16, 4>;
using BC2048v = Cfg<2048, 16, 4, 1, true, 16, 16, 8>;
using BC4096v = Cfg<4096, 16, 2, 1, true, 16, 16, 16>;
using BC8192v = Cfg<8192, 16, 1, 1, true, 16, 16, 16, 2>;
using BC16384v = Cfg<16384, 32, 1, 2, true, 16, 16, 4, 16>;

template <class... Ks>
constexpr int max_lds() {
  int m = 1;
  ((m = Ks::LDS_ELEMS > m ? Ks::LDS_ELEMS : m), ...);
  return m;
}
constexpr int kLdsElems = max_lds<BR2, BR4, BR8, BR16, BR32, BR64, BR128, BR256, BR512, BR1024, BR2048, BR4096,
                                  BR8192, BR16384, BC2, BC4, BC8, BC16, BC32, BC64, BC128, BC256, BC512, BC1024,
                                  BC2048, BC4096, BC8192, BC16384, BRC512, BRC1024, BRC2048, BRC4096,
                                  BRC8192, BR32v, BR64v, BR128v, BR256v, BR512v, BR1024v, BR2048v, BR4096v,
                                  BR8192v, BR16384v, BC32v, BC64v, BC128v, BC256v, BC512v, BC1024v, BC2048v,
                                  BC4096v, BC8192v, BC16384v>();
static_assert(kLdsElems * 8 <= 80 * 1024, "two batched workgroups must fit one CU's LDS");

struct BatchDesc {
  const float2* in;
  float2* out;
  float2* work;  // split transforms: the grid between the row pass with combine and the column pass
  int32_t rows, cols;
  int32_t row_cfg, col_cfg;
  int32_t nrow_items;
  int32_t m1;       // 1: plain; > 1: split transform, rows = m1 * m2, row items combine m1 rows
  int32_t twc_off;  // split transforms: offset of W_rows^j, j < rows, in the twiddle buffer
  int32_t pad;
};

using sched::kColItem;
using sched::kCopyItem;
using sched::kGridItem;
using sched::kMaxQueues;
using sched::kRowItem;

constexpr int kQueueStride = 32;                            // queue heads 128 bytes apart
constexpr int kFinishSlot = kMaxQueues * kQueueStride;      // workgroups that have left the loop
constexpr int kCounterBase = (kMaxQueues + 1) * kQueueStride;  // first per-transform counter
constexpr int kXccIdReg = (3 << 11) | 20;            // hwreg(HW_REG_XCC_ID, 0, 4)

struct BatchArgs {
  const BatchDesc* desc;
  const uint2* items;       // x = fft << 2 | kind, y = first tile | tile count << 16
  const uint32_t* groups;   // group g covers items [groups[g], groups[g + 1])
  int qbeg[kMaxQueues + 1];  // queue x owns groups [qbeg[x], qbeg[x + 1])
  int nq;                   // number of queues (XCDs)
  unsigned* counters;       // [x * kQueueStride] head of queue x, [kFinishSlot] workgroups done,
                            // [kCounterBase + f] finished row items of f
  unsigned* err_host;       // pinned host word: 1 when a bounded wait gave up, 2 when a queue was left undrained
  int drain_slack;          // added to every queue's group count in the drain check (0; > 0 only in tests)
  const float2* tw;         // concatenated twiddle tables, cfg id -> offset in tw_off
  int tw_off[kNumCfg];
  int tw_cnt[kNumCfg];
  int conj;                 // 1: inverse transform
  int n_fft;
  int fenced;               // 1: agent-scope release / acquire (queues not tied to XCDs)
  int max_spins;            // bound of a column item's wait in polls; < 0: give up every wait (tests)
};

constexpr int kMaxSpins = 1 << 24;  // about a second of polling

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniform(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
template <class T>
__device__ __forceinline__ T* uniform(T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return reinterpret_cast<T*>((uint64_t)hi << 32 | lo);
}

// One configuration's tile as its own (flattened) function, so that every
// register array of the pass stays in registers inside the large dispatch.
// Its arguments are plain scalars (passed in registers): a structure passed by
// reference would make every lane write it to and read it from scratch memory.
// Column tiles read the row items' results, so their loads are device-scope.
// A call runs the tiles t0 .. t0 + cnt - 1 of one grid, so the cost of the
// call (saving the registers the callee must preserve) is paid once per run.
// flags: bit 0 conjugates the input, bit 1 the output.
template <class K>
__device__ __noinline__ __attribute__((flatten)) void tile(const float2* in, float2* out, const float2* tw, int tw_count,
                                                           int rows, int cols, int m1, int t0, int cnt, int flags,
                                                           float scale, float2* lds) {
  static_assert(K::valid() && K::THREADS == kThreads, "batched configurations use 512 threads");
  // The arguments arrive in vector registers; they are uniform, so move them
  // to scalar registers (keeps the address arithmetic scalar).
  rows = uniform(rows);
  cols = uniform(cols);
  m1 = uniform(m1);
  PassArgs pa{};
  pa.in = uniform(in);
  pa.out = uniform(out);
  pa.tw = uniform(tw);
  pa.tw_count = uniform(tw_count);
  pa.total = (int64_t)rows * cols;
  // column tiles of a split transform: length rows / m1, m1 row blocks of cols vectors
  pa.nvec = K::COL ? (int64_t)m1 * cols : rows;
  pa.ncols = cols;
  pa.m1 = m1;
  flags = uniform(flags);
  TileIO io;
  io.conj_in = (flags & 1) != 0;
  io.conj_out = (flags & 2) != 0;
  io.scale = uniform(scale);
  t0 = uniform(t0);
  cnt = uniform(cnt);
  for (int i = 0; i < cnt; ++i) {
    if (i > 0) __syncthreads();  // the previous tile's LDS reads are done
    fft_tile<K, -1, K::COL ? kAuxDevice : 0>(pa, t0 + i, lds, io);
  }
}

// Tiles t0 .. t0 + cnt - 1 (tile = m2 index) of the row pass with combine of a
// split transform: in -> work, conjugating the input for the inverse.
template <class K, bool XROW>
__device__ __noinline__ __attribute__((flatten)) void ctile(const float2* in, float2* work, const float2* tw,
                                                            int tw_count, const float2* twc, int rows, int cols,
                                                            int t0, int cnt, int flags, float2* lds) {
  static_assert(K::valid() && K::THREADS == kThreads && !K::COL, "batched configurations use 512 threads");
  rows = uniform(rows);
  cols = uniform(cols);
  PassArgs pa{};
  pa.in = uniform(in);
  pa.out = uniform(work);
  pa.tw = uniform(tw);
  pa.tw_count = uniform(tw_count);
  pa.twc = uniform(twc);
  pa.total = (int64_t)rows * cols;
  pa.nvec = rows;
  pa.ncols = cols;
  pa.m1 = K::C;
  pa.m2 = rows / K::C;
  flags = uniform(flags);
  TileIO io;
  io.conj_in = (flags & 1) != 0;
  t0 = uniform(t0);
  cnt = uniform(cnt);
  for (int i = 0; i < cnt; ++i) {
    if (i > 0) __syncthreads();  // the previous tile's LDS reads are done
    if constexpr (XROW) rowx_tile<K, -1, kAuxNontemporal>(pa, t0 + i, lds, io);
    else rowc_tile<K, -1, kAuxNontemporal>(pa, t0 + i, lds, io);
  }
}

__device__ __forceinline__ void run_ctile(int cfg, const float2* in, float2* work, const float2* tw, int tw_count,
                                          const float2* twc, int rows, int cols, int t0, int cnt, int flags,
                                          float2* lds) {
  switch (cfg) {
    case 41: ctile<BRC512, false>(in, work, tw, tw_count, twc, rows, cols, t0, cnt, flags, lds); break;
    case 42: ctile<BRC1024, true>(in, work, tw, tw_count, twc, rows, cols, t0, cnt, flags, lds); break;
    case 43: ctile<BRC2048, true>(in, work, tw, tw_count, twc, rows, cols, t0, cnt, flags, lds); break;
    case 44: ctile<BRC4096, true>(in, work, tw, tw_count, twc, rows, cols, t0, cnt, flags, lds); break;
    case 45: ctile<BRC8192, true>(in, work, tw, tw_count, twc, rows, cols, t0, cnt, flags, lds); break;
    default: break;
  }
}

// Whole-grid item: a small M x N grid in one workgroup and one pass through
// HBM. Row tile u (configuration KR, C_r rows) is loaded from global memory
// and transformed in registers; then it crosses LDS in row-major order and
// every column-tile thread (configuration KC) takes the points of its columns
// that lie in those rows, so the grid moves through LDS one row tile at a
// time; finally the column tiles are transformed and stored. The LDS holding a
// row tile is the passes' exchange area, used between barriers only.
template <class KR, class KC, int M, int N>
__device__ __noinline__ __attribute__((flatten)) void grid_item(const float2* in, float2* out, const float2* twr,
                                                                int twr_count, const float2* twc, int twc_count,
                                                                int flags, float scale, float2* lds) {
  static_assert(KR::L == N && KC::L == M, "row and column configurations of the grid");
  static_assert(KR::THREADS == kThreads && KC::THREADS == kThreads, "batched configurations use 512 threads");
  static_assert(grid_lds_elems<KR, KC>() <= kLdsElems, "the grid's row tile fits the LDS");
  const Buf src(uniform(in), (uint32_t)(M * N) * 8u);
  const Buf dst(uniform(out), (uint32_t)(M * N) * 8u);
  const Buf tr(uniform(twr), (uint32_t)uniform(twr_count) * 8u);
  const Buf tc(uniform(twc), (uint32_t)uniform(twc_count) * 8u);
  flags = uniform(flags);
  TileIO io;
  io.conj_in = (flags & 1) != 0;
  io.conj_out = (flags & 2) != 0;
  io.scale = uniform(scale);
  grid_tile<KR, KC, -1>(src, dst, tr, tc, io, lds);
}

// The grids handled as whole-grid items (see batched_grid_item on the host).
__device__ __forceinline__ void run_grid(int rows, int cols, const float2* in, float2* out, const float2* twr,
                                         int twr_count, const float2* twc, int twc_count, int flags, float scale,
                                         float2* lds) {
#define FFT2D_GRID(R, C, KR, KC) \
  if (rows == R && cols == C) return grid_item<KR, KC, R, C>(in, out, twr, twr_count, twc, twc_count, flags, scale, lds)
  FFT2D_GRID(64, 64, BR64, BC64);
  FFT2D_GRID(64, 128, BR128, BC64);
  FFT2D_GRID(128, 64, BR64, BC128);
  FFT2D_GRID(128, 128, BR128, BC128);
  FFT2D_GRID(64, 256, BR256, BC64);
  FFT2D_GRID(256, 64, BR64, BC256);
#undef FFT2D_GRID
}

#define FFT2D_TILE_ARGS in, out, tw, tw_count, rows, cols, m1, t0, cnt, flags, scale, lds
__device__ __forceinline__ void run_tile(int cfg, const float2* in, float2* out, const float2* tw, int tw_count,
                                         int rows, int cols, int m1, int t0, int cnt, int flags, float scale,
                                         float2* lds) {
  switch (cfg) {
    case 1: tile<BR2>(FFT2D_TILE_ARGS); break;
    case 2: tile<BR4>(FFT2D_TILE_ARGS); break;
    case 3: tile<BR8>(FFT2D_TILE_ARGS); break;
    case 4: tile<BR16>(FFT2D_TILE_ARGS); break;
    case 5: tile<BR32>(FFT2D_TILE_ARGS); break;
    case 6: tile<BR64>(FFT2D_TILE_ARGS); break;
    case 7: tile<BR128>(FFT2D_TILE_ARGS); break;
    case 8: tile<BR256>(FFT2D_TILE_ARGS); break;
    case 9: tile<BR512>(FFT2D_TILE_ARGS); break;
    case 10: tile<BR1024>(FFT2D_TILE_ARGS); break;
    case 11: tile<BR2048>(FFT2D_TILE_ARGS); break;
    case 12: tile<BR4096>(FFT2D_TILE_ARGS); break;
    case 13: tile<BR8192>(FFT2D_TILE_ARGS); break;
    case 14: tile<BR16384>(FFT2D_TILE_ARGS); break;
    case 17: tile<BC2>(FFT2D_TILE_ARGS); break;
    case 18: tile<BC4>(FFT2D_TILE_ARGS); break;
    case 19: tile<BC8>(FFT2D_TILE_ARGS); break;
    case 20: tile<BC16>(FFT2D_TILE_ARGS); break;
    case 21: tile<BC32>(FFT2D_TILE_ARGS); break;
    case 22: tile<BC64>(FFT2D_TILE_ARGS); break;
    case 23: tile<BC128>(FFT2D_TILE_ARGS); break;
    case 24: tile<BC256>(FFT2D_TILE_ARGS); break;
    case 25: tile<BC512>(FFT2D_TILE_ARGS); break;
    case 26: tile<BC1024>(FFT2D_TILE_ARGS); break;
    case 27: tile<BC2048>(FFT2D_TILE_ARGS); break;
    case 28: tile<BC4096>(FFT2D_TILE_ARGS); break;
    case 29: tile<BC8192>(FFT2D_TILE_ARGS); break;
    case 30: tile<BC16384>(FFT2D_TILE_ARGS); break;
    case 53: tile<BR32v>(FFT2D_TILE_ARGS); break;
    case 54: tile<BR64v>(FFT2D_TILE_ARGS); break;
    case 55: tile<BR128v>(FFT2D_TILE_ARGS); break;
    case 56: tile<BR256v>(FFT2D_TILE_ARGS); break;
    case 57: tile<BR512v>(FFT2D_TILE_ARGS); break;
    case 58: tile<BR1024v>(FFT2D_TILE_ARGS); break;
    case 59: tile<BR2048v>(FFT2D_TILE_ARGS); break;
    case 60: tile<BR4096v>(FFT2D_TILE_ARGS); break;
    case 61: tile<BR8192v>(FFT2D_TILE_ARGS); break;
    case 62: tile<BR16384v>(FFT2D_TILE_ARGS); break;
    case 69: tile<BC32v>(FFT2D_TILE_ARGS); break;
    case 70: tile<BC64v>(FFT2D_TILE_ARGS); break;
    case 71: tile<BC128v>(FFT2D_TILE_ARGS); break;
    case 72: tile<BC256v>(FFT2D_TILE_ARGS); break;
    case 73: tile<BC512v>(FFT2D_TILE_ARGS); break;
    case 74: tile<BC1024v>(FFT2D_TILE_ARGS); break;
    case 75: tile<BC2048v>(FFT2D_TILE_ARGS); break;
    case 76: tile<BC4096v>(FFT2D_TILE_ARGS); break;
    case 77: tile<BC8192v>(FFT2D_TILE_ARGS); break;
    case 78: tile<BC16384v>(FFT2D_TILE_ARGS); break;
    default: break;
  }
}
#undef FFT2D_TILE_ARGS

__global__ void clear_counters(unsigned* c, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) c[i] = 0u;
}

// One word per workgroup: the XCC_ID it ran on (the plan's creation check).
__global__ void xcc_probe(unsigned* ids) {
  if (threadIdx.x == 0) ids[blockIdx.x] = (unsigned)__builtin_amdgcn_s_getreg(kXccIdReg);
}

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void batched_kernel(BatchArgs a) {
  __shared__ float2 lds[kLdsElems];
  __shared__ int s_group;
  __shared__ int s_flag;
  const int xq = (int)((unsigned)__builtin_amdgcn_s_getreg(kXccIdReg) % (unsigned)a.nq);
  unsigned* head = &a.counters[xq * kQueueStride];
  const int gend = a.qbeg[xq + 1];
  for (;;) {
    if (threadIdx.x == 0) s_group = (int)atomicAdd(head, 1u);
    __syncthreads();
    const int g = __builtin_amdgcn_readfirstlane(s_group) + a.qbeg[xq];
    __syncthreads();  // every lane has read s_group before lane 0 may overwrite it
    if (g >= gend) break;
    const int i_end = (int)a.groups[g + 1];
    for (int it = (int)a.groups[g]; it < i_end; ++it) {
      const uint2 item = a.items[it];
      const int f = (int)(item.x >> 2);
      const int kind = (int)(item.x & 3u);
      const int t0 = (int)(item.y & 0xffffu);  // first tile of the run
      const int cnt = (int)(item.y >> 16);     // tiles in the run
      const BatchDesc d = a.desc[f];
      unsigned* done = &a.counters[kCounterBase + f];
      const bool inv = a.conj != 0;
      const float s = inv ? 1.0f / ((float)d.rows * (float)d.cols) : 1.0f;
      if (kind == kCopyItem) {
        if (threadIdx.x == 0) {
          const float2 v = d.in[0];
          d.out[0] = make_float2(v.x * s, v.y * s);
        }
        continue;
      }
      if (kind == kGridItem) {
        // the inverse conjugates on load, then conjugates and scales on store
        run_grid(d.rows, d.cols, d.in, d.out, a.tw + a.tw_off[d.row_cfg], a.tw_cnt[d.row_cfg],
                 a.tw + a.tw_off[d.col_cfg], a.tw_cnt[d.col_cfg], inv ? 3 : 0, s, lds);
        __syncthreads();  // the LDS of this item is free before the next item starts
        continue;
      }
      if (kind == kRowItem) {
        // the inverse conjugates on load; a single-row grid also conjugates and scales on store
        const int flags = inv ? (d.rows == 1 ? 3 : 1) : 0;
        if (d.m1 > 1)
          run_ctile(d.row_cfg, d.in, d.work, a.tw + a.tw_off[d.row_cfg], a.tw_cnt[d.row_cfg], a.tw + d.twc_off,
                    d.rows, d.cols, t0, cnt, flags, lds);
        else
          run_tile(d.row_cfg, d.in, d.out, a.tw + a.tw_off[d.row_cfg], a.tw_cnt[d.row_cfg], d.rows, d.cols, 1,
                   t0, cnt, flags, d.rows == 1 ? s : 1.0f, lds);
        // publish: own stores acknowledged by the L2, workgroup joined, one increment
        if (a.fenced) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_fetch_add(done, (unsigned)cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        if (d.nrow_items > 0) {
          // Bounded wait: the counter always completes (see the file comment);
          // the bound only guarantees that every wave exits even if that were
          // broken, in which case the host flag is set and the item skipped.
          if (threadIdx.x == 0) {
            int spins = 0;
            bool give_up = a.max_spins < 0;
            while (!give_up &&
                   __hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)d.nrow_items) {
              if (spins++ >= a.max_spins) give_up = true;
              else __builtin_amdgcn_s_sleep(2);
            }
            // a plain store to host memory (no PCIe atomic); the host only tests for non-zero
            if (give_up) __hip_atomic_store(a.err_host, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            s_flag = give_up ? 1 : 0;
            if (a.fenced) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          }
          __syncthreads();
          const bool timed_out = s_flag != 0;
          __syncthreads();
          if (timed_out) continue;
        }
        // without a row pass (cols == 1) the column item reads the input and conjugates it itself
        const int flags = inv ? (d.nrow_items > 0 ? 2 : 3) : 0;
        const float2* src = d.m1 > 1 ? d.work : (d.nrow_items > 0 ? d.out : d.in);
        run_tile(d.col_cfg, src, d.out, a.tw + a.tw_off[d.col_cfg], a.tw_cnt[d.col_cfg], d.rows, d.cols, d.m1,
                 t0, cnt, flags, s, lds);
      }
      __syncthreads();  // the LDS of this item is free before the next item starts
    }
  }
  // Drain check. A workgroup leaves the loop only after popping past the end
  // of its queue, so a queue that any workgroup served was popped at least
  // once per group. The last workgroup to leave reads every head; a queue
  // with fewer pops than groups had no workgroup (its XCD received none of
  // this launch's workgroups) and its transforms were not computed: the host
  // flag makes the plan's next call return FFT2D_ERR_INCOMPLETE. Both reads
  // are atomics at agent scope, so they see every other workgroup's pops
  // (each of which returned before that workgroup's increment was issued).
  if (threadIdx.x == 0) {
    const unsigned prev = __hip_atomic_fetch_add(&a.counters[kFinishSlot], 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    if (prev + 1u == gridDim.x) {
      bool undrained = false;
      for (int x = 0; x < a.nq; ++x) {
        const unsigned h = __hip_atomic_fetch_add(&a.counters[x * kQueueStride], 0u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        if ((int64_t)h < (int64_t)(a.qbeg[x + 1] - a.qbeg[x]) + a.drain_slack) undrained = true;
      }
      if (undrained) __hip_atomic_store(a.err_host, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// ---------------------------------------------------------------- host side
template <class K>
constexpr PassKernel bdesc() {
  return meta<K>();
}

const PassKernel* cfg_table() {
  static const PassKernel tab[kNumCfg] = {
      PassKernel{},   bdesc<BR2>(),    bdesc<BR4>(),    bdesc<BR8>(),   bdesc<BR16>(),   bdesc<BR32>(),
      bdesc<BR64>(),  bdesc<BR128>(),  bdesc<BR256>(),  bdesc<BR512>(), bdesc<BR1024>(), bdesc<BR2048>(),
      bdesc<BR4096>(), bdesc<BR8192>(), bdesc<BR16384>(), PassKernel{},  PassKernel{},    bdesc<BC2>(),
      bdesc<BC4>(),   bdesc<BC8>(),    bdesc<BC16>(),   bdesc<BC32>(),  bdesc<BC64>(),   bdesc<BC128>(),
      bdesc<BC256>(), bdesc<BC512>(),  bdesc<BC1024>(), bdesc<BC2048>(), bdesc<BC4096>(), bdesc<BC8192>(),
      bdesc<BC16384>(), PassKernel{},  PassKernel{},   PassKernel{},    PassKernel{},    PassKernel{},
      PassKernel{},   PassKernel{},    PassKernel{},    PassKernel{},   PassKernel{},    bdesc<BRC512>(),
      bdesc<BRC1024>(), bdesc<BRC2048>(), bdesc<BRC4096>(), bdesc<BRC8192>(), PassKernel{}, PassKernel{},
      // variant 1: ids 48 + mode * 16 + log2(L)
      PassKernel{}, PassKernel{}, PassKernel{}, PassKernel{}, PassKernel{}, bdesc<BR32v>(),
      bdesc<BR64v>(), bdesc<BR128v>(), bdesc<BR256v>(), bdesc<BR512v>(), bdesc<BR1024v>(), bdesc<BR2048v>(),
      bdesc<BR4096v>(), bdesc<BR8192v>(), bdesc<BR16384v>(), PassKernel{}, PassKernel{}, PassKernel{},
      PassKernel{}, PassKernel{}, PassKernel{}, bdesc<BC32v>(), bdesc<BC64v>(), bdesc<BC128v>(),
      bdesc<BC256v>(), bdesc<BC512v>(), bdesc<BC1024v>(), bdesc<BC2048v>(), bdesc<BC4096v>(), bdesc<BC8192v>(),
      bdesc<BC16384v>(), PassKernel{}, PassKernel{}, PassKernel{}, PassKernel{}, PassKernel{},
      PassKernel{}, PassKernel{}, PassKernel{}, PassKernel{}, PassKernel{}, PassKernel{},
      PassKernel{}, PassKernel{}, PassKernel{}, PassKernel{}, PassKernel{}, PassKernel{},
  };
  return tab;
}

// Configuration id of an FFT of length L along rows (mode 0) or columns
// (mode 1) in the given variant; lengths below 32 have variant 0 only.
int cfg_id(int variant, int mode, int log2_len) {
  const int v = log2_len >= kMinVariantLog2 ? variant : 0;
  return v * kVariantStride + mode * 16 + log2_len;
}

int ilog2i(int64_t n) {
  int k = 0;
  while ((int64_t(1) << k) < n) ++k;
  return k;
}

// Grids done as one whole-grid item (one workgroup, one pass through HBM):
// the shapes of at most 16384 points whose row and column configurations
// cover the grid in whole tiles (see grid_item).
bool batched_grid_item(int M, int N) {
  return (M == 64 && (N == 64 || N == 128 || N == 256)) || (N == 64 && (M == 128 || M == 256)) ||
         (M == 128 && N == 128);
}

// Split factor of an M x N transform in a batched plan (1 = plain). Column
// tiles of 2048 or more points per column hold at most 8 columns (64-byte row
// segments) and are the batched kernel's slowest items, and 1024-point columns
// measured faster split too; such a transform is split as in the plain path
// when a row-with-combine configuration exists for N (512 <= N <= 8192, M1 =
// its row count) and leaves columns of at most 1024 points (tiles of at least
// 16 columns).
int batched_split(int M, int N) {
  if (M < 1024 || N < 512 || N > 8192) return 1;
  const PassKernel& k = cfg_table()[32 + ilog2i(N)];
  const int m1 = k.C;
  if (k.L != N || m1 < 2 || M % m1 != 0 || M / m1 > 1024) return 1;
  return m1;
}

}  // namespace

struct BatchedPlan {
  int64_t count = 0;
  std::vector<int32_t> rows, cols;
  std::vector<int32_t> row_cfg, col_cfg, nrow, ncol;
  std::vector<int32_t> m1;          // split factor per transform (1 = plain)
  std::vector<uint8_t> grid;        // 1: one whole-grid item
  int n_grid = 0;
  std::vector<uint8_t> plain;       // 1: run by a uniform plan's row and column kernels (see plain_transform)
  int n_plain = 0;
  std::vector<fft2d_plan_t> sub;    // per transform: its uniform plan (plain transforms), else null
  std::vector<fft2d_plan_t> sub_owned;  // one uniform plan per distinct shape of the plain transforms
  // Plain transforms of one shape, in index order, and a uniform plan of all of
  // them as one batch: used when their buffers are consecutive in memory.
  struct PlainGroup {
    int rows = 0, cols = 0;
    std::vector<int64_t> idx;
    fft2d_plan_t whole = nullptr;
  };
  std::vector<PlainGroup> plain_groups;
  std::vector<int64_t> work_off;    // split transforms: offset in d_work (points)
  int64_t work_points = 0;
  int n_split = 0;
  int64_t total_points = 0;
  double flops = 0;
  int num_cu = 0;
  int nq = 1;           // queues = XCDs
  int fenced = 0;       // 1: queues not tied to XCDs, agent-scope release / acquire
  // tuning choice
  int grid_mult = 2;
  int order = 1;
  int group_kib = 256;  // target data per item group
  bool guided = false;  // guided group sizes (fft_batched_guided.hpp)
  unsigned char variant[2][tune::kVariantSlots] = {};  // radix/tile variant per row / column length (log2)
  std::string tune_source = "default";
  // device state
  BatchDesc* d_desc = nullptr;
  BatchDesc* h_desc = nullptr;  // pinned staging copy
  uint2* d_items = nullptr;
  uint32_t* d_groups = nullptr;
  int n_items = 0;
  int n_groups = 0;
  int qbeg[kMaxQueues + 1] = {};
  unsigned* d_counters = nullptr;
  float2* d_work = nullptr;   // intermediate grids of split transforms
  int twc_off[16] = {};       // offset of W_M^j (j < M) in d_tw, index log2 M (split transforms)
  unsigned* h_err = nullptr;  // pinned, coherent: written by the kernel when a wait gives up
  int max_spins = 0;
  int drain_slack = 0;
  float2* d_tw = nullptr;
  int tw_off[kNumCfg] = {};
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  hipEvent_t staged = nullptr;
  bool staged_pending = false;
  std::vector<const void*> last_in, last_out;
};

// Data pointers of transform i in its descriptor. A split transform's
// intermediate grid always lives in the plan's work buffer: keeping it in the
// output (as the plain path does for out-of-place calls) measured 3 % slower
// for the 512-shape set (1.95 against 1.89 ms), though 3 % faster for
// 32 x 1024^2.
void set_desc_ptrs(BatchedPlan* bp, int64_t i, const float2* in, float2* out) {
  BatchDesc& d = bp->h_desc[i];
  d.in = in;
  d.out = out;
  d.work = d.m1 > 1 ? bp->d_work + bp->work_off[(size_t)i] : nullptr;
}


namespace {

// The scheduler's view of the plan's transforms.
std::vector<sched::Shape> sched_shapes(const BatchedPlan& bp) {
  const PassKernel* tab = cfg_table();
  std::vector<sched::Shape> v((size_t)bp.count);
  for (int64_t i = 0; i < bp.count; ++i) {
    sched::Shape& s = v[(size_t)i];
    s.rows = bp.rows[(size_t)i];
    s.cols = bp.cols[(size_t)i];
    s.m1 = bp.m1[(size_t)i];
    s.grid = bp.grid[(size_t)i];
    s.nrow = bp.nrow[(size_t)i];
    s.ncol = bp.ncol[(size_t)i];
    s.row_c = std::max(1, tab[bp.row_cfg[(size_t)i]].C);
    s.col_c = std::max(1, tab[bp.col_cfg[(size_t)i]].C);
  }
  return v;
}

// Guided grouping (fft_batched_guided.hpp) with FFT2D_BATCH_GUIDED=1. On the
// 512-shape set it cuts the kernel's memory traffic from 1.17 to 1.05-1.07 times
// the algorithmic bytes (fewer calls, fewer register saves) but not its time,
// so fixed groups stay the default.
bool use_guided_groups() {
  const char* env = std::getenv("FFT2D_BATCH_GUIDED");
  return env && (std::string(env) == "1" || std::string(env) == "on");
}

// The schedule for a launch of mult workgroups per CU, over the transforms the
// persistent kernel runs (plain transforms have no items).
sched::Schedule build_schedule(const BatchedPlan& bp, int order, int group_kib, int mult) {
  const std::vector<sched::Shape> all = sched_shapes(bp);
  std::vector<sched::Shape> shapes;
  std::vector<uint32_t> ids;
  for (int64_t i = 0; i < bp.count; ++i) {
    if (bp.plain[(size_t)i]) continue;
    shapes.push_back(all[(size_t)i]);
    ids.push_back((uint32_t)i);
  }
  sched::Schedule sc = sched::build_schedule(shapes, bp.nq, order, group_kib);
  if (bp.guided)
    sc = sched::guided(sc, shapes, bp.nq, mult * bp.num_cu / std::max(1, bp.nq), (int64_t)group_kib * 1024 / 8);
  for (sched::Item& it : sc.items) it.x = ids[it.x >> 2] << 2 | (it.x & 3u);
  return sc;
}

hipError_t launch_batched(BatchedPlan* bp, int conj, int grid, hipStream_t s) {
  const int nc = kCounterBase + (int)bp->count;
  hipLaunchKernelGGL(clear_counters, dim3((unsigned)std::min(64, (nc + 255) / 256)), dim3(256), 0, s, bp->d_counters, nc);
  BatchArgs a{};
  a.desc = bp->d_desc;
  a.items = bp->d_items;
  a.groups = bp->d_groups;
  for (int x = 0; x <= kMaxQueues; ++x) a.qbeg[x] = bp->qbeg[x];
  a.nq = bp->nq;
  a.counters = bp->d_counters;
  a.tw = bp->d_tw;
  const PassKernel* tab = cfg_table();
  for (int i = 0; i < kNumCfg; ++i) {
    a.tw_off[i] = bp->tw_off[i];
    a.tw_cnt[i] = tab[i].L ? (int)twiddle_count(tab[i]) : 0;
  }
  a.conj = conj;
  a.n_fft = (int)bp->count;
  a.fenced = bp->fenced;
  a.err_host = bp->h_err;
  a.max_spins = bp->max_spins;
  a.drain_slack = bp->drain_slack;
  hipLaunchKernelGGL(batched_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t upload_schedule(BatchedPlan* bp, const sched::Schedule& sc) {
  if (bp->d_items) (void)hipFree(bp->d_items);
  if (bp->d_groups) (void)hipFree(bp->d_groups);
  bp->d_items = nullptr;
  bp->d_groups = nullptr;
  bp->n_items = (int)sc.items.size();
  bp->n_groups = (int)sc.groups.size() - 1;
  for (int x = 0; x <= kMaxQueues; ++x) bp->qbeg[x] = sc.qbeg[x];
  hipError_t e = hipMalloc((void**)&bp->d_items, std::max<size_t>(1, sc.items.size()) * sizeof(uint2));
  if (e != hipSuccess) return e;
  static_assert(sizeof(sched::Item) == sizeof(uint2), "item layout");
  e = hipMemcpy(bp->d_items, sc.items.data(), sc.items.size() * sizeof(uint2), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  e = hipMalloc((void**)&bp->d_groups, sc.groups.size() * sizeof(uint32_t));
  if (e != hipSuccess) return e;
  return hipMemcpy(bp->d_groups, sc.groups.data(), sc.groups.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
}

std::string shape_signature(const BatchedPlan& bp) {
  std::map<std::pair<int, int>, int> hist;
  for (int64_t i = 0; i < bp.count; ++i) hist[{bp.rows[i], bp.cols[i]}]++;
  std::ostringstream os;
  for (auto& kv : hist) os << kv.first.first << "x" << kv.first.second << "*" << kv.second << ";";
  return os.str();
}

uint64_t fnv1a(const std::string& s) {
  uint64_t h = 1469598103934665603ull;
  for (unsigned char c : s) {
    h ^= c;
    h *= 1099511628211ull;
  }
  return h;
}

std::string cache_path() {
  const char* p = std::getenv("FFT2D_TUNE_CACHE");
  if (p && *p) return p;
  const char* home = std::getenv("HOME");
  if (!home || !*home) return "";
  return std::string(home) + "/.cache/fft2d_tune.txt";
}

void cache_store(const std::string& key, const tune::Choice& c) {
  const std::string path = cache_path();
  if (path.empty()) return;
  std::ofstream out(path, std::ios::app);
  if (!out) {
    const size_t slash = path.find_last_of('/');
    if (slash == std::string::npos) return;
    (void)::mkdir(path.substr(0, slash).c_str(), 0755);  // one level, best effort
    out.open(path, std::ios::app);
  }
  if (out) out << tune::format_line(key, c) << "\n";
}

// Configuration ids and tile counts of every transform for the plan's
// current variant choice (whole-grid items keep the variant-0 tables their
// kernels use), written to the host descriptors as well.
void assign_configs(BatchedPlan* bp) {
  const PassKernel* tab = cfg_table();
  for (int64_t i = 0; i < bp->count; ++i) {
    const size_t k = (size_t)i;
    const int M = bp->rows[k], N = bp->cols[k], m1 = bp->m1[k];
    const bool whole = bp->grid[k] != 0;
    const int ln = ilog2i(N), lm = ilog2i(M / m1);
    const int rc = m1 > 1 ? 32 + ln : (N > 1 ? cfg_id(whole ? 0 : bp->variant[0][ln], 0, ln) : 0);
    const int cc = M > 1 ? cfg_id(whole ? 0 : bp->variant[1][lm], 1, lm) : 0;
    bp->row_cfg[k] = rc;
    bp->col_cfg[k] = cc;
    // a whole-grid item has no row or column tiles (and nothing to wait for)
    bp->nrow[k] = !whole && N > 1 ? (M + tab[rc].C - 1) / tab[rc].C : 0;
    bp->ncol[k] = !whole && M > 1 ? (int)(((int64_t)m1 * N + tab[cc].C - 1) / tab[cc].C) : 0;
    if (bp->h_desc) {
      bp->h_desc[i].row_cfg = rc;
      bp->h_desc[i].col_cfg = cc;
      bp->h_desc[i].nrow_items = bp->nrow[k];
    }
  }
}

// Lengths (mode, log2 L) whose variant the tuner may choose: those that some
// transform runs as row or column tiles with more than one configuration.
std::vector<std::pair<int, int>> tunable_lengths(const BatchedPlan& bp) {
  bool used[2][tune::kVariantSlots] = {};
  for (int64_t i = 0; i < bp.count; ++i) {
    const size_t k = (size_t)i;
    if (bp.grid[k] || bp.plain[k]) continue;
    const int N = bp.cols[k], M = bp.rows[k], m1 = bp.m1[k];
    if (m1 == 1 && N > 1) used[0][ilog2i(N)] = true;
    if (M > 1) used[1][ilog2i(M / m1)] = true;
  }
  std::vector<std::pair<int, int>> v;
  for (int m = 0; m < 2; ++m)
    for (int j = kMinVariantLog2; j < tune::kVariantSlots; ++j)
      if (used[m][j]) v.push_back({m, j});
  return v;
}

// Time one candidate (grid multiplier, order, group size) on scratch buffers; median of reps.
float time_candidate(BatchedPlan* bp, int mult, int order, int group_kib, hipStream_t s, hipEvent_t e0,
                     hipEvent_t e1) {
  if (upload_schedule(bp, build_schedule(*bp, order, group_kib, mult)) != hipSuccess) return 1e30f;
  std::vector<float> ts;
  for (int r = 0; r < 4; ++r) {
    (void)hipEventRecord(e0, s);
    if (launch_batched(bp, 0, mult * bp->num_cu, s) != hipSuccess) return 1e30f;
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) return 1e30f;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (r > 0) ts.push_back(ms);
  }
  std::sort(ts.begin(), ts.end());
  return ts[ts.size() / 2];
}

}  // namespace

// A transform holding at least 1 / (2 nq) of the plan's points and at least
// 2^22 points runs as a plain transform: its uniform plan's row and column
// kernels, launched on the caller's stream after the persistent kernel, spread
// it over every XCD. In the persistent kernel a transform runs on one XCD, so
// a plan of a few large grids leaves XCDs idle or gives each XCD one long row
// phase and one long column phase with a barrier between them: 4 x 1024 x 8192
// takes 0.46 ms there and 0.23 ms as plain transforms, 8 x 2048^2 0.31 against
// 0.27 ms. Smaller grids stay in the persistent kernel, where two launches per
// grid would cost more than they gain (16 x 2048 x 512: 0.15 ms against 0.28).
// FFT2D_BATCH_PLAIN=off keeps every transform in the persistent kernel.
static bool plain_transform(int64_t points, int64_t total, int nq) {
  return points >= (int64_t(1) << 22) && points * 2 * nq >= total;
}

fft2d_status create_batched(int64_t count, const int64_t* rows, const int64_t* cols, BatchedPlan** out,
                            std::string* err) {
  *out = nullptr;
  BatchedPlan* bp = new (std::nothrow) BatchedPlan();
  if (!bp) {
    *err = "host allocation failed";
    return FFT2D_ERR_OUT_OF_MEMORY;
  }
  auto fail = [&](fft2d_status st, const std::string& msg) {
    destroy_batched(bp);
    *err = msg;
    return st;
  };
  auto hipfail = [&](hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? FFT2D_ERR_OUT_OF_MEMORY : FFT2D_ERR_HIP,
                std::string(what) + ": " + hipGetErrorName(e));
  };
  bp->count = count;
  const PassKernel* tab = cfg_table();
  const char* split_env = std::getenv("FFT2D_BATCH_SPLIT");
  const bool allow_split = !(split_env && std::string(split_env) == "off");
  const char* grid_env = std::getenv("FFT2D_BATCH_GRID");
  const bool allow_grid = !(grid_env && std::string(grid_env) == "off");
  for (int64_t i = 0; i < count; ++i) {
    const int M = (int)rows[i], N = (int)cols[i];
    bp->rows.push_back(M);
    bp->cols.push_back(N);
    const int m1 = allow_split ? batched_split(M, N) : 1;
    bp->m1.push_back(m1);
    bp->work_off.push_back(m1 > 1 ? bp->work_points : 0);
    if (m1 > 1) {
      bp->work_points += (int64_t)M * N;
      ++bp->n_split;
    }
    // split: M / m1 row tiles of m1 rows (combine), columns of M / m1 points in m1 row blocks
    const int rc = m1 > 1 ? 32 + ilog2i(N) : (N > 1 ? ilog2i(N) : 0);
    const int cc = M > 1 ? 16 + ilog2i(M / m1) : 0;
    const bool whole = allow_grid && m1 == 1 && batched_grid_item(M, N);
    bp->grid.push_back(whole ? 1 : 0);
    bp->n_grid += whole ? 1 : 0;
    bp->row_cfg.push_back(rc);
    bp->col_cfg.push_back(cc);
    // a whole-grid item has no row or column tiles (and nothing to wait for)
    bp->nrow.push_back(!whole && N > 1 ? (M + tab[rc].C - 1) / tab[rc].C : 0);
    bp->ncol.push_back(!whole && M > 1 ? (int)(((int64_t)m1 * N + tab[cc].C - 1) / tab[cc].C) : 0);
    bp->total_points += (int64_t)M * N;
    const double p = (double)M * N;
    bp->flops += p > 1 ? 5.0 * p * std::log2(p) : 0.0;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hipfail(e, "hipGetDevice");
  e = hipDeviceGetAttribute(&bp->num_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hipfail(e, "hipDeviceGetAttribute");
  if ((e = hipStreamCreateWithFlags(&bp->cap_stream, hipStreamNonBlocking)) != hipSuccess) return hipfail(e, "stream");
  if ((e = hipEventCreateWithFlags(&bp->staged, hipEventDisableTiming)) != hipSuccess) return hipfail(e, "event");
  // Queue layout. One queue per XCD when probe launches of every candidate
  // grid see XCC_ID values 0 .. k-1, each of them; otherwise one queue with
  // agent-scope release / acquire. FFT2D_BATCH_SYNC=fenced forces the latter.
  {
    const int gmax = 3 * bp->num_cu;
    unsigned* ids = nullptr;
    if ((e = hipMalloc((void**)&ids, (size_t)gmax * sizeof(unsigned))) != hipSuccess) return hipfail(e, "probe");
    std::vector<unsigned> h((size_t)gmax);
    int k = 0;
    bool ok = true;
    for (int m = 1; m <= 3 && ok && e == hipSuccess; ++m) {
      const int g = m * bp->num_cu;
      hipLaunchKernelGGL(xcc_probe, dim3((unsigned)g), dim3(64), 0, bp->cap_stream, ids);
      if ((e = hipGetLastError()) != hipSuccess) break;
      if ((e = hipStreamSynchronize(bp->cap_stream)) != hipSuccess) break;
      if ((e = hipMemcpy(h.data(), ids, (size_t)g * sizeof(unsigned), hipMemcpyDeviceToHost)) != hipSuccess) break;
      unsigned mx = 0;
      for (int i = 0; i < g; ++i) mx = std::max(mx, h[(size_t)i]);
      if (mx >= (unsigned)kMaxQueues) {
        ok = false;
        break;
      }
      std::vector<int> seen(mx + 1, 0);
      for (int i = 0; i < g; ++i) ++seen[h[(size_t)i]];
      if (m == 1) k = (int)mx + 1;
      ok = (int)mx + 1 == k && std::find(seen.begin(), seen.end(), 0) == seen.end();
    }
    (void)hipFree(ids);
    if (e != hipSuccess) return hipfail(e, "XCC probe");
    const char* sync_env = std::getenv("FFT2D_BATCH_SYNC");
    const bool force_fenced = sync_env && std::string(sync_env) == "fenced";
    if (ok && !force_fenced) {
      bp->nq = k;
      bp->fenced = 0;
    } else {
      bp->nq = 1;
      bp->fenced = 1;
    }
  }
  // Plain transforms (see plain_transform); the work buffer, split and
  // whole-grid counts then cover the persistent kernel's transforms only.
  {
    const char* plain_env = std::getenv("FFT2D_BATCH_PLAIN");
    const bool allow_plain = !(plain_env && std::string(plain_env) == "off");
    bp->plain.assign((size_t)count, 0);
    bp->sub.assign((size_t)count, nullptr);
    std::map<std::pair<int, int>, fft2d_plan_t> by_shape;
    bp->work_points = 0;
    bp->n_split = 0;
    bp->n_grid = 0;
    for (int64_t i = 0; i < count; ++i) {
      const size_t k = (size_t)i;
      const int64_t pts = (int64_t)bp->rows[k] * bp->cols[k];
      bp->work_off[k] = 0;
      if (allow_plain && plain_transform(pts, bp->total_points, bp->nq)) {
        bp->plain[k] = 1;
        ++bp->n_plain;
        bp->grid[k] = 0;
        auto it = by_shape.find({bp->rows[k], bp->cols[k]});
        if (it == by_shape.end()) {
          fft2d_plan_t sp = nullptr;
          const fft2d_status st = fft2d_plan(&sp, 1, bp->rows[k], bp->cols[k]);
          if (st != FFT2D_OK) return fail(st, std::string("uniform plan of a large transform: ") + fft2d_last_error());
          bp->sub_owned.push_back(sp);
          it = by_shape.emplace(std::make_pair(bp->rows[k], bp->cols[k]), sp).first;
        }
        bp->sub[k] = it->second;
        auto same_shape = [&](const BatchedPlan::PlainGroup& pg) {
          return pg.rows == bp->rows[k] && pg.cols == bp->cols[k];
        };
        auto g = std::find_if(bp->plain_groups.begin(), bp->plain_groups.end(), same_shape);
        if (g == bp->plain_groups.end()) {
          bp->plain_groups.emplace_back();
          g = bp->plain_groups.end() - 1;
          g->rows = bp->rows[k];
          g->cols = bp->cols[k];
        }
        g->idx.push_back(i);
        continue;
      }
      if (bp->m1[k] > 1) {
        bp->work_off[k] = bp->work_points;
        bp->work_points += pts;
        ++bp->n_split;
      }
      bp->n_grid += bp->grid[k];
    }
    for (BatchedPlan::PlainGroup& g : bp->plain_groups) {
      if (g.idx.size() < 2) continue;
      const fft2d_status st = fft2d_plan(&g.whole, (int64_t)g.idx.size(), g.rows, g.cols);
      if (st != FFT2D_OK) return fail(st, std::string("uniform plan of large transforms: ") + fft2d_last_error());
    }
  }
  // twiddle tables of every configuration (all, so a pointer change never needs new tables)
  {
    std::vector<float2> host;
    for (int c = 0; c < kNumCfg; ++c) {
      bp->tw_off[c] = (int)host.size();
      if (tab[c].L == 0) continue;
      const size_t n = twiddle_count(tab[c]);
      host.resize(host.size() + n);
      if (n) fill_twiddles(tab[c], host.data() + bp->tw_off[c]);
    }
    // W_M^j = exp(-2 pi i j / M), j < M, for the column length M of every split
    // transform (the combine's twiddles), each from its own FP64 cos / sin
    for (int64_t i = 0; i < count; ++i) {
      if (bp->m1[(size_t)i] == 1) continue;
      const int lg = ilog2i(bp->rows[(size_t)i]);
      if (bp->twc_off[lg] != 0) continue;
      const int64_t M = bp->rows[(size_t)i];
      bp->twc_off[lg] = (int)host.size();
      for (int64_t j = 0; j < M; ++j) {
        const double a = 2.0 * M_PI * (double)j / (double)M;
        host.push_back(make_float2((float)std::cos(a), (float)(-std::sin(a))));
      }
    }
    if (host.empty()) host.push_back(make_float2(0.f, 0.f));
    if ((e = hipMalloc((void**)&bp->d_tw, host.size() * sizeof(float2))) != hipSuccess) return hipfail(e, "twiddles");
    if ((e = hipMemcpy(bp->d_tw, host.data(), host.size() * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess)
      return hipfail(e, "twiddle upload");
  }
  if ((e = hipMalloc((void**)&bp->d_desc, (size_t)count * sizeof(BatchDesc))) != hipSuccess)
    return hipfail(e, "descriptor table");
  if ((e = hipHostMalloc((void**)&bp->h_desc, (size_t)count * sizeof(BatchDesc), hipHostMallocDefault)) != hipSuccess)
    return hipfail(e, "pinned descriptor staging");
  if ((e = hipMalloc((void**)&bp->d_counters, (size_t)(kCounterBase + count) * sizeof(unsigned))) != hipSuccess)
    return hipfail(e, "counters");
  if (bp->work_points > 0 &&
      (e = hipMalloc((void**)&bp->d_work, (size_t)bp->work_points * sizeof(float2))) != hipSuccess)
    return hipfail(e, "work buffer of split transforms");
  if ((e = hipHostMalloc((void**)&bp->h_err, sizeof(unsigned), hipHostMallocCoherent | hipHostMallocMapped)) !=
      hipSuccess)
    return hipfail(e, "pinned error word");
  *bp->h_err = 0u;
  // Bound of a column item's wait; FFT2D_BATCH_SPIN_LIMIT (-1 ... 2^24, -1 = give up every wait) lets
  // tests force the give-up path from the host.
  bp->max_spins = kMaxSpins;
  if (const char* sl = std::getenv("FFT2D_BATCH_SPIN_LIMIT")) {
    char* end = nullptr;
    const long v = std::strtol(sl, &end, 10);
    if (end != sl && *end == '\0' && v >= -1 && v <= kMaxSpins) bp->max_spins = (int)v;
  }
  // FFT2D_BATCH_DRAIN_SLACK (0 ... 2^20) raises the drain check's expected pops per queue, so that
  // tests can force the undrained-queue report from the host.
  if (const char* ds = std::getenv("FFT2D_BATCH_DRAIN_SLACK")) {
    char* end = nullptr;
    const long v = std::strtol(ds, &end, 10);
    if (end != ds && *end == '\0' && v >= 0 && v <= (1L << 20)) bp->drain_slack = (int)v;
  }
  for (int64_t i = 0; i < count; ++i) {
    BatchDesc& d = bp->h_desc[i];
    d.in = nullptr;
    d.out = nullptr;
    d.rows = bp->rows[(size_t)i];
    d.cols = bp->cols[(size_t)i];
    d.row_cfg = bp->row_cfg[(size_t)i];
    d.col_cfg = bp->col_cfg[(size_t)i];
    d.nrow_items = bp->nrow[(size_t)i];
    d.m1 = bp->m1[(size_t)i];
    d.work = nullptr;  // set with the data pointers (set_desc_ptrs)
    d.twc_off = d.m1 > 1 ? bp->twc_off[ilog2i(d.rows)] : 0;
    d.pad = 0;
  }

  // Autotuner: persistent grid size (workgroups per CU), item order and group
  // size, then the radix/tile variant of every row and column length,
  // measured on scratch buffers of this plan's shapes, cached per shape set.
  // FFT2D_BATCH_VARIANT=0|1 fixes every length's variant (no variant search).
  const char* tune_env = std::getenv("FFT2D_TUNE");
  const std::string mode = tune_env ? tune_env : "cached";
  const char* var_env = std::getenv("FFT2D_BATCH_VARIANT");
  const int forced_variant = (var_env && (std::string(var_env) == "0" || std::string(var_env) == "1"))
                                 ? (var_env[0] - '0') : -1;
  if (forced_variant >= 0)
    for (int m = 0; m < 2; ++m)
      for (int j = 0; j < tune::kVariantSlots; ++j) bp->variant[m][j] = (unsigned char)forced_variant;
  assign_configs(bp);
  std::ostringstream keys;
  bp->guided = use_guided_groups();
  keys << "gfx950|v5|" << (bp->guided ? "guided|" : "") << (bp->n_plain ? "plain" + std::to_string(bp->n_plain) + "|" : "")
       << (bp->n_split ? "split|" : "")
       << (bp->n_grid ? "whole|" : "")
       << (forced_variant >= 0 ? "variant" + std::to_string(forced_variant) + "|" : "") << shape_signature(*bp);
  char keyhex[32];
  std::snprintf(keyhex, sizeof(keyhex), "%016llx", (unsigned long long)fnv1a(keys.str()));
  bool have = false;
  tune::Choice cached;
  if (mode == "off" || bp->n_plain == count) {
    have = true;
    bp->tune_source = "default";
  } else if (mode != "full" && tune::lookup(cache_path(), keyhex, &cached)) {
    have = true;
    bp->tune_source = "cache";
    bp->grid_mult = cached.grid_mult;
    bp->order = cached.order;
    bp->group_kib = cached.group_kib;
    if (forced_variant < 0) std::memcpy(bp->variant, cached.variant, sizeof(bp->variant));
    assign_configs(bp);
  }
  if (!have) {
    float2 *sin = nullptr, *sout = nullptr;
    const size_t bytes = (size_t)bp->total_points * sizeof(float2);
    if ((e = hipMalloc((void**)&sin, bytes)) != hipSuccess) return hipfail(e, "tuning buffers");
    if ((e = hipMalloc((void**)&sout, bytes)) != hipSuccess) {
      (void)hipFree(sin);
      return hipfail(e, "tuning buffers");
    }
    (void)hipMemsetAsync(sin, 0, bytes, bp->cap_stream);
    int64_t off = 0;
    for (int64_t i = 0; i < count; ++i) {
      set_desc_ptrs(bp, i, sin + off, sout + off);
      off += (int64_t)bp->rows[(size_t)i] * bp->cols[(size_t)i];
    }
    auto upload_desc = [&]() {
      return hipMemcpyAsync(bp->d_desc, bp->h_desc, (size_t)count * sizeof(BatchDesc), hipMemcpyHostToDevice,
                            bp->cap_stream);
    };
    e = upload_desc();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = 1e30f;
    if (e == hipSuccess) {
      const int mults[] = {1, 2, 3};
      const int gks[] = {64, 256, 1024};
      for (int m : mults)
        for (int o = 0; o < 2; ++o)
          for (int g : gks) {
            const float t = time_candidate(bp, m, o, g, bp->cap_stream, e0, e1);
            if (t < best) {
              best = t;
              bp->grid_mult = m;
              bp->order = o;
              bp->group_kib = g;
            }
          }
      // variant descent: flip one length at a time, keep a flip that is at least 1 % faster
      if (forced_variant < 0) {
        for (const auto& ml : tunable_lengths(*bp)) {
          unsigned char& v = bp->variant[ml.first][ml.second];
          v ^= 1u;
          assign_configs(bp);
          float t = 1e30f;
          if ((e = upload_desc()) == hipSuccess)
            t = time_candidate(bp, bp->grid_mult, bp->order, bp->group_kib, bp->cap_stream, e0, e1);
          if (e != hipSuccess) break;
          if (t < 0.99f * best) {
            best = t;
          } else {
            v ^= 1u;
          }
        }
        assign_configs(bp);
      }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(bp->cap_stream);
    (void)hipFree(sin);
    (void)hipFree(sout);
    for (int64_t i = 0; i < count; ++i) bp->h_desc[i].in = bp->h_desc[i].out = bp->h_desc[i].work = nullptr;
    if (e != hipSuccess) return hipfail(e, "autotune");
    if (best >= 1e29f) return fail(FFT2D_ERR_HIP, "autotune: every candidate failed");
    bp->tune_source = "tuned";
    tune::Choice c;
    c.grid_mult = bp->grid_mult;
    c.order = bp->order;
    c.group_kib = bp->group_kib;
    std::memcpy(c.variant, bp->variant, sizeof(c.variant));
    cache_store(keyhex, c);
  }
  if ((e = upload_schedule(bp, build_schedule(*bp, bp->order, bp->group_kib, bp->grid_mult))) != hipSuccess)
    return hipfail(e, "item table");

  // One graph per direction: counter clear (a kernel, no memset node) + the persistent kernel.
  for (int dir = 0; dir < 2; ++dir) {
    if ((e = hipStreamBeginCapture(bp->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hipfail(e, "graph capture");
    hipError_t le = launch_batched(bp, dir, bp->grid_mult * bp->num_cu, bp->cap_stream);
    e = hipStreamEndCapture(bp->cap_stream, &bp->graph[dir]);
    if (le != hipSuccess) return hipfail(le, "graph capture launch");
    if (e != hipSuccess) return hipfail(e, "graph capture end");
    if ((e = hipGraphInstantiate(&bp->exec[dir], bp->graph[dir], nullptr, nullptr, 0)) != hipSuccess)
      return hipfail(e, "graph instantiate");
  }
  *out = bp;
  return FFT2D_OK;
}

fft2d_status exec_batched(BatchedPlan* bp, const void* const* in, void* const* out, int direction, hipStream_t s,
                          std::string* err) {
  // An earlier execution left work undone: its results are incomplete.
  const unsigned flag = __atomic_exchange_n(bp->h_err, 0u, __ATOMIC_ACQ_REL);
  if (flag != 0u) {
    *err = flag == 2u ? "an earlier execution of this batched plan left a queue undrained (no workgroup ran on "
                        "one of the XCDs); its outputs are incomplete"
                      : "an earlier execution of this batched plan gave up waiting for row items; its outputs are "
                        "incomplete";
    return FFT2D_ERR_INCOMPLETE;
  }
  bool changed = bp->last_in.size() != (size_t)bp->count;
  for (int64_t i = 0; i < bp->count; ++i) {
    if (!in[i] || !out[i]) {
      *err = "pointer " + std::to_string(i) + " is NULL";
      return FFT2D_ERR_NULL_POINTER;
    }
    if ((reinterpret_cast<uintptr_t>(in[i]) & 7) || (reinterpret_cast<uintptr_t>(out[i]) & 7)) {
      *err = "pointer " + std::to_string(i) + " is not 8-byte aligned";
      return FFT2D_ERR_MISALIGNED;
    }
    const uintptr_t a = reinterpret_cast<uintptr_t>(in[i]), b = reinterpret_cast<uintptr_t>(out[i]);
    const uintptr_t bytes = (uintptr_t)bp->rows[(size_t)i] * bp->cols[(size_t)i] * 8;
    if (a != b && a < b + bytes && b < a + bytes) {
      *err = "input and output " + std::to_string(i) + " overlap without being identical";
      return FFT2D_ERR_OVERLAP;
    }
    if (!changed && (bp->last_in[(size_t)i] != in[i] || bp->last_out[(size_t)i] != out[i])) changed = true;
  }
  hipError_t e;
  if (changed) {
    // the staging copy may still be read by the previous upload
    if (bp->staged_pending && (e = hipEventSynchronize(bp->staged)) != hipSuccess) {
      *err = std::string("staging wait: ") + hipGetErrorName(e);
      return FFT2D_ERR_HIP;
    }
    for (int64_t i = 0; i < bp->count; ++i) set_desc_ptrs(bp, i, (const float2*)in[i], (float2*)out[i]);
    e = hipMemcpyAsync(bp->d_desc, bp->h_desc, (size_t)bp->count * sizeof(BatchDesc), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(bp->staged, s);
    if (e != hipSuccess) {
      *err = std::string("descriptor upload: ") + hipGetErrorName(e);
      return FFT2D_ERR_HIP;
    }
    bp->staged_pending = true;
    bp->last_in.assign(in, in + bp->count);
    bp->last_out.assign(out, out + bp->count);
  }
  if (bp->n_items > 0) {
    e = hipGraphLaunch(bp->exec[direction == FFT2D_INVERSE ? 1 : 0], s);
    if (e != hipSuccess) {
      *err = std::string("graph launch: ") + hipGetErrorName(e);
      return FFT2D_ERR_HIP;
    }
  }
  // Plain transforms: a group whose inputs follow each other in memory, and
  // whose outputs too (the same buffers, or buffers apart from the inputs),
  // runs as one batch (two launches); otherwise each grid on its own.
  for (const BatchedPlan::PlainGroup& g : bp->plain_groups) {
    const uintptr_t bytes = (uintptr_t)g.rows * g.cols * 8;
    const uintptr_t in0 = reinterpret_cast<uintptr_t>(in[g.idx[0]]);
    const uintptr_t out0 = reinterpret_cast<uintptr_t>(out[g.idx[0]]);
    bool run = g.whole != nullptr;
    for (size_t j = 1; run && j < g.idx.size(); ++j)
      run = reinterpret_cast<uintptr_t>(in[g.idx[j]]) == in0 + j * bytes &&
            reinterpret_cast<uintptr_t>(out[g.idx[j]]) == out0 + j * bytes;
    const uintptr_t span = bytes * g.idx.size();
    if (run && in0 != out0 && in0 < out0 + span && out0 < in0 + span) run = false;
    if (run) {
      const fft2d_status st = fft2d_exec(g.whole, in[g.idx[0]], out[g.idx[0]], direction, (void*)s);
      if (st != FFT2D_OK) {
        *err = std::string("plain transforms from ") + std::to_string(g.idx[0]) + ": " + fft2d_last_error();
        return st;
      }
      continue;
    }
    for (int64_t i : g.idx) {
      const fft2d_status st = fft2d_exec(bp->sub[(size_t)i], in[i], out[i], direction, (void*)s);
      if (st != FFT2D_OK) {
        *err = std::string("plain transform ") + std::to_string(i) + ": " + fft2d_last_error();
        return st;
      }
    }
  }
  return FFT2D_OK;
}

void destroy_batched(BatchedPlan* bp) {
  if (!bp) return;
  for (int d = 0; d < 2; ++d) {
    if (bp->exec[d]) (void)hipGraphExecDestroy(bp->exec[d]);
    if (bp->graph[d]) (void)hipGraphDestroy(bp->graph[d]);
  }
  if (bp->staged) {
    (void)hipEventSynchronize(bp->staged);
    (void)hipEventDestroy(bp->staged);
  }
  if (bp->cap_stream) (void)hipStreamDestroy(bp->cap_stream);
  if (bp->d_desc) (void)hipFree(bp->d_desc);
  if (bp->h_desc) (void)hipHostFree(bp->h_desc);
  if (bp->d_items) (void)hipFree(bp->d_items);
  if (bp->d_groups) (void)hipFree(bp->d_groups);
  if (bp->d_counters) (void)hipFree(bp->d_counters);
  if (bp->d_work) (void)hipFree(bp->d_work);
  if (bp->h_err) (void)hipHostFree(bp->h_err);
  if (bp->d_tw) (void)hipFree(bp->d_tw);
  for (fft2d_plan_t sp : bp->sub_owned) (void)fft2d_destroy(sp);
  for (const BatchedPlan::PlainGroup& g : bp->plain_groups)
    if (g.whole) (void)fft2d_destroy(g.whole);
  delete bp;
}

std::string describe_batched(const BatchedPlan* bp) {
  std::ostringstream os;
  os << "batched count=" << bp->count << " points=" << bp->total_points << " items=" << bp->n_items
     << " groups=" << bp->n_groups << " group_kib=" << bp->group_kib << " plain=" << bp->n_plain
     << " split=" << bp->n_split
     << " whole=" << bp->n_grid
     << " queues=" << bp->nq
     << (bp->fenced ? " fenced" : " xcd-local") << " grid=" << bp->grid_mult << "x" << bp->num_cu
     << " order=" << (bp->order ? "chunked" : "rows-then-columns") << (bp->guided ? " guided" : "")
     << " tune=" << bp->tune_source
     << " variants=";
  // the radix/tile variant chosen for every row (r) and column (c) length that has two
  bool first = true;
  for (const auto& ml : tunable_lengths(*bp)) {
    os << (first ? "" : ",") << (ml.first ? "c" : "r") << (1 << ml.second) << ":"
       << (int)bp->variant[ml.first][ml.second];
    first = false;
  }
  if (first) os << "none";
  os
     << " threads=" << kThreads << " lds=" << kLdsElems * 8;
  return os.str();
}

}  // namespace fft2d
