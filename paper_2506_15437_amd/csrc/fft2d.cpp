// C ABI runtime of the 2D FFT library: plans, FP64-derived twiddle tables,
// argument validation, and the row-pass / column-pass launch sequence.
//
// A 2D transform is one FFT along every row followed by one FFT down every
// column (the paper's Section 5 / Fig. 6 scheme: row FFTs, transposition,
// row FFTs; here the transposition is the column pass's strided tile access,
// so the result stays in natural [k][l] order). Each pass is one kernel launch
// that reads and writes every point once.
#include "fft2d.h"
#include "fft_batched.h"
#include "fft_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

using namespace fft2d;

namespace {

constexpr int kVersion = 100;  // 0.1.0

thread_local std::string g_last_error;
std::mutex g_plans_mu;
std::unordered_set<const void*> g_live_plans;

fft2d_status fail(fft2d_status st, const std::string& detail) {
  g_last_error = detail;
  return st;
}

fft2d_status hip_fail(hipError_t e, const char* what) {
  return fail(FFT2D_ERR_HIP, std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
}

bool pow2_in_range(int64_t n) { return n >= 1 && n <= FFT2D_MAX_LEN && (n & (n - 1)) == 0; }

enum PlanKind { kUniform = 1, kBatched = 2 };

// Number of rows M1 that the row pass combines for a split column transform
// (1 = plain two-pass transform). Large grids split so that the row pass holds
// M1 rows of 128 KiB in total and the column pass works on columns of
// rows / M1 points in 16-column tiles. FFT2D_SPLIT=off|auto|<M1> overrides.
int64_t choose_split(int64_t rows, int64_t cols) {
  auto usable = [&](int64_t m1) {
    return m1 > 1 && rows % m1 == 0 && rows / m1 >= 2 && fft2d::find_combine_kernel((int)cols, (int)m1) &&
           (fft2d::find_split_column_kernel((int)(rows / m1)) || fft2d::find_pass_kernel((int)(rows / m1), true));
  };
  const char* env = std::getenv("FFT2D_SPLIT");
  if (env && std::strcmp(env, "off") == 0) return 1;
  if (env && std::strcmp(env, "auto") != 0 && *env) {
    const int64_t m1 = std::atoll(env);
    return usable(m1) ? m1 : 1;
  }
  if (rows * cols < (int64_t(1) << 22)) return 1;
  // cols = 16384: the unsplit column pass runs tiles of 2-4 columns; M1 = 2
  // (32768 points per workgroup) measured faster from 2048 rows on (8192 x
  // 16384: 1.21 against 1.29 ms; 2048 x 16384: 0.238 against 0.250 ms) and
  // not below (1024 x 16384: 0.119 against 0.118 ms).
  if (cols == 16384) return rows >= 2048 && usable(2) ? 2 : 1;
  // M1 rows of the combine fill one workgroup (16384 points; 32768 for
  // cols = 8192, where M1 = 2 would leave 4096-long, 64-byte-wide columns).
  const int64_t m1 = cols == 8192 ? 4 : 16384 / cols;
  if (usable(m1)) return m1;
  return usable(16384 / cols) ? 16384 / cols : 1;
}

// Whether a plan of `batch` grids of `points` points runs the whole-grid
// kernel (one workgroup per grid) rather than the two passes, which spread
// each grid over many workgroups. Measured crossover on MI355X: grids of 4096
// points gain at any batch, grids of 8192 points from about 32 grids, grids of
// 16384 points from about 128. FFT2D_GRID=on|off overrides (default auto).
bool use_grid_kernel(int64_t batch, int64_t points) {
  const char* env = std::getenv("FFT2D_GRID");
  if (env && std::strcmp(env, "off") == 0) return false;
  if (env && std::strcmp(env, "on") == 0) return true;
  const int64_t min_batch = points <= 4096 ? 1 : points <= 8192 ? 32 : 128;
  return batch >= min_batch;
}

// Whether a split plan's column pass uses the 64-points-per-thread kernels
// (512 threads) where there is one (lengths 2048, 4096, 8192) rather than the
// 32-points ones (1024 threads). Measured on MI355X, forward, faster for every
// split shape tried (8192 x 8192: 0.545 against 0.576 ms; 16384 x 4096: 0.572
// against 0.617; 2 x 16384 x 2048: 0.492 against 0.536; 16384 x 2048: 0.234
// against 0.240). FFT2D_SPLIT_COLUMN=narrow|wide overrides (default auto).
bool use_wide_columns() {
  const char* env = std::getenv("FFT2D_SPLIT_COLUMN");
  return !(env && std::strcmp(env, "narrow") == 0);
}

// Whether a split plan's column pass uses a two-stage radix schedule (one LDS
// exchange: 32 x 32 for 1024-point columns, 64 x 32 for 2048-point columns)
// where there is one, rather than three stages (two exchanges). Measured on
// MI355X, column pass, forward, 1 GiB read before each transform: 8192^2
// 275.2 against 294.4 us, 16384 x 2048 109.3 against 119.1 us, 4096^2 45.5
// against 48.2 us. FFT2D_COLUMN_STAGES=two|classic overrides (default two).
bool use_two_stage_columns() {
  const char* env = std::getenv("FFT2D_COLUMN_STAGES");
  return !(env && std::strcmp(env, "classic") == 0);
}

// Whether a plain pass over `vectors` rows or columns, whose default kernel
// takes `c` of them per tile, uses the narrower-tile kernel: when the default
// would give at most one tile per CU (rows; one 1024^2 grid has 256 row tiles
// and gains) or fewer (columns; at 256 column tiles the narrow kernel measured
// 1-3 % slower). FFT2D_FEW_TILES=off|on overrides (default auto).
bool use_few_tiles_kernel(int64_t vectors, int c, bool colmode) {
  const char* env = std::getenv("FFT2D_FEW_TILES");
  if (env && std::strcmp(env, "off") == 0) return false;
  if (env && std::strcmp(env, "on") == 0) return true;
  const int64_t tiles = vectors / c;
  return colmode ? tiles < 256 : tiles <= 256;
}

// Whether a column pass hands each XCD a contiguous range of tiles
// (xcd_remap) rather than running tiles in launch order, which spreads
// consecutive tiles over the 8 XCDs. The remap keeps tiles that share 128-byte
// lines (C * 8 < 128 bytes per row segment) on one XCD's L2; tiles of whole
// lines gain nothing from it, and launch order, where the tiles in flight
// cover one contiguous span of every row, measured faster for them (column
// pass, 1 GiB read before each transform: 4096^2 49.1 against 51.4 us,
// 16384 x 2048 120.3 against 127.4 us, 8 x 2048^2 82.5 against 86.9 us,
// 8192^2 unchanged). FFT2D_COLUMN_REMAP=0|1 overrides.
int use_xcd_remap(const PassKernel& k) {
  const char* env = std::getenv("FFT2D_COLUMN_REMAP");
  if (env && std::strcmp(env, "0") == 0) return 0;
  if (env && std::strcmp(env, "1") == 0) return 1;
  return k.C * 8 < 128 ? 1 : 0;
}

// Whether the few-tiles row pass of 1024-point rows (one row per wave) runs
// its second exchange in registers across the wave's 16-lane rows
// (v_permlane32_swap / v_permlane16_swap) rather than through the LDS.
// Measured on MI355X, row pass of 1024 x 1024, forward, 1 GiB read before
// each transform: 6.95 against 7.06 us (means of four runs each); 512 x 1024
// 5.73 against 5.89 us. FFT2D_ROW_SHUFFLE=on|off overrides (default on).
bool use_wave_shuffle() {
  const char* env = std::getenv("FFT2D_ROW_SHUFFLE");
  return !(env && std::strcmp(env, "off") == 0);
}

// Whether a split plan's two-stage column pass loads its input nontemporally
// (the row pass's output, read once): for grids of at least 256 MiB, about
// the MALL's size, whose intermediate then comes mostly from HBM. Measured on
// MI355X, column pass, forward, 1 GiB read before each transform: 8192^2
// 253.0 against 275.9 us, 16384 x 2048 101.3 against 109.1 us, 4096^2 (from
// the MALL) 45.6 against 45.3 us. FFT2D_COLUMN_NT=auto|on|off overrides.
bool use_nontemporal_columns(int64_t points) {
  const char* env = std::getenv("FFT2D_COLUMN_NT");
  if (env && std::strcmp(env, "on") == 0) return true;
  if (env && std::strcmp(env, "off") == 0) return false;
  return points * 8 >= (int64_t(256) << 20);
}

// Whether a split plan's row pass takes the combine kernel with 64 points per
// thread (256 threads) where there is one (4096-point rows, M1 = 4) rather
// than 32 (512 threads): for at most 1024 tiles (one 4096^2 grid), where both
// run in two rounds of workgroups. Measured on MI355X, row pass, forward, 1 GiB
// read before each transform: 4096^2 51.6-52.5 against 55.2-55.9 us; two
// 4096^2 grids 104.2 against 99.5 us. FFT2D_COMBINE_WIDE=auto|on|off overrides.
bool use_wide_combine(int64_t tiles) {
  const char* env = std::getenv("FFT2D_COMBINE_WIDE");
  if (env && std::strcmp(env, "on") == 0) return true;
  if (env && std::strcmp(env, "off") == 0) return false;
  return tiles <= 1024;
}

// Whether a split plan's row pass runs the combine kernel whose last FFT stage
// works across the workgroup's rows (rowx_kernel: one LDS exchange fewer)
// rather than the one with a separate combine exchange (rowc_kernel), where
// both exist for the row length. Measured on MI355X, row pass, forward, 1 GiB
// read before each transform: 8192^2 224.9 against 246.2 us, 16384 x 2048
// 107.4 against 112.4 us, 8 x 2048^2 102.2 against 109.1 us, 4096^2 55.4
// against 57.2 us. FFT2D_COMBINE=xrow|classic overrides (default xrow).
bool use_cross_row_combine() {
  const char* env = std::getenv("FFT2D_COMBINE");
  return !(env && std::strcmp(env, "classic") == 0);
}

// Same FFT length and radix sequence (hence the same twiddle table).
bool same_schedule(const PassKernel& a, const PassKernel& b) {
  if (a.L != b.L || a.npass != b.npass) return false;
  for (int i = 0; i < a.npass; ++i)
    if (a.radix[i] != b.radix[i]) return false;
  return true;
}

}  // namespace

struct fft2d_plan_s {
  int kind = kUniform;
  int device = 0;
  int64_t batch = 0, rows = 0, cols = 0;
  // Plain transform (m1 == 1): row pass in -> out, column pass out -> out.
  // Split transform (m1 > 1, rows = m1 * m2): row pass with an m1-point
  // combine in -> out, then a column pass of length m2 out -> out; in-place
  // calls go through the work buffer (in -> work -> out).
  int64_t m1 = 1, m2 = 0;
  const PassKernel* row_k = nullptr;  // length-cols FFT along rows (null if cols == 1)
  const PassKernel* col_k = nullptr;  // length-rows (or m2) FFT down columns (null if rows == 1)
  // Small grids: both passes in one whole-grid launch (same radix schedules
  // and tables as row_k / col_k, which fft2d_exec_pass still runs).
  const GridKernel* grid_k = nullptr;
  float2* tw_row = nullptr;
  float2* tw_col = nullptr;
  float2* tw_comb = nullptr;  // W_rows^j, j < rows (split transforms)
  float2* work = nullptr;     // batch*rows*cols points (split transforms)
  int col_remap = 0;          // column passes: 1 = XCD-contiguous tile order (use_xcd_remap)
  BatchedPlan* batched = nullptr;
};

namespace fft2d {

fft2d_status report_error(fft2d_status st, const std::string& detail) { return fail(st, detail); }

void fill_twiddles(const PassKernel& k, float2* tab) {
  // Pass p >= 1, radix R, Ns = product of earlier radices: entry (r, k) is
  // exp(-2 pi i k r / (Ns R)) for r in [1, R), k in [0, Ns). The exponent
  // k r < Ns R is reduced exactly; every value comes from its own FP64 cos/sin
  // and is rounded once to FP32 (no recurrences).
  size_t o = 0;
  int64_t ns = 1;
  for (int p = 0; p < k.npass; ++p) {
    const int R = k.radix[p];
    if (p > 0) {
      const int64_t span = ns * R;
      for (int r = 1; r < R; ++r) {
        for (int64_t kk = 0; kk < ns; ++kk) {
          const double a = 2.0 * M_PI * (double)(kk * r) / (double)span;
          tab[o++] = make_float2((float)std::cos(a), (float)(-std::sin(a)));
        }
      }
    }
    ns *= R;
  }
}

hipError_t upload_twiddles(const PassKernel& k, float2** dev) {
  *dev = nullptr;
  const size_t n = twiddle_count(k);
  if (n == 0) return hipSuccess;
  std::vector<float2> host(n);
  fill_twiddles(k, host.data());
  hipError_t e = hipMalloc((void**)dev, n * sizeof(float2));
  if (e != hipSuccess) {
    *dev = nullptr;
    return e;
  }
  e = hipMemcpy(*dev, host.data(), n * sizeof(float2), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(*dev);
    *dev = nullptr;
  }
  return e;
}

hipError_t upload_root_table(int64_t n, float2** dev) {
  // w[j] = exp(-2 pi i j / n), j < n, each from its own FP64 cos/sin.
  std::vector<float2> host((size_t)n);
  for (int64_t j = 0; j < n; ++j) {
    const double a = 2.0 * M_PI * (double)j / (double)n;
    host[(size_t)j] = make_float2((float)std::cos(a), (float)(-std::sin(a)));
  }
  hipError_t e = hipMalloc((void**)dev, (size_t)n * sizeof(float2));
  if (e != hipSuccess) {
    *dev = nullptr;
    return e;
  }
  e = hipMemcpy(*dev, host.data(), (size_t)n * sizeof(float2), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(*dev);
    *dev = nullptr;
  }
  return e;
}

// Launch one pass kernel: the pass itself, or with probe = 1 or 2 its
// measurement variant (see PassKernel::launch_probe).
fft2d_status launch_one(const PassKernel* k, const PassArgs& a, int sign, hipStream_t s, hipEvent_t t0,
                        hipEvent_t t1, int probe, const char* what) {
  hipError_t e;
  if (probe) {
    if (!k->launch_probe) return fail(FFT2D_ERR_INVALID_SIZE, std::string("no measurement variant of the ") + what);
    e = k->launch_probe(a, probe, s, t0, t1);
  } else {
    e = k->launch(a, sign, s, t0, t1);
  }
  return e == hipSuccess ? FFT2D_OK : hip_fail(e, what);
}

// Enqueue the transform of nb consecutive grids of rows x cols (in, out and
// work point at the first of them): the whole-grid kernel, or the row pass then
// the column pass (only_pass = 0 or 1 restricts it to one of them; t0, t1:
// timing events bound to that pass's launch, or null; probe: 0, or the
// measurement variant of the pass, with only_pass 0 or 1).
fft2d_status run_grids(const fft2d_plan_s* p, int64_t nb, const float2* in, float2* out, float2* work, int sign,
                       float scale, hipStream_t s, int only_pass, hipEvent_t t0, hipEvent_t t1, int probe) {
  const int64_t npts = nb * p->rows * p->cols;
  hipError_t e;
  if (!p->row_k && !p->col_k) {
    e = launch_scale_copy(in, out, npts, scale, s);
    return e == hipSuccess ? FFT2D_OK : hip_fail(e, "scale copy launch");
  }
  if (p->grid_k && only_pass < 0) {
    PassArgs a{};
    a.in = in;
    a.out = out;
    a.tw = p->tw_row;
    a.tw_count = (int64_t)twiddle_count(*p->row_k);
    a.twc = p->tw_col;
    a.total = npts;
    a.nvec = nb;
    a.scale = scale;
    a.nblocks = (int)nb;
    e = p->grid_k->launch(a, sign, s);
    return e == hipSuccess ? FFT2D_OK : hip_fail(e, "whole-grid kernel launch");
  }
  if (p->m1 > 1) {
    // The intermediate grid: `out` itself (the column pass then runs in place)
    // unless the call is in place, where the row pass must not overwrite rows
    // that other workgroups still read: then the plan's work buffer.
    float2* mid = (static_cast<const void*>(in) == static_cast<const void*>(out)) ? work : out;
    if (only_pass != 1) {
      PassArgs a{};
      a.in = in;
      a.out = mid;
      a.tw = p->tw_row;
      a.tw_count = (int64_t)twiddle_count(*p->row_k);
      a.total = npts;
      a.twc = p->tw_comb;
      a.nvec = nb * p->rows;
      a.ncols = p->cols;
      a.m1 = p->m1;
      a.m2 = p->m2;
      a.scale = 1.0f;
      a.nblocks = (int)(nb * p->m2);
      const fft2d_status st = launch_one(p->row_k, a, sign, s, t0, t1, probe, "row pass (combine) launch");
      if (st != FFT2D_OK) return st;
    }
    if (only_pass != 0) {
      PassArgs a{};
      a.in = mid;
      a.out = out;
      a.tw = p->tw_col;
      a.tw_count = (int64_t)twiddle_count(*p->col_k);
      a.total = npts;
      a.nvec = nb * p->m1 * p->cols;
      a.ncols = p->cols;
      a.m1 = p->m1;
      a.m2 = p->m2;
      a.scale = scale;
      a.nblocks = pass_blocks(*p->col_k, a.nvec);
      a.remap = p->col_remap;
      const fft2d_status st = launch_one(p->col_k, a, sign, s, t0, t1, probe, "column pass launch");
      if (st != FFT2D_OK) return st;
    }
    return FFT2D_OK;
  }
  const float2* src = only_pass == 1 ? out : in;
  if (p->row_k && only_pass != 1) {
    PassArgs a{};
    a.in = src;
    a.out = out;
    a.tw = p->tw_row;
    a.tw_count = (int64_t)twiddle_count(*p->row_k);
    a.total = npts;
    a.nvec = nb * p->rows;
    a.ncols = p->cols;
    a.m1 = 1;
    a.scale = p->col_k ? 1.0f : scale;
    a.nblocks = pass_blocks(*p->row_k, a.nvec);
    const fft2d_status st = launch_one(p->row_k, a, sign, s, only_pass == 0 ? t0 : nullptr,
                                      only_pass == 0 ? t1 : nullptr, probe, "row pass launch");
    if (st != FFT2D_OK) return st;
    src = out;
  }
  if (p->col_k && only_pass != 0) {
    PassArgs a{};
    a.in = src;
    a.out = out;
    a.tw = p->tw_col;
    a.tw_count = (int64_t)twiddle_count(*p->col_k);
    a.total = npts;
    a.nvec = nb * p->cols;
    a.ncols = p->cols;
    a.m1 = 1;
    a.scale = scale;
    a.nblocks = pass_blocks(*p->col_k, a.nvec);
    a.remap = p->col_remap;
    const fft2d_status st = launch_one(p->col_k, a, sign, s, only_pass == 1 ? t0 : nullptr,
                                      only_pass == 1 ? t1 : nullptr, probe, "column pass launch");
    if (st != FFT2D_OK) return st;
  }
  return FFT2D_OK;
}

// Points one launch covers at most. Every kernel runs at least two points per
// thread, so a launch stays below 2^30 work-items (a HIP grid dimension holds
// fewer than 2^32); larger batches run as several launches of whole grids.
constexpr int64_t kMaxLaunchPoints = int64_t(1) << 31;

// Enqueue the transform of the plan's whole batch.
fft2d_status run_uniform(const fft2d_plan_s* p, const float2* in, float2* out, int sign, float scale,
                         hipStream_t s, int only_pass = -1, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr,
                         int probe = 0) {
  const int64_t per = p->rows * p->cols;
  const int64_t chunk = std::max<int64_t>(1, kMaxLaunchPoints / per);
  for (int64_t b0 = 0; b0 < p->batch; b0 += chunk) {
    const int64_t nb = std::min(chunk, p->batch - b0);
    const int64_t off = b0 * per;
    const fft2d_status st =
        run_grids(p, nb, in + off, out + off, p->work ? p->work + off : nullptr, sign, scale, s, only_pass, t0, t1,
                  probe);
    if (st != FFT2D_OK) return st;
  }
  return FFT2D_OK;
}

}  // namespace fft2d

namespace {

bool is_live(const void* p) {
  std::lock_guard<std::mutex> g(g_plans_mu);
  return g_live_plans.count(p) != 0;
}

void free_plan(fft2d_plan_s* p) {
  if (!p) return;
  if (p->tw_row) (void)hipFree(p->tw_row);
  if (p->tw_col) (void)hipFree(p->tw_col);
  if (p->tw_comb) (void)hipFree(p->tw_comb);
  if (p->work) (void)hipFree(p->work);
  if (p->batched) destroy_batched(p->batched);
  delete p;
}

// Kernels run on the current HIP device; a plan's tables and buffers live on
// the device that was current when it was made.
fft2d_status check_device(const fft2d_plan_s* p) {
  int cur = -1;
  const hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != p->device)
    return fail(FFT2D_ERR_WRONG_DEVICE, "the current HIP device is " + std::to_string(cur) + ", the plan's is " +
                                            std::to_string(p->device));
  return FFT2D_OK;
}

fft2d_status check_data_ptrs(const void* in, const void* out, int64_t bytes) {
  if (!in || !out) return fail(FFT2D_ERR_NULL_POINTER, "input or output pointer is NULL");
  if ((reinterpret_cast<uintptr_t>(in) & 7) || (reinterpret_cast<uintptr_t>(out) & 7))
    return fail(FFT2D_ERR_MISALIGNED, "data pointers must be 8-byte aligned (complex64)");
  const uintptr_t a = reinterpret_cast<uintptr_t>(in), b = reinterpret_cast<uintptr_t>(out);
  if (a != b && a < b + (uintptr_t)bytes && b < a + (uintptr_t)bytes)
    return fail(FFT2D_ERR_OVERLAP, "input and output overlap without being identical");
  return FFT2D_OK;
}

fft2d_status check_shape(int64_t batch, int64_t rows, int64_t cols) {
  if (batch < 1) return fail(FFT2D_ERR_INVALID_SIZE, "batch must be >= 1");
  if (!pow2_in_range(rows) || !pow2_in_range(cols))
    return fail(FFT2D_ERR_INVALID_SIZE, "rows and cols must be powers of two in [1, 16384], got " +
                                            std::to_string(rows) + "x" + std::to_string(cols));
  // 2^35 points (256 GiB of complex64) bound every grid-size computation well inside 32 bits
  if (batch > (int64_t(1) << 35) / (rows * cols))
    return fail(FFT2D_ERR_INVALID_SIZE, "batch*rows*cols exceeds 2^35 points");
  return FFT2D_OK;
}

// Kernel choice of a uniform plan (split factor, pass kernels, whole-grid
// kernel); host only, no device memory.
fft2d_status select_kernels(fft2d_plan_s* p, int64_t batch, int64_t rows, int64_t cols) {
  p->kind = kUniform;
  p->batch = batch;
  p->rows = rows;
  p->cols = cols;
  p->m1 = choose_split(rows, cols);
  p->m2 = rows / p->m1;

  if (p->m1 > 1) {
    p->row_k = find_combine_kernel((int)cols, (int)p->m1, use_cross_row_combine(), use_wide_combine(batch * p->m2));
    p->col_k = find_split_column_kernel((int)p->m2, use_wide_columns(), use_two_stage_columns(),
                                        use_nontemporal_columns(batch * rows * cols));
    if (!p->col_k) p->col_k = find_pass_kernel((int)p->m2, true);
  } else {
    if (cols > 1) p->row_k = find_pass_kernel((int)cols, false);
    if (rows > 1) p->col_k = find_pass_kernel((int)rows, true);
    if (p->row_k && use_few_tiles_kernel(batch * rows, p->row_k->C, false)) {
      if (const PassKernel* f = find_few_tiles_kernel((int)cols, false, use_wave_shuffle())) p->row_k = f;
    }
    if (p->col_k && use_few_tiles_kernel(batch * cols, p->col_k->C, true)) {
      if (const PassKernel* f = find_few_tiles_kernel((int)rows, true)) p->col_k = f;
    }
    const GridKernel* g = find_grid_kernel((int)rows, (int)cols);
    if (g && p->row_k && p->col_k && same_schedule(g->row, *p->row_k) && same_schedule(g->col, *p->col_k) &&
        use_grid_kernel(batch, rows * cols))
      p->grid_k = g;
  }
  if ((cols > 1 && !p->row_k) || (rows > 1 && !p->col_k))
    return fail(FFT2D_ERR_INVALID_SIZE, "no kernel for this length");
  p->col_remap = p->col_k ? use_xcd_remap(*p->col_k) : 0;
  return FFT2D_OK;
}

// ------------------------------------------------------------------------
// Allocation-free execution (fft2d_exec_noalloc). The twiddle tables and the
// work buffer of in-place split transforms live in one file-scope device
// array instead of plan memory: every GPU the library runs on holds one copy
// of it from the first use of this code object until the process ends. The
// tables are rewritten on the caller's stream by every call, so calls that
// overlap on one GPU race on the array.
constexpr int64_t kNoallocTableSlot = FFT2D_MAX_LEN;  // entries per table (row, column, combine)
constexpr int64_t kNoallocTablePoints = 3 * kNoallocTableSlot;
constexpr int64_t kNoallocWorkPoints = FFT2D_NOALLOC_WORK_BYTES / 8;
static_assert(FFT2D_NOALLOC_WORK_BYTES % 8 == 0, "whole complex64 points");

static __device__ __align__(256) float2 scratch[kNoallocTablePoints + kNoallocWorkPoints];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float2* g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device, once looked up

// The current device's copy of `scratch` (its address is looked up once per
// device, with that device current; host code never uses the array's name as
// an address).
fft2d_status scratch_of_current_device(float2** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(FFT2D_ERR_INVALID_SIZE, "device index " + std::to_string(dev) + " is beyond the library's 64");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(FFT2D_ERR_HIP, "hipGetSymbolAddress(scratch) gave a null address");
    g_scratch[dev] = static_cast<float2*>(ptr);
  }
  *out = g_scratch[dev];
  return FFT2D_OK;
}

// One table to fill on the device: a schedule's inter-pass table (npass >= 2;
// entry (r, k) of pass p >= 1 is exp(-2 pi i k r / (Ns_p R_p)), the layout
// of fill_twiddles) or, with npass == 0, the root table exp(-2 pi i j / count),
// j < count. count == 0: nothing.
struct TableSpec {
  float2* dst;
  int count;
  int npass;
  int off[kMaxPasses + 1];  // first entry of pass p >= 1; off[npass] = count
  int ns[kMaxPasses];
  int radix[kMaxPasses];
};

TableSpec schedule_spec(const PassKernel* k, float2* dst) {
  TableSpec t{};
  t.dst = dst;
  if (!k) return t;
  int o = 0, ns = 1;
  t.npass = k->npass;
  for (int p = 0; p < k->npass; ++p) {
    t.off[p] = o;
    t.ns[p] = ns;
    t.radix[p] = k->radix[p];
    if (p > 0) o += ns * (k->radix[p] - 1);
    ns *= k->radix[p];
  }
  t.off[k->npass] = o;
  t.count = o;
  if (t.npass < 2) t.count = 0;  // a one-pass schedule has no table
  return t;
}

// Every entry from its own angle: sincospi of 2 q / n, exact in FP64 (n is a
// power of two), then rounded once to FP32.
__global__ void fill_tables_kernel(TableSpec t0, TableSpec t1, TableSpec t2) {
  const TableSpec t = blockIdx.y == 0 ? t0 : (blockIdx.y == 1 ? t1 : t2);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < t.count; i += gridDim.x * blockDim.x) {
    int64_t q = i, n = t.count;
    if (t.npass > 0) {
      int p = 1;
      while (p + 1 < t.npass && i >= t.off[p + 1]) ++p;
      const int rel = i - t.off[p];
      q = (int64_t)(rel % t.ns[p]) * (1 + rel / t.ns[p]);
      n = (int64_t)t.ns[p] * t.radix[p];
    }
    double sn = 0.0, cs = 0.0;
    sincospi(2.0 * (double)q / (double)n, &sn, &cs);
    t.dst[i] = make_float2((float)cs, (float)(-sn));
  }
}

}  // namespace

extern "C" {

fft2d_status fft2d_plan(fft2d_plan_t* out, int64_t batch, int64_t rows, int64_t cols) {
  if (!out) return fail(FFT2D_ERR_NULL_POINTER, "plan output pointer is NULL");
  *out = nullptr;
  if (fft2d_status st = check_shape(batch, rows, cols); st != FFT2D_OK) return st;
  fft2d_plan_s* p = new (std::nothrow) fft2d_plan_s();
  if (!p) return fail(FFT2D_ERR_OUT_OF_MEMORY, "host allocation failed");
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipGetDevice");
  }
  if (fft2d_status st = select_kernels(p, batch, rows, cols); st != FFT2D_OK) {
    delete p;
    return st;
  }
  auto oom_or_hip = [&](hipError_t err, const char* what) {
    free_plan(p);
    return err == hipErrorOutOfMemory ? fail(FFT2D_ERR_OUT_OF_MEMORY, what) : hip_fail(err, what);
  };
  if (p->row_k && (e = upload_twiddles(*p->row_k, &p->tw_row)) != hipSuccess) return oom_or_hip(e, "twiddle table");
  if (p->col_k && (e = upload_twiddles(*p->col_k, &p->tw_col)) != hipSuccess) return oom_or_hip(e, "twiddle table");
  if (p->m1 > 1) {
    if ((e = upload_root_table(rows, &p->tw_comb)) != hipSuccess) return oom_or_hip(e, "twiddle table");
    if ((e = hipMalloc((void**)&p->work, (size_t)(batch * rows * cols) * sizeof(float2))) != hipSuccess) {
      p->work = nullptr;
      return oom_or_hip(e, "work buffer");
    }
  }
  {
    std::lock_guard<std::mutex> g(g_plans_mu);
    g_live_plans.insert(p);
  }
  *out = p;
  return FFT2D_OK;
}

fft2d_status fft2d_plan_batched(fft2d_plan_t* out, int64_t count, const int64_t* rows, const int64_t* cols) {
  if (!out) return fail(FFT2D_ERR_NULL_POINTER, "plan output pointer is NULL");
  *out = nullptr;
  if (!rows || !cols) return fail(FFT2D_ERR_NULL_POINTER, "rows/cols arrays are NULL");
  if (count < 1 || count > (int64_t(1) << 24)) return fail(FFT2D_ERR_INVALID_SIZE, "count must be in [1, 2^24]");
  for (int64_t i = 0; i < count; ++i)
    if (!pow2_in_range(rows[i]) || !pow2_in_range(cols[i]))
      return fail(FFT2D_ERR_INVALID_SIZE, "shape " + std::to_string(i) + " is not a power of two in [1, 16384]");
  fft2d_plan_s* p = new (std::nothrow) fft2d_plan_s();
  if (!p) return fail(FFT2D_ERR_OUT_OF_MEMORY, "host allocation failed");
  p->kind = kBatched;
  p->batch = count;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipGetDevice");
  }
  std::string err;
  fft2d_status st = create_batched(count, rows, cols, &p->batched, &err);
  if (st != FFT2D_OK) {
    delete p;
    return fail(st, err);
  }
  {
    std::lock_guard<std::mutex> g(g_plans_mu);
    g_live_plans.insert(p);
  }
  *out = p;
  return FFT2D_OK;
}

fft2d_status fft2d_exec(fft2d_plan_t plan, const void* in, void* out, int direction, void* stream) {
  if (!plan) return fail(FFT2D_ERR_NULL_POINTER, "plan is NULL");
  if (!is_live(plan)) return fail(FFT2D_ERR_INVALID_PLAN, "plan handle is not live");
  if (plan->kind != kUniform) return fail(FFT2D_ERR_WRONG_PLAN_KIND, "batched plan passed to fft2d_exec");
  if (fft2d_status dst = check_device(plan); dst != FFT2D_OK) return dst;
  if (direction != FFT2D_FORWARD && direction != FFT2D_INVERSE)
    return fail(FFT2D_ERR_INVALID_DIRECTION, "direction must be FFT2D_FORWARD (-1) or FFT2D_INVERSE (+1)");
  const int64_t bytes = plan->batch * plan->rows * plan->cols * 8;
  fft2d_status st = check_data_ptrs(in, out, bytes);
  if (st != FFT2D_OK) return st;
  const float scale = direction == FFT2D_INVERSE ? (float)(1.0 / (double)(plan->rows * plan->cols)) : 1.0f;
  return run_uniform(plan, (const float2*)in, (float2*)out, direction, scale, (hipStream_t)stream);
}

fft2d_status fft2d_backward(fft2d_plan_t plan, const void* grad_out, void* grad_in, int forward_direction,
                            void* stream) {
  if (!plan) return fail(FFT2D_ERR_NULL_POINTER, "plan is NULL");
  if (!is_live(plan)) return fail(FFT2D_ERR_INVALID_PLAN, "plan handle is not live");
  if (plan->kind != kUniform) return fail(FFT2D_ERR_WRONG_PLAN_KIND, "batched plan passed to fft2d_backward");
  if (fft2d_status dst = check_device(plan); dst != FFT2D_OK) return dst;
  if (forward_direction != FFT2D_FORWARD && forward_direction != FFT2D_INVERSE)
    return fail(FFT2D_ERR_INVALID_DIRECTION, "direction must be FFT2D_FORWARD (-1) or FFT2D_INVERSE (+1)");
  const int64_t bytes = plan->batch * plan->rows * plan->cols * 8;
  fft2d_status st = check_data_ptrs(grad_out, grad_in, bytes);
  if (st != FFT2D_OK) return st;
  // Adjoint of y = F x (sign -1, unscaled) is F^H: sign +1, unscaled.
  // Adjoint of y = (1/MN) F^H x is (1/MN) F: sign -1, scaled.
  const int sign = -forward_direction;
  const float scale = forward_direction == FFT2D_INVERSE ? (float)(1.0 / (double)(plan->rows * plan->cols)) : 1.0f;
  return run_uniform(plan, (const float2*)grad_out, (float2*)grad_in, sign, scale, (hipStream_t)stream);
}

namespace {

// Shared by fft2d_exec_pass and fft2d_exec_pass_timed.
fft2d_status exec_one_pass(fft2d_plan_t plan, const void* in, void* out, int direction, int pass, void* stream,
                           hipEvent_t t0, hipEvent_t t1, const char* name, int probe = 0) {
  if (!plan) return fail(FFT2D_ERR_NULL_POINTER, "plan is NULL");
  if (!is_live(plan)) return fail(FFT2D_ERR_INVALID_PLAN, "plan handle is not live");
  if (plan->kind != kUniform) return fail(FFT2D_ERR_WRONG_PLAN_KIND, std::string("batched plan passed to ") + name);
  if (fft2d_status dst = check_device(plan); dst != FFT2D_OK) return dst;
  if (direction != FFT2D_FORWARD && direction != FFT2D_INVERSE)
    return fail(FFT2D_ERR_INVALID_DIRECTION, "direction must be FFT2D_FORWARD (-1) or FFT2D_INVERSE (+1)");
  if (pass != 0 && pass != 1) return fail(FFT2D_ERR_INVALID_DIRECTION, "pass must be 0 (rows) or 1 (columns)");
  if ((pass == 0 && !plan->row_k) || (pass == 1 && !plan->col_k))
    return fail(FFT2D_ERR_INVALID_SIZE, "the plan has no such pass (that dimension has length 1)");
  const int64_t per = plan->rows * plan->cols;
  if ((t0 != nullptr || t1 != nullptr) && plan->batch > std::max<int64_t>(1, kMaxLaunchPoints / per))
    return fail(FFT2D_ERR_INVALID_SIZE, "a timed pass must be one launch (batch of at most 2^31 points)");
  const int64_t bytes = plan->batch * per * 8;
  fft2d_status st = check_data_ptrs(in, out, bytes);
  if (st != FFT2D_OK) return st;
  const float scale = direction == FFT2D_INVERSE ? (float)(1.0 / (double)per) : 1.0f;
  return run_uniform(plan, (const float2*)in, (float2*)out, direction, scale, (hipStream_t)stream, pass, t0, t1,
                     probe);
}

}  // namespace

fft2d_status fft2d_exec_pass(fft2d_plan_t plan, const void* in, void* out, int direction, int pass, void* stream) {
  return exec_one_pass(plan, in, out, direction, pass, stream, nullptr, nullptr, "fft2d_exec_pass");
}

fft2d_status fft2d_exec_pass_timed(fft2d_plan_t plan, const void* in, void* out, int direction, int pass,
                                   void* start_event, void* stop_event, void* stream) {
  if (!start_event || !stop_event) return fail(FFT2D_ERR_NULL_POINTER, "start_event and stop_event must be events");
  return exec_one_pass(plan, in, out, direction, pass, stream, (hipEvent_t)start_event, (hipEvent_t)stop_event,
                       "fft2d_exec_pass_timed");
}

fft2d_status fft2d_exec_pass_ablated(fft2d_plan_t plan, const void* in, void* out, int pass, int ablation,
                                    void* start_event, void* stop_event, void* stream) {
  if (ablation != FFT2D_ABLATE_ARITHMETIC && ablation != FFT2D_ABLATE_EXCHANGE)
    return fail(FFT2D_ERR_INVALID_DIRECTION, "ablation must be FFT2D_ABLATE_ARITHMETIC or FFT2D_ABLATE_EXCHANGE");
  if ((start_event == nullptr) != (stop_event == nullptr))
    return fail(FFT2D_ERR_NULL_POINTER, "give both timing events or neither");
  return exec_one_pass(plan, in, out, FFT2D_FORWARD, pass, stream, (hipEvent_t)start_event, (hipEvent_t)stop_event,
                       "fft2d_exec_pass_ablated", ablation);
}

fft2d_status fft2d_exec_batched(fft2d_plan_t plan, const void* const* in, void* const* out, int direction,
                                void* stream) {
  if (!plan) return fail(FFT2D_ERR_NULL_POINTER, "plan is NULL");
  if (!is_live(plan)) return fail(FFT2D_ERR_INVALID_PLAN, "plan handle is not live");
  if (plan->kind != kBatched) return fail(FFT2D_ERR_WRONG_PLAN_KIND, "uniform plan passed to fft2d_exec_batched");
  if (fft2d_status dst = check_device(plan); dst != FFT2D_OK) return dst;
  if (direction != FFT2D_FORWARD && direction != FFT2D_INVERSE)
    return fail(FFT2D_ERR_INVALID_DIRECTION, "direction must be FFT2D_FORWARD (-1) or FFT2D_INVERSE (+1)");
  if (!in || !out) return fail(FFT2D_ERR_NULL_POINTER, "pointer arrays are NULL");
  std::string err;
  fft2d_status st = exec_batched(plan->batched, in, out, direction, (hipStream_t)stream, &err);
  return st == FFT2D_OK ? st : fail(st, err);
}

fft2d_status fft2d_destroy(fft2d_plan_t plan) {
  if (!plan) return FFT2D_OK;
  {
    std::lock_guard<std::mutex> g(g_plans_mu);
    if (!g_live_plans.erase(plan)) return fail(FFT2D_ERR_INVALID_PLAN, "plan handle is not live");
  }
  free_plan(plan);
  return FFT2D_OK;
}

const char* fft2d_status_string(fft2d_status st) {
  switch (st) {
    case FFT2D_OK: return "success";
    case FFT2D_ERR_NULL_POINTER: return "null pointer";
    case FFT2D_ERR_INVALID_SIZE: return "invalid size";
    case FFT2D_ERR_INVALID_DIRECTION: return "invalid direction";
    case FFT2D_ERR_MISALIGNED: return "misaligned pointer";
    case FFT2D_ERR_WRONG_PLAN_KIND: return "wrong plan kind";
    case FFT2D_ERR_OUT_OF_MEMORY: return "out of memory";
    case FFT2D_ERR_HIP: return "HIP runtime error";
    case FFT2D_ERR_INVALID_PLAN: return "invalid plan";
    case FFT2D_ERR_OVERLAP: return "overlapping buffers";
    case FFT2D_ERR_INCOMPLETE: return "incomplete earlier execution";
    case FFT2D_ERR_WRONG_DEVICE: return "wrong device";
  }
  return "unknown status";
}

const char* fft2d_last_error(void) { return g_last_error.c_str(); }

fft2d_status fft2d_plan_describe(fft2d_plan_t plan, char* buf, int64_t buflen) {
  if (!plan || !buf) return fail(FFT2D_ERR_NULL_POINTER, "plan or buffer is NULL");
  if (buflen < 1) return fail(FFT2D_ERR_INVALID_SIZE, "buffer length must be >= 1");
  if (!is_live(plan)) return fail(FFT2D_ERR_INVALID_PLAN, "plan handle is not live");
  std::string d;
  auto desc = [](const PassKernel* k) {
    if (!k) return std::string("none");
    std::string s = "L=" + std::to_string(k->L) + " radix=";
    for (int i = 0; i < k->npass; ++i) s += (i ? "x" : "") + std::to_string(k->radix[i]);
    s += " E=" + std::to_string(k->E) + " C=" + std::to_string(k->C) + " Q=" + std::to_string(k->Q) +
         " threads=" + std::to_string(k->threads) + " lds=" + std::to_string(k->lds_bytes) +
         (k->wpe > 1 ? " wpe=" + std::to_string(k->wpe) : "") + (k->nt ? " nt" : "") +
         (k->shuffle ? " shuffle" : "");
    return s;
  };
  if (plan->kind == kUniform) {
    d = "uniform batch=" + std::to_string(plan->batch) + " " + std::to_string(plan->rows) + "x" +
        std::to_string(plan->cols) + " split=" + std::to_string(plan->m1) +
        (plan->grid_k ? " grid[threads=" + std::to_string(plan->grid_k->threads) +
                            " lds=" + std::to_string(plan->grid_k->lds_bytes) + "]"
                      : std::string()) +
        " row[" + desc(plan->row_k) +
        (plan->m1 > 1 ? (plan->row_k->xrow ? " combine xrow" : " combine") : "") + "] col[" + desc(plan->col_k) + (plan->col_remap ? " xcd-remap" : "") +
        "]";
  } else {
    d = describe_batched(plan->batched);
  }
  std::snprintf(buf, (size_t)buflen, "%s", d.c_str());
  return FFT2D_OK;
}

fft2d_status fft2d_plan_twiddles(fft2d_plan_t plan, int which, void* host_out, int64_t capacity, int64_t* count) {
  if (!plan || !count) return fail(FFT2D_ERR_NULL_POINTER, "plan or count pointer is NULL");
  if (!is_live(plan)) return fail(FFT2D_ERR_INVALID_PLAN, "plan handle is not live");
  if (plan->kind != kUniform) return fail(FFT2D_ERR_WRONG_PLAN_KIND, "twiddle tables belong to uniform plans");
  if (which < 0 || which > 2) return fail(FFT2D_ERR_INVALID_SIZE, "which must be 0 (row), 1 (column) or 2 (combine)");
  const float2* dev = nullptr;
  int64_t n = 0;
  if (which == 0 && plan->row_k) {
    dev = plan->tw_row;
    n = (int64_t)twiddle_count(*plan->row_k);
  } else if (which == 1 && plan->col_k) {
    dev = plan->tw_col;
    n = (int64_t)twiddle_count(*plan->col_k);
  } else if (which == 2 && plan->m1 > 1) {
    dev = plan->tw_comb;
    n = plan->rows;
  }
  *count = n;
  const int64_t copy = std::min<int64_t>(n, capacity);
  if (copy > 0) {
    if (!host_out) return fail(FFT2D_ERR_NULL_POINTER, "output buffer is NULL");
    const hipError_t e = hipMemcpy(host_out, dev, (size_t)copy * sizeof(float2), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "twiddle download");
  }
  return FFT2D_OK;
}

fft2d_status fft2d_exec_noalloc(int64_t batch, int64_t rows, int64_t cols, const void* in, void* out,
                                int direction, void* stream) {
  if (fft2d_status st = check_shape(batch, rows, cols); st != FFT2D_OK) return st;
  if (direction != FFT2D_FORWARD && direction != FFT2D_INVERSE)
    return fail(FFT2D_ERR_INVALID_DIRECTION, "direction must be FFT2D_FORWARD (-1) or FFT2D_INVERSE (+1)");
  const int64_t points = batch * rows * cols;
  if (fft2d_status st = check_data_ptrs(in, out, points * 8); st != FFT2D_OK) return st;
  fft2d_plan_s p;  // kernel choice only: its tables and work buffer are the scratch array
  if (fft2d_status st = select_kernels(&p, batch, rows, cols); st != FFT2D_OK) return st;
  const bool in_place = static_cast<const void*>(in) == static_cast<const void*>(out);
  if (p.m1 > 1 && in_place && points > kNoallocWorkPoints)
    return fail(FFT2D_ERR_INVALID_SIZE,
                "an in-place call of this shape needs a work buffer of " + std::to_string(points * 8) +
                    " bytes; the allocation-free entry point has " + std::to_string(kNoallocWorkPoints * 8) +
                    " (call it out of place, or use fft2d_plan / fft2d_exec)");
  float2* base = nullptr;
  if (fft2d_status st = scratch_of_current_device(&base); st != FFT2D_OK) return st;
  p.tw_row = base;
  p.tw_col = base + kNoallocTableSlot;
  p.tw_comb = base + 2 * kNoallocTableSlot;
  p.work = (p.m1 > 1 && in_place) ? base + kNoallocTablePoints : nullptr;
  const TableSpec tr = schedule_spec(p.row_k, p.tw_row);
  const TableSpec tc = schedule_spec(p.col_k, p.tw_col);
  TableSpec tm{};
  tm.dst = p.tw_comb;
  tm.count = p.m1 > 1 ? (int)rows : 0;
  const hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(fill_tables_kernel, dim3((unsigned)(kNoallocTableSlot / 256), 3), dim3(256), 0, s, tr, tc, tm);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "twiddle table kernel launch");
  const float scale = direction == FFT2D_INVERSE ? (float)(1.0 / (double)(rows * cols)) : 1.0f;
  return run_uniform(&p, (const float2*)in, (float2*)out, direction, scale, s);
}

int fft2d_version(void) { return kVersion; }

}  // extern "C"
