// Internal interface between the C ABI runtime (fft2d.cpp) and the HIP kernels
// (fft_kernels.hip). Not installed; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <string>

#include "fft2d.h"

namespace fft2d {

constexpr int kMaxPasses = 6;

// Arguments of one pass launch. A pass applies a length-L FFT to `nvec`
// vectors. Row mode: vector v is the L contiguous points starting at v*L.
// Column mode: vector v = g*ncols + col is column `col` of grid g, its element
// e at g*L*ncols + e*ncols + col (stride ncols points; with m1 > 1, vector
// v = (g*m1 + k1)*ncols + col has element e at row k1 + m1*e of grid g).
//
// Split column transform (M = M1 * M2). A row pass with combine handles, per
// workgroup, the M1 rows M2*m1 + m2 (m1 < M1) of one grid: it transforms each
// row, applies an M1-point DFT across them (m1 -> k1), multiplies output k1 by
// W_M^(m2 k1) and stores it to row M1*m2 + k1. A column pass with m1 = M1 then
// transforms, for each k1, the length-M2 column of rows k1 + M1*m2 (m2 < M2)
// and stores element k2 to row k1 + M1*k2: the same rows, so it can run in
// place. Together they are the length-M column DFT (four-step
// factorisation); m1 = 1 is the plain column pass.
struct PassArgs {
  const float2* in;
  float2* out;
  const float2* tw;   // inter-pass twiddle table of this pass kernel's schedule
  int64_t tw_count;   // entries of tw
  const float2* twc;  // row pass with combine: W_M^j for j < M
  int64_t total;      // points in the in and out buffers (bounds of every access)
  int64_t nvec;       // number of vectors
  int64_t ncols;      // column mode: points per row (N); unused in row mode
  int64_t m1;         // column mode: M1 of a split transform (1 = plain)
  int64_t m2;         // row pass with combine: M2 = M / M1
  float scale;        // multiplies every output point
  int nblocks;        // grid size (for the XCD-aware block remap)
  int remap;          // column mode: 1 = XCD-contiguous tile order (xcd_remap), 0 = launch order
};

// One compiled pass kernel: a length-L FFT with a fixed radix schedule,
// E points per thread, C vectors per workgroup, exchanged through LDS in Q
// rounds. `launch` enqueues it with the given exponent sign (-1 or +1). When
// t0 or t1 is not null the launch goes through hipExtLaunchKernel with them as
// its start and stop events, which then carry the kernel's own begin and end
// times (no marker packets between the kernel and its neighbours).
struct PassKernel {
  int L, E, T, C, Q, threads;
  int colmode;
  int combine;  // row pass with an M1 = C point combine across its rows (split column transform)
  int xrow;     // combine kernel whose last FFT stage runs across its rows (one LDS exchange fewer)
  int shuffle;  // an exchange runs in registers across the wave's lanes instead of through the LDS
  int wpe;  // minimum waves per SIMD the kernel was compiled for
  int nt;   // nontemporal input loads
  int npass;
  int radix[kMaxPasses];
  size_t lds_bytes;
  hipError_t (*launch)(const PassArgs&, int dir, hipStream_t, hipEvent_t t0, hipEvent_t t1);
  // Measurement variants (mode 1: loads, LDS exchanges and stores without
  // arithmetic; mode 2: loads and stores only); null where not compiled.
  hipError_t (*launch_probe)(const PassArgs&, int mode, hipStream_t, hipEvent_t t0, hipEvent_t t1);
};

// One compiled whole-grid kernel: the 2D transform of `rows` x `cols` grids,
// one workgroup per grid. Launch with PassArgs in/out/total, nvec = nblocks =
// number of grids, tw = the row schedule's table, twc = the column schedule's
// table, scale.
struct GridKernel {
  int rows, cols, threads;
  PassKernel row, col;  // shapes (radix schedules) of its row and column FFTs
  size_t lds_bytes;
  hipError_t (*launch)(const PassArgs&, int dir, hipStream_t);
};

// Default kernel for a length L in [2, 16384] (power of two); nullptr otherwise.
const PassKernel* find_pass_kernel(int L, bool colmode);
// Pass of length L with narrower tiles, for passes with few tiles (nullptr
// if none); `shuffle` prefers a variant with an exchange in registers across
// the wave's lanes where there is one.
const PassKernel* find_few_tiles_kernel(int L, bool colmode, bool shuffle = false);
// Row pass with an M1-point combine across M1 rows of length L (nullptr if
// none); `cross_row` prefers the variant whose last stage runs across the rows
// (rowx_kernel) where both exist, `wide` one with more than 32 points per
// thread among those.
const PassKernel* find_combine_kernel(int L, int m1, bool cross_row = true, bool wide = false);
// Column pass for the length-M2 columns of a split transform; `two_stage`
// prefers a two-stage radix schedule (one LDS exchange) where there is one
// (`nt`: its variant with nontemporal input loads), then `wide` the
// 64-points-per-thread variant where there is one (large grids).
const PassKernel* find_split_column_kernel(int L, bool wide = false, bool two_stage = false, bool nt = false);
// Whole-grid kernel for rows x cols grids (nullptr if none).
const GridKernel* find_grid_kernel(int rows, int cols);
// All compiled variants for a length (for the autotuner); returns the count.
int list_pass_kernels(int L, bool colmode, const PassKernel** out, int cap);

// Grid size for a pass over nvec vectors.
inline int pass_blocks(const PassKernel& k, int64_t nvec) { return (int)((nvec + k.C - 1) / k.C); }

// Number of twiddle entries of a schedule and the table contents: for pass
// p >= 1 with radix R and Ns = R_0 * ... * R_{p-1}, entry (r, k), r in
// [1, R), k in [0, Ns), holds exp(-2 pi i k r / (Ns R)) computed in FP64 and
// rounded once to FP32. Layout: passes in order, within a pass r-major.
size_t twiddle_count(const PassKernel& k);
void fill_twiddles(const PassKernel& k, float2* host_table);

// Record `detail` as this host thread's fft2d_last_error() and return `st`.
fft2d_status report_error(fft2d_status st, const std::string& detail);

// Scaled copy for 1x1 grids (and the trivial dimension): out[i] = in[i]*scale.
hipError_t launch_scale_copy(const float2* in, float2* out, int64_t n, float scale, hipStream_t s);

}  // namespace fft2d
