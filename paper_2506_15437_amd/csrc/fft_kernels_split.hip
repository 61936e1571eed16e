// Kernel tables of split column transforms: row passes with an M1-point combine and the
// column passes of length rows/M1. The kernels of the benchmarked grids (4096^2,
// 8192^2, 16384 x 2048, 8 x 2048^2) also carry their measurement variants
// (describe's PROBE flag).
#include "fft_pass.hpp"
#include "fft_tables.h"

namespace fft2d {

using namespace dev;

namespace {

// Row passes with an M1-point combine (split column transforms): M1 rows of
// length L per workgroup, 128 KiB of data, 512 threads, 68 KiB of LDS (and
// one 256 KiB variant of 1024 threads for L = 8192).
using RC8192x2 = Cfg<8192, 32, 2, 2, false, 16, 16, 32>;
using RC8192x4 = Cfg<8192, 32, 4, 2, false, 16, 16, 32>;
using RC16384x2 = Cfg<16384, 32, 2, 2, false, 16, 16, 16, 4>;
using RC4096x4 = Cfg<4096, 32, 4, 2, false, 16, 16, 16>;
using RC2048x8 = Cfg<2048, 32, 8, 2, false, 16, 16, 8>;
using RC1024x16 = Cfg<1024, 32, 16, 2, false, 16, 16, 4>;

// Column passes of split transforms: 16 columns (128-byte row segments).
using S512 = Cfg<512, 32, 16, 2, true, 16, 32>;
using S1024 = Cfg<1024, 32, 16, 2, true, 16, 16, 4>;
using S2048 = Cfg<2048, 32, 16, 2, true, 16, 16, 8>;
using S4096 = Cfg<4096, 32, 8, 2, true, 16, 16, 16>;

// The same with the row FFT's last stage across the M1 rows (rowx_kernel): the
// last radix times M1 is the points per thread, and the combine DFT runs in
// registers on that stage's outputs, so there is no separate combine exchange.
using RX8192x4 = Cfg<8192, 32, 4, 2, false, 32, 32, 8>;
using RX16384x2 = Cfg<16384, 32, 2, 2, false, 32, 32, 16>;
using RX4096x4 = Cfg<4096, 32, 4, 2, false, 32, 16, 8>;
using RX2048x8 = Cfg<2048, 32, 8, 2, false, 32, 16, 4>;
using RX1024x16 = Cfg<1024, 32, 16, 2, false, 32, 16, 2>;
// 64 points per thread (256 threads, 64 loads in flight per thread) for grids
// with few tiles.
using RX4096x4W = Cfg<4096, 64, 4, 2, false, 64, 4, 16>;

const PassKernel kCombineKernels[] = {
    describe<RC8192x2, kKindCombine, 4>(), describe<RC8192x4, kKindCombine, 1, true, true>(),
    describe<RC16384x2, kKindCombine, 1>(),
    describe<RC4096x4, kKindCombine, 4, true, true>(),
    describe<RC2048x8, kKindCombine, 4, true, true>(),
    describe<RC1024x16, kKindCombine, 4>(),
    describe<RX8192x4, kKindCrossRow, 1, true, true>(), describe<RX16384x2, kKindCrossRow, 1>(),
    describe<RX4096x4, kKindCrossRow, 4, true, true>(), describe<RX2048x8, kKindCrossRow, 4, true, true>(),
    describe<RX1024x16, kKindCrossRow, 4>(), describe<RX4096x4W, kKindCrossRow, 1, true, true>(),
};
const PassKernel kSplitColKernels[] = {
    describe<S512>(), describe<S1024, kKindPass, 1, false, true>(), describe<S2048>(), describe<S4096>(),
};
// Column passes with 64 points per thread (512 threads) for split transforms
// whose data come from HBM rather than the MALL (large grids): more loads in
// flight per thread, fewer waves.
using S2048W = Cfg<2048, 64, 16, 2, true, 16, 16, 8>;
using S4096W = Cfg<4096, 64, 8, 4, true, 16, 16, 16>;
using S8192W = Cfg<8192, 64, 4, 2, true, 16, 16, 32>;
const PassKernel kSplitColWideKernels[] = {
    describe<S2048W, kKindPass, 1, false, true>(), describe<S4096W>(), describe<S8192W>(),
};
// Two-stage schedules (one LDS exchange): radix 32 x 32 for 1024-point columns
// (32 points per thread), radix 64 x 32 for 2048-point columns (64 points per
// thread).
using S1024B = Cfg<1024, 32, 16, 2, true, 32, 32>;
using S2048B = Cfg<2048, 64, 16, 2, true, 64, 32>;
const PassKernel kSplitColTwoStageKernels[] = {
    describe<S1024B, kKindPass, 1, false, true>(), describe<S2048B, kKindPass, 1, false, true>(),
};
// The same with nontemporal input loads, for grids larger than the MALL (the
// column pass then reads the row pass's output from HBM).
const PassKernel kSplitColTwoStageNtKernels[] = {
    describe<S1024B, kKindPass, 1, true, true>(), describe<S2048B, kKindPass, 1, true, true>(),
};

}  // namespace

const PassKernel* combine_kernel_table(int* count) {
  *count = (int)(sizeof(kCombineKernels) / sizeof(kCombineKernels[0]));
  return kCombineKernels;
}

const PassKernel* split_col_kernel_table(int* count) {
  *count = (int)(sizeof(kSplitColKernels) / sizeof(kSplitColKernels[0]));
  return kSplitColKernels;
}

const PassKernel* split_col_two_stage_kernel_table(int* count, bool nt) {
  if (nt) {
    *count = (int)(sizeof(kSplitColTwoStageNtKernels) / sizeof(kSplitColTwoStageNtKernels[0]));
    return kSplitColTwoStageNtKernels;
  }
  *count = (int)(sizeof(kSplitColTwoStageKernels) / sizeof(kSplitColTwoStageKernels[0]));
  return kSplitColTwoStageKernels;
}

const PassKernel* split_col_wide_kernel_table(int* count) {
  *count = (int)(sizeof(kSplitColWideKernels) / sizeof(kSplitColWideKernels[0]));
  return kSplitColWideKernels;
}

}  // namespace fft2d
