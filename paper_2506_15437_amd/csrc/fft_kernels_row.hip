// Row-pass kernel table (contiguous vectors).
#include "fft_pass.hpp"
#include "fft_tables.h"

namespace fft2d {

using namespace dev;

namespace {

// ------------------------------------------------------------ kernel table
// Row mode: vectors are contiguous; a few rows per workgroup for short rows.
using R2 = Cfg<2, 2, 128, 1, false, 2>;
using R4 = Cfg<4, 4, 128, 1, false, 4>;
using R8 = Cfg<8, 8, 64, 1, false, 8>;
using R16 = Cfg<16, 16, 64, 1, false, 16>;
using R32 = Cfg<32, 8, 32, 1, false, 8, 4>;
using R64 = Cfg<64, 8, 16, 1, false, 8, 8>;
using R128 = Cfg<128, 16, 16, 1, false, 16, 8>;
using R256 = Cfg<256, 16, 8, 1, false, 16, 16>;
using R512 = Cfg<512, 32, 8, 1, false, 32, 16>;
using R1024 = Cfg<1024, 32, 4, 1, false, 32, 32>;
using R2048 = Cfg<2048, 16, 2, 1, false, 16, 16, 8>;
using R4096 = Cfg<4096, 16, 1, 1, false, 16, 16, 16>;
using R8192 = Cfg<8192, 32, 1, 1, false, 32, 16, 16>;
using R16384 = Cfg<16384, 64, 1, 2, false, 64, 16, 16>;  // 256 threads, two workgroups per CU

// One row of 1024 per 64-thread workgroup, for row passes with few tiles
// (e.g. one 1024 x 1024 grid: 256 tiles of 4 rows, or 1024 of one).
using R1024F = Cfg<1024, 16, 1, 1, false, 16, 16, 4>;
const PassKernel kRowFewKernels[] = {
    describe<R1024F, kKindPass, 1, true, true>(),
    describe<R1024F, kKindWaveRow, 1, true, true>(),  // second exchange in registers (v_permlane16/32_swap)
};

const PassKernel kRowKernels[] = {
    describe<R2>(),   describe<R4>(),   describe<R8>(),    describe<R16>(),   describe<R32>(),
    describe<R64>(),  describe<R128>(), describe<R256>(),  describe<R512>(),  describe<R1024>(),
    describe<R2048>(), describe<R4096>(), describe<R8192>(), describe<R16384, kKindPass, 1, true, true>(),
};

}  // namespace

const PassKernel* row_few_kernel_table(int* count) {
  *count = (int)(sizeof(kRowFewKernels) / sizeof(kRowFewKernels[0]));
  return kRowFewKernels;
}

const PassKernel* row_kernel_table(int* count) {
  *count = (int)(sizeof(kRowKernels) / sizeof(kRowKernels[0]));
  return kRowKernels;
}

}  // namespace fft2d
