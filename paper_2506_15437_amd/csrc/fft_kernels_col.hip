// Column-pass kernel table (strided vectors).
#include "fft_pass.hpp"
#include "fft_tables.h"

namespace fft2d {

using namespace dev;

namespace {

// Column mode: C columns per workgroup (C*8-byte row segments), the LDS
// exchange split into Q rounds where C*L points would not fit 160 KiB.
using C2 = Cfg<2, 2, 256, 1, true, 2>;
using C4 = Cfg<4, 4, 256, 1, true, 4>;
using C8 = Cfg<8, 8, 128, 1, true, 8>;
using C16 = Cfg<16, 16, 128, 1, true, 16>;
using C32 = Cfg<32, 8, 64, 1, true, 8, 4>;
using C64 = Cfg<64, 8, 32, 1, true, 8, 8>;
using C128 = Cfg<128, 16, 32, 1, true, 16, 8>;
using C256 = Cfg<256, 16, 16, 1, true, 16, 16>;
using C512 = Cfg<512, 32, 16, 1, true, 32, 16>;
using C1024 = Cfg<1024, 32, 16, 1, true, 32, 32>;
using C2048 = Cfg<2048, 16, 8, 1, true, 16, 16, 8>;
using C4096 = Cfg<4096, 32, 8, 2, true, 16, 16, 16>;
using C8192 = Cfg<8192, 32, 4, 2, true, 16, 16, 32>;
using C16384 = Cfg<16384, 32, 2, 2, true, 16, 16, 16, 4>;

// Narrower tiles for column passes that would otherwise leave most CUs idle
// (fewer tiles than CUs, e.g. one 1024 x 1024 grid: 64 tiles of 16 columns).
using C512F = Cfg<512, 16, 8, 1, true, 16, 16, 2>;     // 256 threads, 8 columns
using C1024F = Cfg<1024, 16, 4, 1, true, 16, 16, 4>;   // 256 threads, 4 columns
using C2048F = Cfg<2048, 16, 4, 1, true, 16, 16, 8>;   // 512 threads, 4 columns
const PassKernel kColFewKernels[] = {
    describe<C512F>(), describe<C1024F, kKindPass, 1, false, true>(), describe<C2048F>(),
};

const PassKernel kColKernels[] = {
    describe<C2>(),   describe<C4>(),   describe<C8>(),    describe<C16>(),   describe<C32>(),
    describe<C64>(),  describe<C128>(), describe<C256, kKindPass, 1, false, true>(),  describe<C512>(),  describe<C1024>(),
    describe<C2048>(), describe<C4096>(), describe<C8192>(), describe<C16384>(),
};

}  // namespace

const PassKernel* col_few_kernel_table(int* count) {
  *count = (int)(sizeof(kColFewKernels) / sizeof(kColFewKernels[0]));
  return kColFewKernels;
}

const PassKernel* col_kernel_table(int* count) {
  *count = (int)(sizeof(kColKernels) / sizeof(kColKernels[0]));
  return kColKernels;
}

}  // namespace fft2d
