// Whole-grid kernel table: the 2D transform of a small grid in one launch,
// one workgroup per grid, every point read and written once (instead of one
// launch and one HBM round trip per pass).
#include "fft_pass.hpp"
#include "fft_tables.h"

namespace fft2d {

using namespace dev;

namespace {

// A row tile of KR::C rows passes through the LDS at a time and the whole
// grid sits in registers for the column FFTs (M N / threads points per
// thread). The radix schedules equal the plain row and column passes' of the
// same lengths, so the plan's twiddle tables serve both. 512 threads for grids
// with both sides >= 64; grids with a side of 32 use as many threads as their
// 32-point vectors allow (128 or 256 for up to 4096 points, 512 for 8192).
using GR64 = Cfg<64, 8, 64, 1, false, 8, 8>;
using GR128 = Cfg<128, 16, 64, 1, false, 16, 8>;
using GR256 = Cfg<256, 16, 32, 1, false, 16, 16>;
using GC64 = Cfg<64, 8, 64, 1, true, 8, 8>;
using GC128 = Cfg<128, 16, 64, 1, true, 16, 8>;
using GC256 = Cfg<256, 16, 32, 1, true, 16, 16>;
// Shapes with a side of 32: GR<L>_<C> / GC<L>_<C> run length-L FFTs on C rows /
// columns per tile.
using GR32_32 = Cfg<32, 8, 32, 1, false, 8, 4>;     // 128 threads
using GR32_64 = Cfg<32, 8, 64, 1, false, 8, 4>;     // 256 threads
using GR32_128 = Cfg<32, 8, 128, 1, false, 8, 4>;   // 512 threads
using GR64_32 = Cfg<64, 8, 32, 1, false, 8, 8>;     // 256 threads
using GR128_32 = Cfg<128, 16, 32, 1, false, 16, 8>; // 256 threads
using GC32_32 = Cfg<32, 8, 32, 1, true, 8, 4>;
using GC32_64 = Cfg<32, 8, 64, 1, true, 8, 4>;
using GC32_128 = Cfg<32, 8, 128, 1, true, 8, 4>;
using GC64_32 = Cfg<64, 8, 32, 1, true, 8, 8>;
using GC128_32 = Cfg<128, 16, 32, 1, true, 16, 8>;

template <class KR, class KC>
hipError_t launch_grid(const PassArgs& a, int dir, hipStream_t s) {
  if (dir < 0) hipLaunchKernelGGL((grid_kernel<KR, KC, -1>), dim3(a.nblocks), dim3(KR::THREADS), 0, s, a);
  else hipLaunchKernelGGL((grid_kernel<KR, KC, +1>), dim3(a.nblocks), dim3(KR::THREADS), 0, s, a);
  return hipGetLastError();
}

template <class KR, class KC>
constexpr GridKernel describe_grid() {
  GridKernel g{};
  g.rows = KC::L;
  g.cols = KR::L;
  g.threads = KR::THREADS;
  g.row = meta<KR>();
  g.col = meta<KC>();
  g.lds_bytes = (size_t)grid_lds_elems<KR, KC>() * 8;
  g.launch = &launch_grid<KR, KC>;
  return g;
}

// rows x cols: 64 x 64, 64 x 128, 128 x 64, 128 x 128, 64 x 256, 256 x 64;
// 32 x 32, 32 x 64, 64 x 32, 32 x 128, 128 x 32, 32 x 256, 256 x 32
const GridKernel kGridKernels[] = {
    describe_grid<GR64, GC64>(),       describe_grid<GR128, GC64>(),     describe_grid<GR64, GC128>(),
    describe_grid<GR128, GC128>(),     describe_grid<GR256, GC64>(),     describe_grid<GR64, GC256>(),
    describe_grid<GR32_32, GC32_32>(), describe_grid<GR64_32, GC32_64>(), describe_grid<GR32_64, GC64_32>(),
    describe_grid<GR128_32, GC32_64>(), describe_grid<GR32_64, GC128_32>(), describe_grid<GR256, GC32_128>(),
    describe_grid<GR32_128, GC256>(),
};

}  // namespace

const GridKernel* grid_kernel_table(int* count) {
  *count = (int)(sizeof(kGridKernels) / sizeof(kGridKernels[0]));
  return kGridKernels;
}

}  // namespace fft2d
