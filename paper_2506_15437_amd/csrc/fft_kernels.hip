// Kernel lookup over the compiled pass tables, and the scaled copy kernel.
#include "fft_pass.hpp"
#include "fft_tables.h"

namespace fft2d {
namespace {

using namespace dev;

__global__ void scale_copy_kernel(const float2* __restrict__ in, float2* __restrict__ out, int64_t n, float sc) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    const float2 v = in[i];
    out[i] = make_float2(v.x * sc, v.y * sc);
  }
}

}  // namespace

const PassKernel* find_pass_kernel(int L, bool colmode) {
  int n = 0;
  const PassKernel* tab = colmode ? col_kernel_table(&n) : row_kernel_table(&n);
  for (int i = 0; i < n; ++i)
    if (tab[i].L == L) return &tab[i];
  return nullptr;
}

const PassKernel* find_few_tiles_kernel(int L, bool colmode, bool shuffle) {
  int n = 0;
  const PassKernel* tab = colmode ? col_few_kernel_table(&n) : row_few_kernel_table(&n);
  const PassKernel* any = nullptr;
  for (int i = 0; i < n; ++i) {
    if (tab[i].L != L) continue;
    if ((tab[i].shuffle != 0) == shuffle) return &tab[i];
    if (!any) any = &tab[i];
  }
  return any;
}

const PassKernel* find_combine_kernel(int L, int m1, bool cross_row, bool wide) {
  int n = 0;
  const PassKernel* tab = combine_kernel_table(&n);
  const PassKernel* any = nullptr;
  const PassKernel* kind = nullptr;
  for (int i = 0; i < n; ++i) {
    if (tab[i].L != L || tab[i].C != m1) continue;
    if ((tab[i].xrow != 0) == cross_row) {
      if ((tab[i].E > 32) == wide) return &tab[i];
      if (!kind) kind = &tab[i];
    }
    if (!any) any = &tab[i];
  }
  return kind ? kind : any;
}

const PassKernel* find_split_column_kernel(int L, bool wide, bool two_stage, bool nt) {
  int n = 0;
  if (two_stage) {
    const PassKernel* tab = split_col_two_stage_kernel_table(&n, nt);
    for (int i = 0; i < n; ++i)
      if (tab[i].L == L && (wide || tab[i].E <= 32)) return &tab[i];
  }
  if (wide) {
    const PassKernel* tab = split_col_wide_kernel_table(&n);
    for (int i = 0; i < n; ++i)
      if (tab[i].L == L) return &tab[i];
  }
  const PassKernel* tab = split_col_kernel_table(&n);
  for (int i = 0; i < n; ++i)
    if (tab[i].L == L) return &tab[i];
  return nullptr;
}

const GridKernel* find_grid_kernel(int rows, int cols) {
  int n = 0;
  const GridKernel* tab = grid_kernel_table(&n);
  for (int i = 0; i < n; ++i)
    if (tab[i].rows == rows && tab[i].cols == cols) return &tab[i];
  return nullptr;
}

int list_pass_kernels(int L, bool colmode, const PassKernel** out, int cap) {
  const PassKernel* k = find_pass_kernel(L, colmode);
  if (!k) return 0;
  if (cap > 0) out[0] = k;
  return 1;
}

size_t twiddle_count(const PassKernel& k) {
  size_t n = 0, ns = 1;
  for (int p = 0; p < k.npass; ++p) {
    if (p > 0) n += ns * (size_t)(k.radix[p] - 1);
    ns *= (size_t)k.radix[p];
  }
  return n;
}

hipError_t launch_scale_copy(const float2* in, float2* out, int64_t n, float scale, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(scale_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, out, n, scale);
  return hipGetLastError();
}

}  // namespace fft2d
