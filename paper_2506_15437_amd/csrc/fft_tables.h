// Tables of compiled pass kernels (defined in the fft_kernels_*.hip units).
#pragma once

#include "fft_internal.h"

namespace fft2d {

const PassKernel* row_kernel_table(int* count);
const PassKernel* row_few_kernel_table(int* count);
const PassKernel* col_kernel_table(int* count);
const PassKernel* col_few_kernel_table(int* count);
const PassKernel* combine_kernel_table(int* count);
const PassKernel* split_col_kernel_table(int* count);
const PassKernel* split_col_wide_kernel_table(int* count);
const PassKernel* split_col_two_stage_kernel_table(int* count, bool nt);
const GridKernel* grid_kernel_table(int* count);

}  // namespace fft2d
