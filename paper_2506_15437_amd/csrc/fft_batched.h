// Internal interface of the batched (many shapes, one persistent launch) path.
#pragma once

#include "fft2d.h"

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>

namespace fft2d {

struct BatchedPlan;

fft2d_status create_batched(int64_t count, const int64_t* rows, const int64_t* cols, BatchedPlan** out,
                            std::string* err);
fft2d_status exec_batched(BatchedPlan* bp, const void* const* in, void* const* out, int direction, hipStream_t s,
                          std::string* err);
void destroy_batched(BatchedPlan* bp);
std::string describe_batched(const BatchedPlan* bp);

}  // namespace fft2d
