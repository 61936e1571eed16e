// Batched path (placeholder until the persistent kernel lands).
#include "fft_batched.h"

namespace fft2d {

struct BatchedPlan {
  int64_t count = 0;
};

fft2d_status create_batched(int64_t, const int64_t*, const int64_t*, BatchedPlan** out, std::string* err) {
  *out = nullptr;
  *err = "batched plans are not available in this build";
  return FFT2D_ERR_WRONG_PLAN_KIND;
}

fft2d_status exec_batched(BatchedPlan*, const void* const*, void* const*, int, hipStream_t, std::string* err) {
  *err = "batched plans are not available in this build";
  return FFT2D_ERR_WRONG_PLAN_KIND;
}

void destroy_batched(BatchedPlan* bp) { delete bp; }

std::string describe_batched(const BatchedPlan*) { return "batched"; }

}  // namespace fft2d
