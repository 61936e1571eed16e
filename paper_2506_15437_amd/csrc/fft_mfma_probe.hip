// Measurement aid: the 16-point DFT as radix-2 butterflies on the vector ALU
// against the same DFT as a dense matrix product on the matrix cores (MFMA).
//
// The paper runs its butterflies either on the Tensix vector unit or as a
// matrix operation on its matrix (FPU) engine (Section 4); here the question
// is whether gfx950's FP32 matrix cores beat the vector butterflies for a
// small radix. Both kernels apply the same operator `reps` times to vectors
// held in registers, so the measurement is of arithmetic, not of memory:
//   x <- Pi F x, with F the unscaled 16-point forward DFT and Pi the
//   permutation that swaps the two base-4 digits of the point index
//   (point 4q + r goes to point q + 4r), and after every 8 applications
//   x <- x * 2^-16 (exact), so that the result (Pi F / 4)^reps x stays in range.
//
// Butterfly kernel: one 16-point vector per lane, dft<16> (4 radix-2 DIT
// steps, compile-time twiddles), Pi as a register renaming.
// Matrix kernel: the DFT as the real 32 x 32 matrix [[C, -S], [S, C]] times
// 16 vectors (32 real components each) per wave, as 2 x 8
// v_mfma_f32_16x16x4_f32 instructions (two 16-row output tiles, eight
// 4-deep K chunks). Lane l (q = l / 16, j = l % 16) holds points q + 4m
// (m = 0..3) of vector j as the B operand; the output tile registers r hold
// points 4q + r, which is the input layout of Pi F x, so the loop needs no
// data movement between applications. Each wave keeps 4 groups of 16
// vectors (64 vectors, like the butterfly kernel) in flight.
#include "fft2d.h"
#include "fft_pass.hpp"

#include <string>

namespace fft2d {
namespace {

using namespace dev;

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kProbeThreads = 256;

__device__ __forceinline__ float2 scl(float2 v, float s) { return make_float2(v.x * s, v.y * s); }

__global__ __launch_bounds__(kProbeThreads) void dft16_butterfly_kernel(const float2* __restrict__ in,
                                                                        float2* __restrict__ out, int64_t nvec,
                                                                        int reps) {
  const int64_t v = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
  if (v >= nvec) return;
  float2 x[16];
  static_for<0, 16>([&](auto I) { x[decltype(I)::value] = in[v * 16 + decltype(I)::value]; });
  for (int it = 0; it < reps; ++it) {
    dft<16, -1>(x);
    float2 y[16];
    static_for<0, 16>([&](auto I) {  // Pi: point 4q + r -> q + 4r
      constexpr int n = decltype(I)::value;
      y[(n >> 2) + 4 * (n & 3)] = x[n];
    });
    static_for<0, 16>([&](auto I) { x[decltype(I)::value] = y[decltype(I)::value]; });
    if ((it & 7) == 7) static_for<0, 16>([&](auto I) { x[decltype(I)::value] = scl(x[decltype(I)::value], 0x1p-16f); });
  }
  static_for<0, 16>([&](auto I) { out[v * 16 + decltype(I)::value] = x[decltype(I)::value]; });
}

__global__ __launch_bounds__(kProbeThreads) void dft16_mfma_kernel(const float2* __restrict__ in,
                                                                   float2* __restrict__ out, int64_t nvec,
                                                                   int reps) {
  constexpr int G = 4;  // groups of 16 vectors per wave
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4, j = lane & 15;
  const int64_t wave = ((int64_t)blockIdx.x * kProbeThreads + threadIdx.x) >> 6;
  const int64_t v0 = wave * 64;  // first vector of this wave
  if (v0 >= nvec) return;        // whole waves only (nvec is a multiple of 64)
  // A operand: W[16 t + i][4 c + k] with i = j, k = q, for output tile t and K chunk c
  float a[2][8];
  for (int t = 0; t < 2; ++t)
    for (int c = 0; c < 8; ++c) {
      const int o = j;               // output point
      const int n = (4 * c + q) & 15;  // input point
      const bool in_im = c >= 4;
      double sn = 0.0, cs = 0.0;
      sincospi(2.0 * (double)((o * n) & 15) / 16.0, &sn, &cs);
      const double s = -sn;  // F = cos + i s with s = -sin(2 pi o n / 16)
      double w;
      if (t == 0) w = in_im ? -s : cs;  // Yr = C Xr - S Xi
      else w = in_im ? cs : s;          // Yi = S Xr + C Xi
      a[t][c] = (float)w;
    }
  // B operand per group: b[g][c] = component 4c + q of vector j: c < 4 real part of
  // point q + 4c, c >= 4 imaginary part of point q + 4(c - 4)
  float b[G][8];
  for (int g = 0; g < G; ++g) {
    const int64_t v = v0 + 16 * g + j;
    for (int m = 0; m < 4; ++m) {
      const float2 p = in[v * 16 + q + 4 * m];
      b[g][m] = p.x;
      b[g][4 + m] = p.y;
    }
  }
  for (int it = 0; it < reps; ++it) {
    f4v d[G][2];
    for (int g = 0; g < G; ++g)
      for (int t = 0; t < 2; ++t) d[g][t] = f4v{0.f, 0.f, 0.f, 0.f};
    for (int c = 0; c < 8; ++c)
      for (int g = 0; g < G; ++g)
        for (int t = 0; t < 2; ++t) d[g][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t][c], b[g][c], d[g][t], 0, 0, 0);
    // output register r of tile 0 / 1 = real / imaginary part of point 4q + r, i.e. point q + 4r of Pi F x
    const float sc = ((it & 7) == 7) ? 0x1p-16f : 1.0f;
    for (int g = 0; g < G; ++g)
      for (int r = 0; r < 4; ++r) {
        b[g][r] = d[g][0][r] * sc;
        b[g][4 + r] = d[g][1][r] * sc;
      }
  }
  for (int g = 0; g < G; ++g) {
    const int64_t v = v0 + 16 * g + j;
    for (int m = 0; m < 4; ++m) out[v * 16 + q + 4 * m] = make_float2(b[g][m], b[g][4 + m]);
  }
}

}  // namespace
}  // namespace fft2d

using namespace fft2d;

extern "C" fft2d_status fft2d_probe_dft16(int method, const void* in, void* out, int64_t count, int reps,
                                          void* start_event, void* stop_event, void* stream) {
  if (method != FFT2D_DFT16_BUTTERFLY && method != FFT2D_DFT16_MFMA)
    return report_error(FFT2D_ERR_INVALID_DIRECTION, "method must be FFT2D_DFT16_BUTTERFLY or FFT2D_DFT16_MFMA");
  if (!in || !out) return report_error(FFT2D_ERR_NULL_POINTER, "input or output pointer is NULL");
  if ((start_event == nullptr) != (stop_event == nullptr))
    return report_error(FFT2D_ERR_NULL_POINTER, "give both timing events or neither");
  if (count < 64 || count % 64 != 0 || count > (int64_t(1) << 26) || reps < 8 || reps > 4096 || reps % 8 != 0)
    return report_error(FFT2D_ERR_INVALID_SIZE,
                        "count must be a multiple of 64 in [64, 2^26] and reps a multiple of 8 in [8, 4096]");
  if ((reinterpret_cast<uintptr_t>(in) & 7) || (reinterpret_cast<uintptr_t>(out) & 7))
    return report_error(FFT2D_ERR_MISALIGNED, "data pointers must be 8-byte aligned (complex64)");
  const uintptr_t a = reinterpret_cast<uintptr_t>(in), b = reinterpret_cast<uintptr_t>(out);
  const uintptr_t bytes = (uintptr_t)count * 128u;
  if (a != b && a < b + bytes && b < a + bytes)
    return report_error(FFT2D_ERR_OVERLAP, "input and output overlap without being identical");
  // butterflies: one vector per thread; matrix cores: 64 vectors per wave, 4 waves per block
  const bool bf = method == FFT2D_DFT16_BUTTERFLY;
  const unsigned grid = (unsigned)(bf ? count / kProbeThreads + (count % kProbeThreads != 0) : (count / 64 + 3) / 4);
  void (*k)(const float2*, float2*, int64_t, int) = bf ? dft16_butterfly_kernel : dft16_mfma_kernel;
  const float2* pin = static_cast<const float2*>(in);
  float2* pout = static_cast<float2*>(out);
  int64_t n = count;
  void* args[] = {&pin, &pout, &n, &reps};
  const hipError_t e = hipExtLaunchKernel(reinterpret_cast<const void*>(k), dim3(grid), dim3(kProbeThreads), args,
                                          0, (hipStream_t)stream, (hipEvent_t)start_event, (hipEvent_t)stop_event,
                                          0);
  if (e != hipSuccess)
    return report_error(FFT2D_ERR_HIP, std::string("probe kernel launch: ") + hipGetErrorName(e));
  return FFT2D_OK;
}
