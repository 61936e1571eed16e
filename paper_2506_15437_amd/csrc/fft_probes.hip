// Measurement probes behind the design of the pass kernels (no transform
// uses them): copies with column-tile access patterns of several row-segment
// widths, and the LDS read and write bandwidth of one workgroup per CU.
#include "fft_internal.h"

#include <hip/hip_ext.h>

#include <cstdint>
#include <string>

namespace fft2d {
namespace {

typedef float f2v __attribute__((ext_vector_type(2)));

constexpr int kProbeCopyThreads = 512;

// Column-tile copy of a rows x cols complex64 grid: tile (residue k1 < M1, row
// block hb, column block cb) holds rows k1 + M1 (hb H + m), m < H, and columns
// cb CW ... cb CW + CW - 1 (row segments of CW * 8 bytes); 512 threads, lane
// layout of the column pass (columns fastest), each thread H CW / 512 points.
// The host checks rows % (M1 H) == 0 and cols % CW == 0, so every index lies
// inside the grid.
template <int CW, int H, bool NT>
__global__ __launch_bounds__(kProbeCopyThreads) void tile_copy_kernel(const float2* __restrict__ in,
                                                                     float2* __restrict__ out, int64_t cols,
                                                                     int64_t m1) {
  constexpr int TG = kProbeCopyThreads / CW;
  constexpr int E = H * CW / kProbeCopyThreads;
  const int t = threadIdx.x, c = t % CW, tt = t / CW;
  const int64_t ntc = cols / CW;
  const int64_t kh = blockIdx.x / ntc, cb = blockIdx.x % ntc;
  const int64_t hb = kh / m1, k1 = kh % m1;
  auto idx = [&](int64_t m) { return (k1 + m1 * (hb * H + m)) * cols + cb * CW + c; };
  f2v d[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const f2v* p = reinterpret_cast<const f2v*>(in + idx(tt + TG * j));
    d[j] = NT ? __builtin_nontemporal_load(p) : *p;
  }
#pragma unroll
  for (int j = 0; j < E; ++j) *reinterpret_cast<f2v*>(out + idx(tt + TG * j)) = d[j];
}

// LDS bandwidth: every thread of a 1024-thread workgroup reads (or writes)
// kLdsIters times T (4, 8 or 16 bytes) at lane-consecutive addresses inside a
// 128 KiB array; the result (sink) keeps the reads live.
constexpr int kLdsThreads = 1024, kLdsIters = 4096, kLdsBytes = 128 * 1024;

template <class T, bool WRITE>
__global__ __launch_bounds__(kLdsThreads) void lds_bandwidth_kernel(float* sink) {
  __shared__ __attribute__((aligned(16))) char lds[kLdsBytes];
  T* l = reinterpret_cast<T*>(lds);
  constexpr int NE = kLdsBytes / (int)sizeof(T);
  const int t = threadIdx.x;
  for (int i = t; i < NE; i += kLdsThreads) l[i] = T{};
  __syncthreads();
  float a = 0.f;
#pragma unroll 16
  for (int it = 0; it < kLdsIters; ++it) {
    const int i = (t + it * 64) & (NE - 1);
    if constexpr (WRITE) {
      T v{};
      reinterpret_cast<float*>(&v)[0] = (float)it;
      l[i] = v;
    } else {
      const T v = l[i];
#pragma unroll
      for (int q = 0; q < (int)(sizeof(T) / 4); ++q) a += reinterpret_cast<const float*>(&v)[q];
    }
  }
  __syncthreads();
  if constexpr (WRITE) a = reinterpret_cast<float*>(l)[t];
  sink[(int64_t)blockIdx.x * kLdsThreads + t] = a;
}

hipError_t launch(const void* k, unsigned grid, unsigned threads, void** args, void* t0, void* t1, void* s) {
  return hipExtLaunchKernel(k, dim3(grid), dim3(threads), args, 0, (hipStream_t)s, (hipEvent_t)t0,
                            (hipEvent_t)t1, 0);
}

}  // namespace
}  // namespace fft2d

using namespace fft2d;

extern "C" fft2d_status fft2d_probe_tile_copy(const void* in, void* out, int64_t rows, int64_t cols,
                                              int tile_cols, int residues, int nontemporal, void* start_event,
                                              void* stop_event, void* stream) {
  if (!in || !out) return report_error(FFT2D_ERR_NULL_POINTER, "input or output pointer is NULL");
  if ((start_event == nullptr) != (stop_event == nullptr))
    return report_error(FFT2D_ERR_NULL_POINTER, "give both timing events or neither");
  const int h = tile_cols == 16 ? 2048 : tile_cols == 32 ? 1024 : tile_cols == 64 ? 512 : 0;
  if (h == 0) return report_error(FFT2D_ERR_INVALID_SIZE, "tile_cols must be 16, 32 or 64");
  if (residues < 1 || rows < 1 || cols < 1 || rows % ((int64_t)residues * h) != 0 || cols % tile_cols != 0 ||
      rows * cols > (int64_t(1) << 28))
    return report_error(FFT2D_ERR_INVALID_SIZE,
                        "rows must be a multiple of residues * tile rows (2048, 1024, 512 for 16, 32, 64 columns), "
                        "cols of tile_cols, and rows * cols at most 2^28");
  if ((reinterpret_cast<uintptr_t>(in) & 7) || (reinterpret_cast<uintptr_t>(out) & 7))
    return report_error(FFT2D_ERR_MISALIGNED, "data pointers must be 8-byte aligned (complex64)");
  const uintptr_t a = reinterpret_cast<uintptr_t>(in), b = reinterpret_cast<uintptr_t>(out);
  const uintptr_t bytes = (uintptr_t)(rows * cols) * 8u;
  if (a < b + bytes && b < a + bytes) return report_error(FFT2D_ERR_OVERLAP, "input and output overlap");
  const void* k = nullptr;
  const bool nt = nontemporal != 0;
  if (tile_cols == 16) k = nt ? (const void*)tile_copy_kernel<16, 2048, true> : (const void*)tile_copy_kernel<16, 2048, false>;
  else if (tile_cols == 32) k = nt ? (const void*)tile_copy_kernel<32, 1024, true> : (const void*)tile_copy_kernel<32, 1024, false>;
  else k = nt ? (const void*)tile_copy_kernel<64, 512, true> : (const void*)tile_copy_kernel<64, 512, false>;
  const float2* pin = static_cast<const float2*>(in);
  float2* pout = static_cast<float2*>(out);
  int64_t c = cols, m1 = residues;
  void* args[] = {&pin, &pout, &c, &m1};
  const unsigned grid = (unsigned)((rows / h) * (cols / tile_cols));
  const hipError_t e = launch(k, grid, kProbeCopyThreads, args, start_event, stop_event, stream);
  if (e != hipSuccess) return report_error(FFT2D_ERR_HIP, std::string("probe launch: ") + hipGetErrorName(e));
  return FFT2D_OK;
}

extern "C" fft2d_status fft2d_probe_lds(int width_bytes, int write, void* sink, int64_t sink_floats, int64_t* bytes,
                                        void* start_event, void* stop_event, void* stream) {
  if (!sink || !bytes) return report_error(FFT2D_ERR_NULL_POINTER, "sink or bytes is NULL");
  if ((start_event == nullptr) != (stop_event == nullptr))
    return report_error(FFT2D_ERR_NULL_POINTER, "give both timing events or neither");
  if (width_bytes != 4 && width_bytes != 8 && width_bytes != 16)
    return report_error(FFT2D_ERR_INVALID_SIZE, "width_bytes must be 4, 8 or 16");
  if (reinterpret_cast<uintptr_t>(sink) & 3) return report_error(FFT2D_ERR_MISALIGNED, "sink must be 4-byte aligned");
  const void* k = nullptr;
  if (width_bytes == 4) k = write ? (const void*)lds_bandwidth_kernel<float, true> : (const void*)lds_bandwidth_kernel<float, false>;
  else if (width_bytes == 8) k = write ? (const void*)lds_bandwidth_kernel<float2, true> : (const void*)lds_bandwidth_kernel<float2, false>;
  else k = write ? (const void*)lds_bandwidth_kernel<float4, true> : (const void*)lds_bandwidth_kernel<float4, false>;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return report_error(FFT2D_ERR_HIP, std::string("device query: ") + hipGetErrorName(e));
  if (sink_floats < (int64_t)cus * kLdsThreads)
    return report_error(FFT2D_ERR_INVALID_SIZE, "sink must hold (compute units) x 1024 floats");
  float* s = static_cast<float*>(sink);
  void* args[] = {&s};
  e = launch(k, (unsigned)cus, kLdsThreads, args, start_event, stop_event, stream);
  if (e != hipSuccess) return report_error(FFT2D_ERR_HIP, std::string("probe launch: ") + hipGetErrorName(e));
  *bytes = (int64_t)cus * kLdsThreads * kLdsIters * width_bytes;
  return FFT2D_OK;
}
