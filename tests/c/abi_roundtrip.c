/*
 * Plain C client of the fft2d C ABI (no C++, no Python): reads a rows x cols
 * complex64 grid from a file, runs the forward transform and the inverse of
 * its result through fft2d_plan / fft2d_exec on a HIP stream, writes both
 * results, and checks a few error paths of the ABI.
 *
 * usage: abi_roundtrip <rows> <cols> <input.bin> <forward.bin> <roundtrip.bin>
 * exit status 0 on success; the caller compares the outputs with its reference.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fft2d.h"

static int check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    return 1;
  }
  return 0;
}

static int check_fft(fft2d_status st, const char* what) {
  if (st != FFT2D_OK) {
    fprintf(stderr, "%s: %s (%s)\n", what, fft2d_status_string(st), fft2d_last_error());
    return 1;
  }
  return 0;
}

static int write_file(const char* path, const void* data, size_t bytes) {
  FILE* f = fopen(path, "wb");
  if (!f) return 1;
  const size_t n = fwrite(data, 1, bytes, f);
  fclose(f);
  return n != bytes;
}

int main(int argc, char** argv) {
  if (argc != 6) {
    fprintf(stderr, "usage: %s rows cols input forward roundtrip\n", argv[0]);
    return 2;
  }
  const int64_t rows = atoll(argv[1]), cols = atoll(argv[2]);
  const size_t bytes = (size_t)rows * (size_t)cols * 8u;
  float* host = (float*)malloc(bytes);
  if (!host) return 1;
  FILE* f = fopen(argv[3], "rb");
  if (!f || fread(host, 1, bytes, f) != bytes) {
    fprintf(stderr, "cannot read %s\n", argv[3]);
    return 1;
  }
  fclose(f);

  /* error paths: a size that is not a power of two, a NULL handle */
  fft2d_plan_t bad = NULL;
  if (fft2d_plan(&bad, 1, 3, 8) != FFT2D_ERR_INVALID_SIZE || bad != NULL) {
    fprintf(stderr, "expected FFT2D_ERR_INVALID_SIZE\n");
    return 1;
  }
  if (fft2d_exec(NULL, NULL, NULL, FFT2D_FORWARD, NULL) == FFT2D_OK) {
    fprintf(stderr, "expected an error for a NULL plan\n");
    return 1;
  }

  void *x = NULL, *y = NULL, *z = NULL;
  hipStream_t s;
  if (check_hip(hipStreamCreate(&s), "hipStreamCreate")) return 1;
  if (check_hip(hipMalloc(&x, bytes), "hipMalloc") || check_hip(hipMalloc(&y, bytes), "hipMalloc") ||
      check_hip(hipMalloc(&z, bytes), "hipMalloc"))
    return 1;
  if (check_hip(hipMemcpy(x, host, bytes, hipMemcpyHostToDevice), "upload")) return 1;

  fft2d_plan_t plan = NULL;
  if (check_fft(fft2d_plan(&plan, 1, rows, cols), "fft2d_plan")) return 1;
  if (check_fft(fft2d_exec(plan, x, y, FFT2D_FORWARD, s), "forward")) return 1;
  if (check_fft(fft2d_exec(plan, y, z, FFT2D_INVERSE, s), "inverse")) return 1;
  if (check_hip(hipStreamSynchronize(s), "synchronize")) return 1;

  if (check_hip(hipMemcpy(host, y, bytes, hipMemcpyDeviceToHost), "download") || write_file(argv[4], host, bytes))
    return 1;
  if (check_hip(hipMemcpy(host, z, bytes, hipMemcpyDeviceToHost), "download") || write_file(argv[5], host, bytes))
    return 1;

  char desc[512];
  if (fft2d_plan_describe(plan, desc, sizeof desc) == FFT2D_OK) printf("%s\n", desc);
  if (check_fft(fft2d_destroy(plan), "fft2d_destroy")) return 1;
  hipFree(x);
  hipFree(y);
  hipFree(z);
  hipStreamDestroy(s);
  free(host);
  printf("ok\n");
  return 0;
}
