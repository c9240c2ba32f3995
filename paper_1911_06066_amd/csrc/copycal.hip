// Copy kernels of known size for calibrating the HBM byte counters
// (FETCH_SIZE, WRITE_SIZE): dst[i] = src[i] over n elements of 8 or 4 bytes,
// read and written with the same coalesced per-lane widths the solver's
// staging and vector passes use.  Built into its own small library
// (libstmcal.so), not part of the solver's interface.
#include <hip/hip_runtime.h>
#include <stddef.h>

template <typename T>
__global__ __launch_bounds__(256) void copy_kernel(const T* __restrict__ src, T* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// Copies `bytes` bytes (a multiple of width) from src to dst on stream with
// width-byte elements (8 or 4).  Returns a hipError_t value.
extern "C" int stmcal_copy(const void* src, void* dst, size_t bytes, int width, void* stream) {
  if (width != 8 && width != 4) return (int)hipErrorInvalidValue;
  if (bytes % (size_t)width) return (int)hipErrorInvalidValue;
  const size_t n = bytes / (size_t)width;
  const int blocks = 256 * 16;  // 16 workgroups per CU, grid-stride over the rest
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (width == 8)
    hipLaunchKernelGGL(copy_kernel<double>, dim3(blocks), dim3(256), 0, st, static_cast<const double*>(src),
                       static_cast<double*>(dst), n);
  else
    hipLaunchKernelGGL(copy_kernel<float>, dim3(blocks), dim3(256), 0, st, static_cast<const float*>(src),
                       static_cast<float*>(dst), n);
  return (int)hipGetLastError();
}
