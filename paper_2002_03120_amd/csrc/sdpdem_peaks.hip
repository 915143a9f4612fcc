// sdpdem_peaks.hip -- measurement helpers for the benchmark: the vector-ALU
// issue rate of plain (unpacked) FP32 and FP64 fused multiply-adds, and a
// device-to-device stream copy, each timed with HIP events on the caller's
// stream.  Not part of the particle method: the benchmark divides the
// kernels' measured rates by these.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kChains = 8;  // independent FMA chains per thread

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}

template <class T>
__global__ __launch_bounds__(256) void k_fma(T* out, int iters, T b, T c) {
  T a[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = (T)(threadIdx.x + k);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = fma_t(a[k], b, c);
  }
  T s = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += a[k];
  if (s == (T)-1.2345) out[blockIdx.x] = s;  // keep the chains live
}

__global__ __launch_bounds__(256) void k_copy(const uint4* __restrict__ src,
                                              uint4* __restrict__ dst, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] = src[i];
}

template <class F>
float timed(hipStream_t st, F launch) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return -1.f;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return -1.f;
  }
  launch();  // warm-up
  (void)hipEventRecord(a, st);
  launch();
  (void)hipEventRecord(b, st);
  float ms = -1.f;
  if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess)
    ms = -1.f;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms;
}

}  // namespace

extern "C" {

// FMA lane-operations per second of one launch of `blocks` x 256 threads,
// each running 8 chains of `iters` dependent FMAs (fp64 != 0: double);
// out: a device buffer of `blocks` elements of the type (never written in
// practice).  Returns -1 on a HIP error.
double sdpdem_peak_fma(int fp64, int blocks, int iters, void* out, void* hip_stream) {
  hipStream_t st = (hipStream_t)hip_stream;
  float ms;
  if (fp64)
    ms = timed(st, [&] {
      k_fma<double><<<blocks, 256, 0, st>>>((double*)out, iters, 0.999999, 1e-7);
    });
  else
    ms = timed(st, [&] {
      k_fma<float><<<blocks, 256, 0, st>>>((float*)out, iters, 0.999999f, 1e-7f);
    });
  if (ms <= 0.f || hipGetLastError() != hipSuccess) return -1.0;
  return (double)blocks * 256.0 * kChains * iters / (ms * 1e-3);
}

// Bytes moved per second (read + write) copying `bytes` (a multiple of 16)
// from src to dst, both device buffers.  Returns -1 on a HIP error.
double sdpdem_peak_copy(const void* src, void* dst, size_t bytes, void* hip_stream) {
  hipStream_t st = (hipStream_t)hip_stream;
  const size_t n = bytes / 16;
  const float ms = timed(st, [&] {
    k_copy<<<256 * 32, 256, 0, st>>>((const uint4*)src, (uint4*)dst, n);
  });
  if (ms <= 0.f || hipGetLastError() != hipSuccess) return -1.0;
  return 2.0 * (double)(n * 16) / (ms * 1e-3);
}

}  // extern "C"
