// Measurement aids: achievable HBM copy bandwidth and FP32/FP64 arithmetic peaks of
// the device the library runs on, so kernel fractions can be quoted against measured
// ceilings as well as the published ones.  No counterpart in the paper.
#include <math.h>

#include <algorithm>
#include <vector>

#include "sdl_internal.h"

namespace sdl {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kProbeThreads = 256;
constexpr int kChains = 16;

__global__ void __launch_bounds__(kProbeThreads) copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                             size_t n4) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n4; e += (size_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

// kChains independent FMA chains per thread; the result is written only if it takes
// a value it never reaches, which keeps the arithmetic alive.
template <typename T>
__global__ void __launch_bounds__(kProbeThreads) fma_kernel(T* sink, int iters) {
  T a[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = (T)(threadIdx.x + k) * (T)1e-3;
  const T b = (T)0.99999, c = (T)1e-6;
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = fma(a[k], b, c);
  }
  T s = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += a[k];
  if (s == (T)-1) sink[0] = s;
}

template <int KIND>  // 0: 16x16x4 FP32, 1: 4x4x1 (16 blocks) FP32
__global__ void __launch_bounds__(kProbeThreads) mfma_kernel(float* sink, int iters) {
  f32x4 acc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
  const float a = 1e-3f * (threadIdx.x % 64), b = 1e-3f;
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (KIND == 0)
        acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[k], 0, 0, 0);
      else
        acc[k] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, acc[k], 0, 0, 0);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 4; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  if (s == -1.f) sink[0] = s;
}

// BF16 matrix-core chains, FP32 accumulation.  KIND 0: 4x4x4 (16 blocks), 1: 16x16x16,
// 2: 16x16x32.  Operands are small nonzero bfloat16 values.
template <int KIND>
__global__ void __launch_bounds__(kProbeThreads) mfma_bf16_kernel(float* sink, int iters) {
  f32x4 acc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
  const short h = (short)(0x3A80 + (threadIdx.x % 64));  // about 1e-3
  const s16x4 a4 = {h, h, h, h};
  bf16x8 a8;
#pragma unroll
  for (int k = 0; k < 8; ++k) a8[k] = (__bf16)(1e-3f * (float)(threadIdx.x % 64 + k));
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (KIND == 0)
        acc[k] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(a4, a4, acc[k], 0, 0, 0);
      else if (KIND == 1)
        acc[k] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a4, a4, acc[k], 0, 0, 0);
      else
        acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a8, a8, acc[k], 0, 0, 0);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 4; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  if (s == -1.f) sink[0] = s;
}

int device_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
  return n;
}

// Best time (ms) of reps launches of f, each bracketed by events on st; one warm-up launch.
template <class F>
hipError_t best_ms(F f, int reps, hipStream_t st, double* out) {
  hipEvent_t e0, e1;
  hipError_t err = hipEventCreate(&e0);
  if (err != hipSuccess) return err;
  if ((err = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return err;
  }
  double best = 1e300;
  f();
  err = hipGetLastError();
  for (int r = 0; r < reps && err == hipSuccess; ++r) {
    if ((err = hipEventRecord(e0, st)) != hipSuccess) break;
    f();
    if ((err = hipGetLastError()) != hipSuccess) break;
    if ((err = hipEventRecord(e1, st)) != hipSuccess) break;
    if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
    float ms = 0.f;
    if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
    best = std::min(best, (double)ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *out = best;
  return err;
}

}  // namespace

hipError_t probe_hbm_copy(void* dst, const void* src, size_t bytes, int reps, hipStream_t st, double* gbs) {
  const size_t n4 = bytes / 16;
  const int blocks = device_cus() * 8;
  double ms = 0.0;
  hipError_t e = best_ms(
      [&] {
        hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(kProbeThreads), 0, st, (const float4*)src, (float4*)dst, n4);
      },
      reps, st, &ms);
  *gbs = ms > 0 ? 2.0 * (double)(n4 * 16) / (ms * 1e-3) / 1e9 : 0.0;
  return e;
}

hipError_t probe_peak(int kind, float* sink, int reps, hipStream_t st, double* tflops) {
  const int blocks = device_cus() * 8;  // 8 waves per SIMD
  const int iters = 4096;
  const double threads = (double)blocks * kProbeThreads, waves = threads / 64.0;
  double flops = 0.0, ms = 0.0;
  hipError_t e = hipSuccess;
  switch (kind) {
    case 0:
      flops = 2.0 * kChains * iters * threads;
      e = best_ms([&] { hipLaunchKernelGGL(fma_kernel<float>, dim3(blocks), dim3(kProbeThreads), 0, st, sink, iters); },
                  reps, st, &ms);
      break;
    case 1:
      flops = 2048.0 * 4 * iters * waves;
      e = best_ms([&] { hipLaunchKernelGGL(mfma_kernel<0>, dim3(blocks), dim3(kProbeThreads), 0, st, sink, iters); },
                  reps, st, &ms);
      break;
    case 2:
      flops = 512.0 * 4 * iters * waves;
      e = best_ms([&] { hipLaunchKernelGGL(mfma_kernel<1>, dim3(blocks), dim3(kProbeThreads), 0, st, sink, iters); },
                  reps, st, &ms);
      break;
    case 3:
      flops = 2.0 * kChains * iters * threads;
      e = best_ms(
          [&] {
            hipLaunchKernelGGL(fma_kernel<double>, dim3(blocks), dim3(kProbeThreads), 0, st, (double*)sink, iters);
          },
          reps, st, &ms);
      break;
    case 4:
      flops = 2.0 * 16 * 64 * 4 * iters * waves;  // 16 blocks of 4x4x4
      e = best_ms(
          [&] { hipLaunchKernelGGL(mfma_bf16_kernel<0>, dim3(blocks), dim3(kProbeThreads), 0, st, sink, iters); },
          reps, st, &ms);
      break;
    case 5:
      flops = 2.0 * 16 * 16 * 16 * 4 * iters * waves;
      e = best_ms(
          [&] { hipLaunchKernelGGL(mfma_bf16_kernel<1>, dim3(blocks), dim3(kProbeThreads), 0, st, sink, iters); },
          reps, st, &ms);
      break;
    case 6:
      flops = 2.0 * 16 * 16 * 32 * 4 * iters * waves;
      e = best_ms(
          [&] { hipLaunchKernelGGL(mfma_bf16_kernel<2>, dim3(blocks), dim3(kProbeThreads), 0, st, sink, iters); },
          reps, st, &ms);
      break;
    default:
      return hipErrorInvalidValue;
  }
  *tflops = ms > 0 ? flops / (ms * 1e-3) / 1e12 : 0.0;
  return e;
}

}  // namespace sdl
