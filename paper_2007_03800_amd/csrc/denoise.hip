// Patch-denoising driver of the experiments in Sec. IV: an H x W image is cut into all
// (H - m1 + 1)(W - m2 + 1) overlapping m1 x m2 patches (stride 1), the patches are coded (the
// error-driven 2D-OMP of sdl_sparse_code with err2), and the image is put back together from the
// coded patches D1 X_k D2^T, every pixel the plain average of the estimates of the patches that
// cover it.
//
// Image: row-major, pixel (y, x) at y W + x.  Patch k = r C + c (C = W - m2 + 1) holds pixel
// (r + i, c + j) at its (i, j), stored column-major like every signal of the library.
// The rebuild runs in two passes: every patch's estimate D1 X_k D2^T into a buffer (one wave
// per patch), then a gather in which each output pixel sums its covering patches' estimates in
// a fixed order; there are no atomics and the result is reproducible.
#include "sdl_internal.h"

namespace sdl {
namespace {

template <typename T>
__global__ void image_to_patches_kernel(const T* __restrict__ img, int H, int W, int m1, int m2, T* __restrict__ out,
                                        int64_t total) {
  const int C = W - m2 + 1, M = m1 * m2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e / M;
    const int px = (int)(e % M), i = px % m1, j = px / m1;
    const int64_t r = k / C, c = k % C;
    out[e] = img[(r + i) * W + (c + j)];
  }
}

// Estimate of every coded patch, D1 X_k D2^T, one wave per patch: the support slots of a patch
// are wave-uniform (scalar loads and branches); unused slots (-1) are skipped wherever they are.
template <typename T>
__global__ void __launch_bounds__(kWave) patch_estimates_kernel(const int32_t* __restrict__ supp,
                                                               const T* __restrict__ coef, const T* __restrict__ D1,
                                                               const T* __restrict__ D2, int64_t N, int m1, int m2,
                                                               int n1, int n2, int s, T* __restrict__ blocks) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sD1 = reinterpret_cast<T*>(smem_raw);  // m1 x n1
  T* sD2 = sD1 + m1 * n1;                    // m2 x n2
  for (int e = threadIdx.x; e < m1 * n1; e += blockDim.x) sD1[e] = D1[e];
  for (int e = threadIdx.x; e < m2 * n2; e += blockDim.x) sD2[e] = D2[e];
  __syncthreads();
  const int M = m1 * m2;
  for (int64_t k = blockIdx.x; k < N; k += gridDim.x) {
    for (int px = threadIdx.x; px < M; px += blockDim.x) {
      const int i = px % m1, j = px / m1;
      T v = 0;
      for (int t = 0; t < s; ++t) {
        const int a = supp[k * s + t];
        if (a < 0) continue;
        v += coef[k * s + t] * sD1[i + m1 * (a % n1)] * sD2[j + m2 * (a / n1)];
      }
      blocks[k * M + px] = v;
    }
  }
}

// One thread per output pixel: the estimates of the covering patches (r, c) in increasing r,
// then c, summed in that order and divided by their count.
template <typename T>
__global__ void __launch_bounds__(256) overlap_average_kernel(const T* __restrict__ blocks, int H, int W, int m1,
                                                              int m2, T* __restrict__ img) {
  const int C = W - m2 + 1, R = H - m1 + 1, M = m1 * m2;
  const int64_t npix = (int64_t)H * W;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(p / W), x = (int)(p % W);
    const int r0 = y - m1 + 1 > 0 ? y - m1 + 1 : 0, r1 = y < R - 1 ? y : R - 1;
    const int c0 = x - m2 + 1 > 0 ? x - m2 + 1 : 0, c1 = x < C - 1 ? x : C - 1;
    T acc = 0;
    for (int r = r0; r <= r1; ++r)
      for (int c = c0; c <= c1; ++c) acc += blocks[((int64_t)r * C + c) * M + (y - r) + m1 * (x - c)];
    img[p] = acc / (T)((r1 - r0 + 1) * (c1 - c0 + 1));
  }
}

}  // namespace

template <typename T>
hipError_t launch_image_to_patches(const T* img, int H, int W, int m1, int m2, T* out, hipStream_t st) {
  const int64_t total = (int64_t)(H - m1 + 1) * (W - m2 + 1) * m1 * m2;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(image_to_patches_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, st, img, H, W, m1, m2, out,
                     total);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_patches_to_image(const int32_t* supp, const T* coef, const T* D1, const T* D2, int H, int W, int m1,
                                   int m2, int n1, int n2, int s, T* blocks, T* img, hipStream_t st) {
  const int64_t npix = (int64_t)H * W;
  if (npix <= 0) return hipSuccess;
  const int64_t N = (int64_t)(H - m1 + 1) * (W - m2 + 1);
  const int64_t g1 = N < 65536 ? N : 65536;
  const size_t lds = sizeof(T) * ((size_t)m1 * n1 + (size_t)m2 * n2);
  hipLaunchKernelGGL(patch_estimates_kernel<T>, dim3((unsigned)g1), dim3(kWave), lds, st, supp, coef, D1, D2, N, m1,
                     m2, n1, n2, s, blocks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t blocks2 = (npix + 255) / 256;
  if (blocks2 > 65536) blocks2 = 65536;
  hipLaunchKernelGGL(overlap_average_kernel<T>, dim3((unsigned)blocks2), dim3(256), 0, st, blocks, H, W, m1, m2, img);
  return hipGetLastError();
}

template hipError_t launch_image_to_patches<float>(const float*, int, int, int, int, float*, hipStream_t);
template hipError_t launch_image_to_patches<double>(const double*, int, int, int, int, double*, hipStream_t);
template hipError_t launch_patches_to_image<float>(const int32_t*, const float*, const float*, const float*, int, int,
                                                   int, int, int, int, int, float*, float*, hipStream_t);
template hipError_t launch_patches_to_image<double>(const int32_t*, const double*, const double*, const double*, int,
                                                    int, int, int, int, int, int, double*, double*, hipStream_t);

}  // namespace sdl
