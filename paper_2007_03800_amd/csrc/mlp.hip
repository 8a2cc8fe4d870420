// Learned support proposal: the kernels of a small MLP (vec(Y)/||Y|| -> hidden ->
// hidden -> one logit per atom) and of the proposal step that turns its logits into
// a code.  Not a step of the paper's method: a learned front end whose output is
// only accepted when its least-squares residual passes a calibrated test, 2D-OMP
// (Sec. III step 1) being the fallback.
//
// GEMMs run on the matrix cores: 16x16x32 BF16 MFMA with FP32 accumulation
// (lane l supplies A[l%16][8(l/16)..8(l/16)+7] and B[8(l/16)..+7][l%16]; result v of
// lane l is D[4(l/16)+v][l%16]), or 16x16x4 FP32 MFMA in the FP32 check mode.
// Workgroup tile 64x64x32 staged through LDS in K-contiguous layout, four waves of
// 32x32 (all operand layouts, FP32 or BF16); the BF16 forward layers use a 128x128
// tile kernel with register-prefetched 16-byte loads.  Epilogues are fused: bias + exact-erf GELU (keeping the pre-activation for
// the backward pass), multiplication by GELU'(z) when back-propagating, FP32 store.
#include <hip/hip_bf16.h>
#include <math.h>

#include "mlp_internal.h"

namespace sdl {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 32, KP = BK + 8;  // LDS row length (16-byte aligned, bank spread)

template <typename T>
__device__ inline T from_float(float x);
template <>
__device__ inline float from_float<float>(float x) { return x; }
template <>
__device__ inline __bf16 from_float<__bf16>(float x) { return (__bf16)x; }

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
  // d/dz [z Phi(z)] = Phi(z) + z phi(z)
  const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * z * z);
  return cdf + z * pdf;
}

// A(M x K), B(K x N): opA 0 = row-major A[m*lda+k], 1 = stored transposed A[k*lda+m];
// opB 0 = row-major B[k*ldb+n], 1 = stored transposed B[n*ldb+k].
template <typename T, int OPA, int OPB>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g) {
  __shared__ __align__(16) T As[BM][KP];
  __shared__ __align__(16) T Bs[BN][KP];
  const T* A = static_cast<const T*>(g.A);
  const T* B = static_cast<const T*>(g.B);
  const int tid = threadIdx.x, w = tid / 64, lane = tid % 64;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wm = (w / 2) * 32, wn = (w % 2) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < g.K; k0 += BK) {
    // stage A tile -> As[m][k], B tile -> Bs[n][k]  (BM*BK = 2048 elements, 8 per thread)
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = tid + 256 * u;
      if (OPA == 0) {
        const int m = e / BK, k = e % BK;
        As[m][k] = A[(size_t)(m0 + m) * g.lda + k0 + k];
      } else {
        const int k = e / BM, m = e % BM;
        As[m][k] = A[(size_t)(k0 + k) * g.lda + m0 + m];
      }
      if (OPB == 0) {
        const int k = e / BN, n = e % BN;
        Bs[n][k] = B[(size_t)(k0 + k) * g.ldb + n0 + n];
      } else {
        const int n = e / BK, k = e % BK;
        Bs[n][k] = B[(size_t)(n0 + n) * g.ldb + k0 + k];
      }
    }
    __syncthreads();
    const int r16 = lane % 16, kq = lane / 16;
    if constexpr (sizeof(T) == 2) {
      bf16x8 af[2], bfr[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = *reinterpret_cast<const bf16x8*>(&As[wm + 16 * i + r16][8 * kq]);
#pragma unroll
      for (int j = 0; j < 2; ++j) bfr[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn + 16 * j + r16][8 * kq]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        float af[2], bfr[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) af[i] = (float)As[wm + 16 * i + r16][kk + kq];
#pragma unroll
        for (int j = 0; j < 2; ++j) bfr[j] = (float)Bs[wn + 16 * j + r16][kk + kq];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bfr[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // epilogue
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm + 16 * i + 4 * (lane / 16) + v;
        const int n = n0 + wn + 16 * j + lane % 16;
        float x = acc[i][j][v];
        const size_t o = (size_t)m * g.ldc + n;
        switch (g.epi) {
          case kEpiStoreF32:
            if (g.bias) x += g.bias[n];
            static_cast<float*>(g.C)[o] = x;
            break;
          case kEpiBiasGelu: {
            const float z = x + g.bias[n];
            if (g.Z) g.Z[o] = z;
            static_cast<T*>(g.C)[o] = from_float<T>(gelu(z));
            break;
          }
          case kEpiGeluGrad:
            static_cast<T*>(g.C)[o] = from_float<T>(x * gelu_grad(g.Z[o]));
            break;
          default:
            break;
        }
      }
}

// BF16 C = A B^T (A: M x K activations, row-major; B: N x K weights, row-major) for the
// forward layers.  Each MFMA operand fragment (one row, 8 consecutive k) is 16 contiguous
// bytes of A or B, so lanes load their fragments straight from global memory into
// registers (no LDS, no barriers), four K slices in flight.  Workgroup tile 128 x 128,
// four waves of 64 x 64 (4 x 4 MFMA 16x16x32 tiles), rows >= M masked.  Same epilogues as
// gemm_kernel.
constexpr int TM = 128, TN = 128, TK = 32;
constexpr int kXcds = 8;  // accelerator complex dies of an MI355X

__global__ void __launch_bounds__(256) gemm_nt_bf16_kernel(GemmArgs g) {
  const __bf16* A = static_cast<const __bf16*>(g.A);
  const __bf16* B = static_cast<const __bf16*>(g.B);
  const int tid = threadIdx.x, w = tid / 64, lane = tid % 64;
  // workgroups are dealt round-robin to the 8 XCDs (each with its own L2): give each XCD a
  // contiguous run of tiles, so the N tiles of one row panel of A share an L2
  const int ntn = gridDim.x, ntiles = gridDim.x * gridDim.y;
  const int lin = blockIdx.x + gridDim.x * blockIdx.y;
  int tile = lin;
  if (ntiles % kXcds == 0) tile = (lin % kXcds) * (ntiles / kXcds) + lin / kXcds;
  const int m0 = (tile / ntn) * TM, n0 = (tile % ntn) * TN;
  const int wm = (w / 2) * 64, wn = (w % 2) * 64;
  const int r16 = lane % 16, kq = lane / 16;
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const __bf16* pa[4];
  const __bf16* pb[4];
  bool va[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + wm + 16 * i + r16;
    va[i] = m < g.M;
    pa[i] = A + (size_t)(va[i] ? m : 0) * g.lda + 8 * kq;
    pb[i] = B + (size_t)(n0 + wn + 16 * i + r16) * g.ldb + 8 * kq;
  }
  auto load = [&](bf16x8 (&a)[4], bf16x8 (&b)[4], int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = *reinterpret_cast<const bf16x8*>(pa[i] + k0);
      if (!va[i]) a[i] = bf16x8{};
      b[i] = *reinterpret_cast<const bf16x8*>(pb[i] + k0);
    }
  };
  auto mma = [&](const bf16x8 (&a)[4], const bf16x8 (&b)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  };
  // four K slices in flight per wave (the global-load latency is several times one
  // slice's MFMA work); stage indices are static after unrolling by four
  constexpr int NS = 4;
  bf16x8 a[NS][4], b[NS][4];
  const int nk = g.K / TK;
#pragma unroll
  for (int u = 0; u < NS - 1; ++u)
    if (u < nk) load(a[u], b[u], u * TK);
  for (int ks = 0; ks < nk; ks += NS) {
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int k = ks + u;
      if (k < nk) {
        if (k + NS - 1 < nk) load(a[(u + NS - 1) % NS], b[(u + NS - 1) % NS], (k + NS - 1) * TK);
        mma(a[u], b[u]);
      }
    }
  }
  // epilogue through LDS, 32 rows of the wave's 64 x 64 tile at a time: the raw sums go in
  // in the MFMA layout and come out as runs of 4 consecutive columns, where bias, GELU /
  // GELU' and the conversion are applied and every store is a contiguous 8- or 16-byte chunk
  __shared__ __align__(16) float stile[4][32][64 + 4];
  float(*st)[68] = stile[w];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) st[16 * i + 4 * kq + v][16 * j + r16] = acc[2 * h + i][j][v];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = lane + 64 * u, r = e / 16, c4 = 4 * (e % 16);
      const int m = m0 + wm + 32 * h + r, n = n0 + wn + c4;
      if (m >= g.M) continue;
      const float4 x = *reinterpret_cast<const float4*>(&st[r][c4]);
      const size_t o = (size_t)m * g.ldc + n;
      float y[4] = {x.x, x.y, x.z, x.w};
      if (g.epi == kEpiStoreF32) {
        if (g.bias) {
          const float4 b = *reinterpret_cast<const float4*>(g.bias + n);
          y[0] += b.x; y[1] += b.y; y[2] += b.z; y[3] += b.w;
        }
        *reinterpret_cast<float4*>(static_cast<float*>(g.C) + o) = make_float4(y[0], y[1], y[2], y[3]);
      } else {
        if (g.epi == kEpiBiasGelu) {
          const float4 b = *reinterpret_cast<const float4*>(g.bias + n);
          y[0] += b.x; y[1] += b.y; y[2] += b.z; y[3] += b.w;
          if (g.Z) *reinterpret_cast<float4*>(g.Z + o) = make_float4(y[0], y[1], y[2], y[3]);
#pragma unroll
          for (int q = 0; q < 4; ++q) y[q] = gelu(y[q]);
        } else {  // kEpiGeluGrad
          const float4 z = *reinterpret_cast<const float4*>(g.Z + o);
          y[0] *= gelu_grad(z.x); y[1] *= gelu_grad(z.y); y[2] *= gelu_grad(z.z); y[3] *= gelu_grad(z.w);
        }
        __bf16* co = static_cast<__bf16*>(g.C) + o;
        bf16x4 ov;
#pragma unroll
        for (int q = 0; q < 4; ++q) ov[q] = (__bf16)y[q];
        *reinterpret_cast<bf16x4*>(co) = ov;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// X[b][p] = Y_{idx(b)}[p] / ||Y_{idx(b)}||_F in the compute type (vec order = column-major)
template <typename T>
__global__ void prep_input_kernel(const float* Y, const int32_t* idx, int64_t B, int M, T* X, float* ynorm2) {
  const int64_t b = blockIdx.x;
  if (b >= B) return;
  const int64_t src = idx ? idx[b] : b;
  const float* y = Y + src * M;
  __shared__ float red[64];
  float s = 0.f;
  for (int p = threadIdx.x; p < M; p += blockDim.x) s += y[p] * y[p];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 32; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const float nrm2 = red[0];
  const float inv = nrm2 > 0.f ? rsqrtf(nrm2) : 0.f;
  for (int p = threadIdx.x; p < M; p += blockDim.x) X[b * M + p] = from_float<T>(y[p] * inv);
  if (ynorm2 && threadIdx.x == 0) ynorm2[b] = nrm2;
}

// dZ = (sigmoid(z) - label) / (B * A), label = 1 on the atoms of the code; per-block FP64 loss partials
template <typename T>
__global__ void __launch_bounds__(256) bce_grad_kernel(const float* Z, const int32_t* supp, const int32_t* idx, int64_t B,
                                                       int A, int s, T* dZ, double* loss_part) {
  __shared__ double red[256];
  const int64_t b = blockIdx.x;
  const int64_t src = idx ? idx[b] : b;
  double l = 0.0;
  const float scale = 1.0f / ((float)B * (float)A);
  for (int a = threadIdx.x; a < A; a += blockDim.x) {
    float y = 0.f;
    for (int t = 0; t < s; ++t) y = supp[src * s + t] == a ? 1.f : y;
    const float z = Z[b * A + a];
    const float sig = 1.f / (1.f + expf(-z));
    dZ[b * A + a] = from_float<T>((sig - y) * scale);
    // stable BCE with logits: max(z,0) - z*y + log(1 + exp(-|z|))
    l += (double)(fmaxf(z, 0.f) - z * y + log1pf(expf(-fabsf(z))));
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[b] = red[0];
}

// db[n] = sum_b dZ[b][n], fixed order (one thread per column)
template <typename T>
__global__ void bias_grad_kernel(const T* dZ, int64_t B, int N, float* db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int64_t b = 0; b < B; ++b) s += (float)dZ[b * N + n];
  db[n] = s;
}

__global__ void sum_kernel(const double* x, int64_t n, double scale, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += x[i];
  *out = s * scale;
}

// Adam on the FP32 master parameters, then the compute-type copy
template <typename T>
__global__ void adam_kernel(float* p, float* m, float* v, const float* g, T* pc, int64_t n, float lr, float b1, float b2,
                            float eps, float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / bc1, vh = vi / bc2;
  const float pi = p[i] - lr * mh / (sqrtf(vh) + eps);
  p[i] = pi;
  if (pc) pc[i] = from_float<T>(pi);
}

template <typename T>
__global__ void copy_params_kernel(const float* p, T* pc, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pc[i] = from_float<T>(p[i]);
}

}  // namespace

template <typename T>
hipError_t launch_gemm(const GemmArgs& g, int opA, int opB, hipStream_t st) {
  const bool aligned = ((reinterpret_cast<uintptr_t>(g.A) | reinterpret_cast<uintptr_t>(g.B) |
                         reinterpret_cast<uintptr_t>(g.C) | reinterpret_cast<uintptr_t>(g.Z) |
                         reinterpret_cast<uintptr_t>(g.bias)) & 15u) == 0;
  if (sizeof(T) == 2 && opA == 0 && opB == 1 && aligned && g.N % TN == 0 && g.K % TK == 0 && g.lda % 8 == 0 &&
      g.ldb % 8 == 0 && g.ldc % 4 == 0) {
    hipLaunchKernelGGL(gemm_nt_bf16_kernel, dim3(g.N / TN, (g.M + TM - 1) / TM), dim3(256), 0, st, g);
    return hipGetLastError();
  }
  const dim3 grid(g.N / BN, g.M / BM);
  if (opA == 0 && opB == 1) hipLaunchKernelGGL((gemm_kernel<T, 0, 1>), grid, dim3(256), 0, st, g);
  else if (opA == 0 && opB == 0) hipLaunchKernelGGL((gemm_kernel<T, 0, 0>), grid, dim3(256), 0, st, g);
  else if (opA == 1 && opB == 0) hipLaunchKernelGGL((gemm_kernel<T, 1, 0>), grid, dim3(256), 0, st, g);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prep_input(const float* Y, const int32_t* idx, int64_t B, int M, T* X, float* ynorm2, hipStream_t st) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(prep_input_kernel<T>, dim3((unsigned)B), dim3(64), 0, st, Y, idx, B, M, X, ynorm2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bce_grad(const float* Z, const int32_t* supp, const int32_t* idx, int64_t B, int A, int s, T* dZ,
                           double* loss_part, double* loss, hipStream_t st) {
  hipLaunchKernelGGL(bce_grad_kernel<T>, dim3((unsigned)B), dim3(256), 0, st, Z, supp, idx, B, A, s, dZ, loss_part);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(64), 0, st, loss_part, B, 1.0 / ((double)B * A), loss);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bias_grad(const T* dZ, int64_t B, int N, float* db, hipStream_t st) {
  hipLaunchKernelGGL(bias_grad_kernel<T>, dim3((N + 255) / 256), dim3(256), 0, st, dZ, B, N, db);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adam(float* p, float* m, float* v, const float* g, T* pc, int64_t n, float lr, int step,
                       hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float bc1 = 1.f - powf(b1, (float)step), bc2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, m, v, g, pc, n, lr, b1, b2,
                     eps, bc1, bc2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy_params(const float* p, T* pc, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(copy_params_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, pc, n);
  return hipGetLastError();
}

#define SDL_MLP_INST(T)                                                                                           \
  template hipError_t launch_gemm<T>(const GemmArgs&, int, int, hipStream_t);                                   \
  template hipError_t launch_prep_input<T>(const float*, const int32_t*, int64_t, int, T*, float*, hipStream_t); \
  template hipError_t launch_bce_grad<T>(const float*, const int32_t*, const int32_t*, int64_t, int, int, T*,    \
                                         double*, double*, hipStream_t);                                         \
  template hipError_t launch_bias_grad<T>(const T*, int64_t, int, float*, hipStream_t);                          \
  template hipError_t launch_adam<T>(float*, float*, float*, const float*, T*, int64_t, float, int, hipStream_t); \
  template hipError_t launch_copy_params<T>(const float*, T*, int64_t, hipStream_t);
SDL_MLP_INST(float)
SDL_MLP_INST(__bf16)
#undef SDL_MLP_INST

}  // namespace sdl
