// TMOD dictionary update kernels (Algorithm 1 steps 1-4; Corollary 1, Proposition 1).
//
// Side 1 (D1 update, Corollary 1):  T_k = X_k D2^T (n1 x m2)
//     A = sum_k T_k T_k^T (n1 x n1),  B = sum_k Y_k T_k^T (m1 x n1),  D1* = B A^{-1}
// Side 2 (D2 update, Proposition 1): Z_k = D1 X_k (m1 x n2), U_k = Z_k^T
//     A = sum_k Z_k^T Z_k (n2 x n2),  B = sum_k Y_k^T Z_k (m2 x n2),  D2* = B A^{-1}
// Both are written once with "row atoms" ra (i for side 1, j for side 2), the
// signal seen as Yt (Y for side 1, Y^T for side 2) and the fixed dictionary Do
// (D2 for side 1, D1 for side 2): T[ra][c] = sum over code entries x * Do[c, rb].
//
// One GPU plays every node of Algorithm 1: each workgroup owns a contiguous
// slice of signals (a "node"), accumulates its partial sums, and writes them as
// FP64 partials; a fixed-order FP64 reduction (the master's sum) and an FP64
// Cholesky solve on one workgroup follow.  Nothing uses floating-point atomics,
// so results are bitwise reproducible.
#include <math.h>

#include "sdl_internal.h"

namespace sdl {
namespace {

// out[e] = sum over workgroup partials b of part[b][e], in a fixed order: four
// interleaved stripes per entry, then the stripes in order.
__global__ void __launch_bounds__(256) reduce_partials_kernel(const double* __restrict__ part, int nblk, int nent,
                                                              double* out) {
  __shared__ double red[4][64];
  const int el = threadIdx.x % 64, stripe = threadIdx.x / 64;
  const int e = blockIdx.x * 64 + el;
  double v = 0.0;
  if (e < nent) {
#pragma unroll 8
    for (int b = stripe; b < nblk; b += 4) v += part[(size_t)b * nent + e];
  }
  red[stripe][el] = v;
  __syncthreads();
  if (stripe == 0 && e < nent) out[e] = ((red[0][el] + red[1][el]) + red[2][el]) + red[3][el];
}

// D (mr x na FP64) -> compute-type copy, FP64 and compute-type Gram D^T D.
template <typename T>
__device__ void write_copies(const double* D, int mr, int na, T* Dc, double* G64, T* Gc) {
  for (int e = threadIdx.x; e < mr * na; e += blockDim.x) Dc[e] = (T)D[e];
  for (int e = threadIdx.x; e < na * na; e += blockDim.x) {
    const int i = e % na, j = e / na;
    double v = 0.0;
    for (int p = 0; p < mr; ++p) v += D[p + mr * i] * D[p + mr * j];
    G64[e] = v;
    Gc[e] = (T)v;
  }
}

template <typename T>
__global__ void dict_prep_kernel(const double* D, int mr, int na, T* Dc, double* G64, T* Gc) {
  write_copies<T>(D, mr, na, Dc, G64, Gc);
}

constexpr double kSpdRelTol = 1e-12;  // pivot <= tol * diagonal entry -> not positive definite
constexpr int kLd = SDL_MAX_N + 1;     // padded LDS row length

__device__ inline void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wavefront: FP64 Cholesky of the Gram sum on the used atoms, two triangular
// solves with mr right-hand sides, normalisation.  sums = [A (na x na) | B (mr x na)],
// column-major.  All steps are wave-synchronous (no workgroup barriers).
template <typename T>
__global__ void __launch_bounds__(64)
    tmod_solve_kernel(const double* sums, int mr, int na, double* D, T* Dc, double* G64, T* Gc, double* w,
                      int* status, unsigned long long* counters) {
  __shared__ double C[SDL_MAX_N * kLd];
  __shared__ double X[SDL_MAX_N * kLd];  // X[k][p]: right-hand sides / solution, atom k, row p
  __shared__ double diag0[SDL_MAX_N];
  __shared__ int U[SDL_MAX_N];
  const int lane = threadIdx.x;
  const double* A = sums;
  const double* B = sums + na * na;
  // used atoms (positive diagonal), compacted in index order with a ballot
  const bool used = lane < na && A[lane + na * lane] > 0.0;
  const unsigned long long mask = __ballot(used);
  const int nu = __popcll(mask);
  if (used) U[__popcll(mask & ((1ull << lane) - 1ull))] = lane;
  if (lane == 0 && nu < na) atomicAdd(&counters[kCtrUnusedAtoms], (unsigned long long)(na - nu));
  wsync();
  for (int e = lane; e < nu * nu; e += 64) {
    const int k = e % nu, l = e / nu;
    C[k * kLd + l] = A[U[k] + na * U[l]];
    if (k == l) diag0[k] = C[k * kLd + k];
  }
  for (int e = lane; e < nu * mr; e += 64) {
    const int k = e % nu, p = e / nu;
    X[k * kLd + p] = B[p + mr * U[k]];
  }
  wsync();
  bool bad = false;
  for (int k = 0; k < nu && !bad; ++k) {
    const double d = C[k * kLd + k];
    if (!(d > kSpdRelTol * diag0[k])) {
      bad = true;
      break;
    }
    const double lkk = sqrt(d), inv = 1.0 / lkk;
    wsync();
    if (lane == 0) C[k * kLd + k] = lkk;
    for (int i = k + 1 + lane; i < nu; i += 64) C[i * kLd + k] *= inv;
    wsync();
    const int rem = nu - k - 1;
    for (int e = lane; e < rem * rem; e += 64) {
      const int i = k + 1 + e % rem, j = k + 1 + e / rem;
      if (j <= i) C[i * kLd + j] -= C[i * kLd + k] * C[j * kLd + k];
    }
    wsync();
  }
  if (!bad) {
    // L Z = X (forward), then L^T X = Z (backward); columns p in parallel
    for (int k = 0; k < nu; ++k) {
      const double inv = 1.0 / C[k * kLd + k];
      for (int p = lane; p < mr; p += 64) X[k * kLd + p] *= inv;
      wsync();
      for (int e = lane; e < (nu - k - 1) * mr; e += 64) {
        const int i = k + 1 + e / mr, p = e % mr;
        X[i * kLd + p] -= C[i * kLd + k] * X[k * kLd + p];
      }
      wsync();
    }
    for (int k = nu - 1; k >= 0; --k) {
      const double inv = 1.0 / C[k * kLd + k];
      for (int p = lane; p < mr; p += 64) X[k * kLd + p] *= inv;
      wsync();
      for (int e = lane; e < k * mr; e += 64) {
        const int i = e / mr, p = e % mr;
        X[i * kLd + p] -= C[k * kLd + i] * X[k * kLd + p];
      }
      wsync();
    }
    // normalisation W: unit-norm columns; a zero column keeps the old atom; unused atoms kept
    for (int i = lane; i < na; i += 64) w[i] = 1.0;
    wsync();
    for (int k = lane; k < nu; k += 64) {
      const int i = U[k];
      double nrm = 0.0;
      for (int p = 0; p < mr; ++p) nrm += X[k * kLd + p] * X[k * kLd + p];
      nrm = sqrt(nrm);
      if (nrm > 0.0) {
        w[i] = nrm;
        for (int p = 0; p < mr; ++p) D[p + mr * i] = X[k * kLd + p] / nrm;
      }
    }
  } else {
    for (int i = lane; i < na; i += 64) w[i] = 1.0;
    if (lane == 0) {
      atomicOr(status, kStatusSingular);
      atomicAdd(&counters[kCtrSingular], 1ull);
    }
  }
  __threadfence_block();
  wsync();
  write_copies<T>(D, mr, na, Dc, G64, Gc);
}

template <typename T>
__global__ void rescale_kernel(int side, int n1, int s, int64_t N, const int32_t* supp, T* coef,
                               const double* w) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * s) return;
  const int at = supp[e];
  if (at < 0) return;
  const int idx = side == 1 ? at % n1 : at / n1;
  coef[e] = (T)((double)coef[e] * w[idx]);
}

constexpr int kRmseThreads = 256;

template <typename T>
__global__ void __launch_bounds__(kRmseThreads) rmse_partial_kernel(const T* res2, int64_t N, int nblk, double* part) {
  __shared__ double red[kRmseThreads];
  const int64_t k0 = (N * blockIdx.x) / nblk, k1 = (N * (blockIdx.x + 1)) / nblk;
  double v = 0.0;
  for (int64_t k = k0 + threadIdx.x; k < k1; k += kRmseThreads) v += (double)res2[k];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = kRmseThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void rmse_final_kernel(const double* part, int nblk, double denom, double* trace, int stride, int offset,
                                  int* counter) {
  if (threadIdx.x != 0) return;
  double v = 0.0;
  for (int b = 0; b < nblk; ++b) v += part[b];
  const int it = *counter;
  trace[(size_t)it * stride + offset] = denom > 0 ? sqrt(v / denom) : 0.0;
  *counter = it + 1;
}

template <typename T>
__global__ void check_finite_kernel(const T* x, int64_t n, int* status) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    if (!isfinite((double)x[e])) {
      atomicOr(status, kStatusNonfinite);
      return;
    }
  }
}

__global__ void fill_int_kernel(int* p, int n, int v) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}

}  // namespace

hipError_t launch_reduce_partials(const double* part, int nblk, int nent, double* out, hipStream_t st) {
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((nent + 63) / 64), dim3(256), 0, st, part, nblk, nent, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tmod_solve(const double* sums, int mr, int na, double* D, T* Dc, double* G64, T* Gc, double* w,
                             int* status, unsigned long long* counters, hipStream_t st) {
  hipLaunchKernelGGL(tmod_solve_kernel<T>, dim3(1), dim3(64), 0, st, sums, mr, na, D, Dc, G64, Gc, w,
                     status, counters);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dict_prep(const double* D, int mr, int na, T* Dc, double* G64, T* Gc, hipStream_t st) {
  hipLaunchKernelGGL(dict_prep_kernel<T>, dim3(1), dim3(256), 0, st, D, mr, na, Dc, G64, Gc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rescale(int side, int n1, int s, int64_t N, const int32_t* supp, T* coef, const double* w,
                          hipStream_t st) {
  const int64_t n = N * s;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(rescale_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, side, n1, s, N, supp,
                     coef, w);
  return hipGetLastError();
}

int rmse_num_blocks(int64_t N) {
  int64_t b = (N + 4095) / 4096;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

template <typename T>
hipError_t launch_rmse(const T* res2, int64_t N, double denom, double* part, int nblk, double* trace, int stride,
                       int offset, int* counter, hipStream_t st) {
  hipLaunchKernelGGL(rmse_partial_kernel<T>, dim3(nblk), dim3(kRmseThreads), 0, st, res2, N, nblk, part);
  hipLaunchKernelGGL(rmse_final_kernel, dim3(1), dim3(64), 0, st, part, nblk, denom, trace, stride, offset, counter);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_check_finite(const T* x, int64_t n, int* status, hipStream_t st) {
  if (n == 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(check_finite_kernel<T>, dim3((unsigned)g), dim3(256), 0, st, x, n, status);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int n, int v, hipStream_t st) {
  hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

#define SDL_INST(T)                                                                                            \
  template hipError_t launch_tmod_solve<T>(const double*, int, int, double*, T*, double*, T*, double*, int*,  \
                                           unsigned long long*, hipStream_t);                                 \
  template hipError_t launch_dict_prep<T>(const double*, int, int, T*, double*, T*, hipStream_t);             \
  template hipError_t launch_rescale<T>(int, int, int, int64_t, const int32_t*, T*, const double*,            \
                                        hipStream_t);                                                         \
  template hipError_t launch_rmse<T>(const T*, int64_t, double, double*, int, double*, int, int, int*,        \
                                     hipStream_t);                                                            \
  template hipError_t launch_check_finite<T>(const T*, int64_t, int*, hipStream_t);
SDL_INST(float)
SDL_INST(double)
#undef SDL_INST

}  // namespace sdl
