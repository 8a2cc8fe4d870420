// TMOD dictionary update kernels (Algorithm 1 steps 1-4; Corollary 1, Result 1).
//
// Side 1 (D1 update, Corollary 1):  T_k = X_k D2^T (n1 x m2)
//     A = sum_k T_k T_k^T (n1 x n1),  B = sum_k Y_k T_k^T (m1 x n1),  D1* = B A^{-1}
// Side 2 (D2 update, Result 1): Z_k = D1 X_k (m1 x n2), U_k = Z_k^T
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
#include "tmod_device.h"

namespace sdl {
namespace {

// Fixed-order two-stage reduction of P partial rows of nent doubles: stage 1 sums
// consecutive chunks of kChunk rows per entry (in row order), stage 2 the chunk sums
// (in chunk order).
constexpr int kChunk = 64;

__global__ void reduce_stage1_kernel(const double* __restrict__ part, int P, int nent, double* stage) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (e >= nent) return;
  const int b0 = c * kChunk, b1 = (c + 1) * kChunk < P ? (c + 1) * kChunk : P;
  double v = 0.0;
  if (b1 - b0 == kChunk) {
    // a whole chunk: every load issued before the adds, which stay in row order
    double q[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) q[u] = part[(size_t)(b0 + u) * nent + e];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) v += q[u];
  } else {
    for (int b = b0; b < b1; ++b) v += part[(size_t)b * nent + e];
  }
  stage[(size_t)c * nent + e] = v;
}

// The last reduction stage alone: out[e] = sum over the nrow rows of src (row stride ld)
// in row order, for e < n (the same order as the solve kernel's first stage).
__global__ void reduce_final_kernel(const double* __restrict__ src, int nrow, int ld, int n, double* out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double v = 0.0;
  for (int b = 0; b < nrow; ++b) v += src[(size_t)b * ld + e];
  out[e] = v;
}

constexpr int kSolveThreads = 512;
constexpr int kDirectRows = 2 * kChunk;  // up to this many partial rows the solve sums them itself

// The master step of Algorithm 1 (steps 2 and 4) in one workgroup: the last stage of
// the fixed-order reduction, sums[e] = sum over the nrow rows of src (row stride ld)
// in row order, then the solve and normalisation on the reduced [A | B]; optionally
// the reduced sum of squared residuals (sums[r.idx]) becomes the RMSE of the sweep
// that produced the codes.
template <typename T>
__global__ void __launch_bounds__(kSolveThreads)
    tmod_solve_kernel(const double* __restrict__ src, int nrow, int ld, double* sums, int mr, int na, double* D,
                      T* Dc, double* G64, T* Gc, double* w, int* status, unsigned long long* counters, RmseOut r,
                      int sums_in_lds) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int tid = threadIdx.x;
  // the reduced sums go to global memory (the caller's copy) and, when sums_in_lds, to the
  // front of LDS, where the solve reads them
  double* ssum = reinterpret_cast<double*>(smem_raw);
  for (int e = tid; e < ld; e += blockDim.x) {
    double v = 0.0;
    int b = 0;
    for (; b + 8 <= nrow; b += 8) {  // eight loads in flight, adds in row order
      double q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) q[u] = src[(size_t)(b + u) * ld + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) v += q[u];
    }
    for (; b < nrow; ++b) v += src[(size_t)b * ld + e];
    sums[e] = v;
    if (sums_in_lds) ssum[e] = v;
  }
  __syncthreads();
  const double* rs = sums_in_lds ? ssum : sums;
  if (r.trace && tid == 0) {
    const int it = *r.counter;
    r.trace[(size_t)it + r.offset] = r.denom > 0 ? sqrt(rs[r.idx] / r.denom) : 0.0;
    *r.counter = it + 1;
  }
  solve_update_block<T>(rs, mr, na, D, Dc, G64, Gc, w, status, counters,
                        smem_raw + (sums_in_lds ? solve_sums_lds_bytes(ld) : 0), tid, blockDim.x);
}

// The dictionary's compute-type copy and its Gram matrix (FP64 and compute type), with D
// staged in LDS at an odd column stride first: the Gram entries then read LDS without bank
// conflicts instead of global memory.
template <typename T>
__global__ void dict_prep_kernel(const double* D, int mr, int na, T* Dc, double* G64, T* Gc) {
  __shared__ double sD[(SDL_MAX_M + 1) * SDL_MAX_N];
  const int ldd = mr + 1, tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < mr * na; e += nt) {
    const double v = D[e];
    sD[e % mr + ldd * (e / mr)] = v;
    Dc[e] = (T)v;
  }
  __syncthreads();
  for (int e = tid; e < na * na; e += nt) {
    const int i = e % na, j = e / na;
    double v = 0.0;
    for (int p = 0; p < mr; ++p) v += sD[p + ldd * i] * sD[p + ldd * j];
    G64[e] = v;
    Gc[e] = (T)v;
  }
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

__global__ void sum_final_kernel(const double* part, int nblk, double* out) {
  if (threadIdx.x != 0) return;
  double v = 0.0;
  for (int b = 0; b < nblk; ++b) v += part[b];
  *out = v;
}

__global__ void fill_double_kernel(double* p, int n, double v) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
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

__global__ void check_finite_bf16_kernel(const uint16_t* x, int64_t n, int* status) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    if ((x[e] & 0x7F80u) == 0x7F80u) {  // exponent all ones: infinity or NaN
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

int launch_reduce_stage1(const double* part, int P, int ld, double* stage, const double** src, hipStream_t st,
                         hipError_t* err) {
  *err = hipSuccess;
  if (P <= kDirectRows) {
    *src = part;
    return P;
  }
  const int nchunk = (P + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(reduce_stage1_kernel, dim3((ld + 255) / 256, nchunk), dim3(256), 0, st, part, P, ld, stage);
  *err = hipGetLastError();
  *src = stage;
  return nchunk;
}

int reduce_stage_rows(int P) { return (P + kChunk - 1) / kChunk; }

hipError_t launch_reduce_final(const double* src, int nrow, int ld, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(reduce_final_kernel, dim3((n + 255) / 256), dim3(256), 0, st, src, nrow, ld, n, out);
  return hipGetLastError();
}

hipError_t launch_fill_double(double* p, int n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_double_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tmod_solve(const double* src, int nrow, int ld, double* sums, int mr, int na, double* D, T* Dc,
                             double* G64, T* Gc, double* w, int* status, unsigned long long* counters,
                             const RmseOut& r, hipStream_t st) {
  // the reduced sums stay in LDS too when they fit beside the solve's workspace
  const size_t base = solve_lds_bytes(na, mr), with = base + solve_sums_lds_bytes(ld);
  const int in_lds = with <= solve_lds_bytes(SDL_MAX_N, SDL_MAX_M) ? 1 : 0;
  hipLaunchKernelGGL(tmod_solve_kernel<T>, dim3(1), dim3(kSolveThreads), in_lds ? with : base, st, src, nrow, ld,
                     sums, mr, na, D, Dc, G64, Gc, w, status, counters, r, in_lds);
  return hipGetLastError();
}

hipError_t tmod_solve_init_device() {
  const int bytes = (int)solve_lds_bytes(SDL_MAX_N, SDL_MAX_M);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&tmod_solve_kernel<float>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&tmod_solve_kernel<double>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
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
hipError_t launch_sum_res2(const T* res2, int64_t N, double* part, int nblk, double* out, hipStream_t st) {
  hipLaunchKernelGGL(rmse_partial_kernel<T>, dim3(nblk), dim3(kRmseThreads), 0, st, res2, N, nblk, part);
  hipLaunchKernelGGL(sum_final_kernel, dim3(1), dim3(64), 0, st, part, nblk, out);
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

hipError_t launch_check_finite_bf16(const uint16_t* x, int64_t n, int* status, hipStream_t st) {
  if (n == 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(check_finite_bf16_kernel, dim3((unsigned)g), dim3(256), 0, st, x, n, status);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int n, int v, hipStream_t st) {
  hipLaunchKernelGGL(fill_int_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

#define SDL_INST(T)                                                                                            \
  template hipError_t launch_tmod_solve<T>(const double*, int, int, double*, int, int, double*, T*, double*, T*, \
                                           double*, int*, unsigned long long*, const RmseOut&, hipStream_t);  \
  template hipError_t launch_dict_prep<T>(const double*, int, int, T*, double*, T*, hipStream_t);             \
  template hipError_t launch_rescale<T>(int, int, int, int64_t, const int32_t*, T*, const double*,            \
                                        hipStream_t);                                                         \
  template hipError_t launch_rmse<T>(const T*, int64_t, double, double*, int, double*, int, int, int*,        \
                                     hipStream_t);                                                            \
  template hipError_t launch_check_finite<T>(const T*, int64_t, int*, hipStream_t);                          \
  template hipError_t launch_sum_res2<T>(const T*, int64_t, double*, int, double*, hipStream_t);
SDL_INST(float)
SDL_INST(double)
#undef SDL_INST

}  // namespace sdl
