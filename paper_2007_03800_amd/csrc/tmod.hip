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

constexpr int kSumThreads = 256;
constexpr int kMaxEntPerThread = 32;  // (na^2 + mr*na) / 256 for na, mr <= 64

template <typename T>
__global__ void __launch_bounds__(kSumThreads) tmod_sums_kernel(TmodArgs<T> a, double* part, int nblk, int bs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int side = a.side, n1 = a.n1, s = a.s;
  const int na = side == 1 ? a.n1 : a.n2;
  const int mr = side == 1 ? a.m1 : a.m2;  // rows of Yt
  const int mc = side == 1 ? a.m2 : a.m1;  // cols of Yt (= rows of Do)
  const int M = a.m1 * a.m2;
  const int nent = na * na + mr * na;
  T* Tb = sm;                    // bs x na x mc
  T* Yb = Tb + bs * na * mc;     // bs x mr x mc  (Yt[r][c] at r*mc + c)
  const int tid = threadIdx.x;
  const int64_t k0 = (a.N * blockIdx.x) / nblk, k1 = (a.N * (blockIdx.x + 1)) / nblk;

  T acc[kMaxEntPerThread];
#pragma unroll
  for (int u = 0; u < kMaxEntPerThread; ++u) acc[u] = 0;

  for (int64_t kb = k0; kb < k1; kb += bs) {
    const int nb = (int)((k1 - kb) < bs ? (k1 - kb) : bs);
    for (int e = tid; e < bs * na * mc; e += kSumThreads) Tb[e] = 0;
    for (int e = tid; e < bs * M; e += kSumThreads) {
      const int b = e / M, pix = e % M;
      T v = 0;
      if (b < nb) v = a.Y[(kb + b) * M + pix];
      const int p = pix % a.m1, q = pix / a.m1;  // Y[p, q]
      const int r = side == 1 ? p : q, c = side == 1 ? q : p;
      Yb[b * mr * mc + r * mc + c] = v;
    }
    __syncthreads();
    for (int e = tid; e < nb * mc; e += kSumThreads) {
      const int b = e / mc, c = e % mc;
      const int64_t k = kb + b;
      for (int t = 0; t < s; ++t) {
        const int at = a.supp[k * s + t];
        if (at < 0) continue;
        const int i = at % n1, j = at / n1;
        const int ra = side == 1 ? i : j, rb = side == 1 ? j : i;
        Tb[(b * na + ra) * mc + c] += a.coef[k * s + t] * a.Dother[c + mc * rb];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kMaxEntPerThread; ++u) {
      const int e = tid + u * kSumThreads;
      if (e < nent) {
        T v = acc[u];
        if (e < na * na) {
          const int r1 = e % na, r2 = e / na;
          for (int b = 0; b < nb; ++b) {
            const T* t1 = Tb + (b * na + r1) * mc;
            const T* t2 = Tb + (b * na + r2) * mc;
            for (int c = 0; c < mc; ++c) v += t1[c] * t2[c];
          }
        } else {
          const int f = e - na * na;
          const int r = f % mr, ra = f / mr;
          for (int b = 0; b < nb; ++b) {
            const T* yr = Yb + b * mr * mc + r * mc;
            const T* tr = Tb + (b * na + ra) * mc;
            for (int c = 0; c < mc; ++c) v += yr[c] * tr[c];
          }
        }
        acc[u] = v;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < kMaxEntPerThread; ++u) {
    const int e = tid + u * kSumThreads;
    if (e < nent) part[(size_t)blockIdx.x * nent + e] = (double)acc[u];
  }
}

__global__ void reduce_partials_kernel(const double* __restrict__ part, int nblk, int nent, double* out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nent) return;
  double v = 0.0;
  for (int b = 0; b < nblk; ++b) v += part[(size_t)b * nent + e];
  out[e] = v;
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

constexpr int kSolveThreads = 256;
constexpr double kSpdRelTol = 1e-12;  // pivot <= tol * diagonal entry -> not positive definite

// sums = [A (na x na) | B (mr x na)], both column-major.
template <typename T>
__global__ void __launch_bounds__(kSolveThreads)
    tmod_solve_kernel(const double* sums, int mr, int na, double* D, T* Dc, double* G64, T* Gc, double* w,
                      int* status, unsigned long long* counters) {
  __shared__ double C[SDL_MAX_N * SDL_MAX_N];
  __shared__ double Xs[SDL_MAX_M * SDL_MAX_N];  // solution D*, mr x na column-major
  __shared__ double diag0[SDL_MAX_N];
  __shared__ int U[SDL_MAX_N];
  __shared__ int nu_s, bad_s;
  const int tid = threadIdx.x;
  const double* A = sums;
  const double* B = sums + na * na;
  if (tid == 0) {
    int nu = 0;
    for (int i = 0; i < na; ++i)
      if (A[i + na * i] > 0.0) U[nu++] = i;
    nu_s = nu;
    bad_s = 0;
    if (nu < na) atomicAdd(&counters[kCtrUnusedAtoms], (unsigned long long)(na - nu));
  }
  __syncthreads();
  const int nu = nu_s;
  // compacted Gram sum on the used atoms (the system decouples exactly for unused ones)
  for (int e = tid; e < nu * nu; e += kSolveThreads) {
    const int k = e % nu, l = e / nu;
    C[k * nu + l] = A[U[k] + na * U[l]];
    if (k == l) diag0[k] = A[U[k] + na * U[k]];
  }
  __syncthreads();
  // right-looking Cholesky, lower triangle of C (row-major, ld nu)
  for (int k = 0; k < nu; ++k) {
    if (tid == 0) {
      const double d = C[k * nu + k];
      if (!(d > kSpdRelTol * diag0[k])) bad_s = 1;
      else C[k * nu + k] = sqrt(d);
    }
    __syncthreads();
    if (bad_s) break;
    const double lkk = C[k * nu + k];
    for (int i = k + 1 + tid; i < nu; i += kSolveThreads) C[i * nu + k] /= lkk;
    __syncthreads();
    const int rem = nu - k - 1;
    for (int e = tid; e < rem * rem; e += kSolveThreads) {
      const int i = k + 1 + e % rem, j = k + 1 + e / rem;
      if (j <= i) C[i * nu + j] -= C[i * nu + k] * C[j * nu + k];
    }
    __syncthreads();
  }
  const bool bad = bad_s != 0;
  if (!bad) {
    // D* A_UU = B_U  <=>  A_UU (row p of D*)^T = (row p of B_U)^T; one thread per row p
    for (int p = tid; p < mr; p += kSolveThreads) {
      double* x = Xs + p;  // stride mr over atoms
      for (int k = 0; k < nu; ++k) {
        double v = B[p + mr * U[k]];
        for (int l = 0; l < k; ++l) v -= C[k * nu + l] * x[mr * l];
        x[mr * k] = v / C[k * nu + k];
      }
      for (int k = nu - 1; k >= 0; --k) {
        double v = x[mr * k];
        for (int l = k + 1; l < nu; ++l) v -= C[l * nu + k] * x[mr * l];
        x[mr * k] = v / C[k * nu + k];
      }
    }
    __syncthreads();
    // normalise the solved atoms (W); zero or unused columns keep the old atom
    for (int i = tid; i < na; i += kSolveThreads) w[i] = 1.0;
    __syncthreads();
    for (int k = tid; k < nu; k += kSolveThreads) {
      const int i = U[k];
      double nrm = 0.0;
      for (int p = 0; p < mr; ++p) nrm += Xs[p + mr * k] * Xs[p + mr * k];
      nrm = sqrt(nrm);
      if (nrm > 0.0) {
        w[i] = nrm;
        for (int p = 0; p < mr; ++p) D[p + mr * i] = Xs[p + mr * k] / nrm;
      }
    }
  } else {
    for (int i = tid; i < na; i += kSolveThreads) w[i] = 1.0;
    if (tid == 0) {
      atomicOr(status, kStatusSingular);
      atomicAdd(&counters[kCtrSingular], 1ull);
    }
  }
  __threadfence_block();
  __syncthreads();
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

int tmod_num_blocks(int64_t N) {
  // ~64+ signals per workgroup, at most 2048 workgroups (8 per CU)
  int64_t b = (N + 63) / 64;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

template <typename T>
hipError_t launch_tmod_sums(const TmodArgs<T>& a, double* part, int nblk, hipStream_t st) {
  const int na = a.side == 1 ? a.n1 : a.n2;
  const int mr = a.side == 1 ? a.m1 : a.m2;
  const int mc = a.side == 1 ? a.m2 : a.m1;
  const int per = na * mc + mr * mc;  // elements per staged signal
  int bs = (int)(32768 / (per * sizeof(T)));
  if (bs > 16) bs = 16;
  if (bs < 1) bs = 1;
  const size_t lds = (size_t)bs * per * sizeof(T);
  hipLaunchKernelGGL(tmod_sums_kernel<T>, dim3(nblk), dim3(kSumThreads), lds, st, a, part, nblk, bs);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* part, int nblk, int nent, double* out, hipStream_t st) {
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((nent + 255) / 256), dim3(256), 0, st, part, nblk, nent, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tmod_solve(const double* sums, int mr, int na, double* D, T* Dc, double* G64, T* Gc, double* w,
                             int* status, unsigned long long* counters, hipStream_t st) {
  hipLaunchKernelGGL(tmod_solve_kernel<T>, dim3(1), dim3(kSolveThreads), 0, st, sums, mr, na, D, Dc, G64, Gc, w,
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
  template hipError_t launch_tmod_sums<T>(const TmodArgs<T>&, double*, int, hipStream_t);                    \
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
