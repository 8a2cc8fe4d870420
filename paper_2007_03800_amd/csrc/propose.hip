// Learned support proposal, inference side: logits -> s atoms -> least squares.
//
// Sixteen lanes share a signal (four signals per wave): each lane holds every 16th
// logit, s rounds of a group arg-max (ties -> smallest atom index) pick the atoms in
// decreasing logit order, then the group solves the least-squares problem on them with
// the same Gram entries G1[i,i'] G2[j,j'] as 2D-OMP (Cholesky in FP32 registers,
// redundantly per lane), forms the residual explicitly and flags the proposal as
// accepted when ||r||^2 <= tau * ||Y||^2.  Rejected signals are listed (ascending) for
// the 2D-OMP fallback by a deterministic three-pass compaction.
#include <limits.h>
#include <math.h>

#include "mlp_internal.h"

namespace sdl {
namespace {

constexpr int kGroup = 16;

__device__ inline float group16_sum(float v) {
#pragma unroll
  for (int o = 1; o < kGroup; o <<= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

template <int VPL, int SMAX>
__global__ void __launch_bounds__(256) propose_kernel(ProposeArgs a) {
  extern __shared__ __align__(16) float sm[];
  const int m1 = a.m1, m2 = a.m2, n1 = a.n1, n2 = a.n2, s = a.s, M = m1 * m2, A = n1 * n2;
  float* sG1 = sm;
  float* sG2 = sG1 + n1 * n1;
  float* sD1 = sG2 + n2 * n2;
  float* sD2 = sD1 + m1 * n1;
  for (int e = threadIdx.x; e < n1 * n1; e += blockDim.x) sG1[e] = a.G1[e];
  for (int e = threadIdx.x; e < n2 * n2; e += blockDim.x) sG2[e] = a.G2[e];
  for (int e = threadIdx.x; e < m1 * n1; e += blockDim.x) sD1[e] = a.D1[e];
  for (int e = threadIdx.x; e < m2 * n2; e += blockDim.x) sD2[e] = a.D2[e];
  __syncthreads();
  const int sub = threadIdx.x % kGroup;
  const int64_t k = (int64_t)blockIdx.x * (blockDim.x / kGroup) + threadIdx.x / kGroup;
  const bool valid = k < a.N;

  float v[VPL];
#pragma unroll
  for (int u = 0; u < VPL; ++u) v[u] = valid ? a.logits[k * A + sub + kGroup * u] : -INFINITY;
  int sel[SMAX];
#pragma unroll
  for (int t = 0; t < SMAX; ++t) {
    sel[t] = 0;
    if (t < s) {
      float bv = -INFINITY;
      int ba = INT_MAX;
#pragma unroll
      for (int u = 0; u < VPL; ++u) {
        const bool c = v[u] > bv;
        bv = c ? v[u] : bv;
        ba = c ? sub + kGroup * u : ba;
      }
#pragma unroll
      for (int o = 1; o < kGroup; o <<= 1) {
        const float ov = __shfl_xor(bv, o, kWave);
        const int oa = __shfl_xor(ba, o, kWave);
        const bool c = ov > bv || (ov == bv && oa < ba);
        bv = c ? ov : bv;
        ba = c ? oa : ba;
      }
      sel[t] = ba < A ? ba : 0;
#pragma unroll
      for (int u = 0; u < VPL; ++u) v[u] = (sub + kGroup * u == ba) ? -INFINITY : v[u];
    }
  }
  // least squares on the proposed support
  const float* y = a.Y + (valid ? k : 0) * M;
  float yl[4];
  float yy = 0.f;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const int e = sub + kGroup * w;
    yl[w] = (valid && e < M) ? y[e] : 0.f;
    yy += yl[w] * yl[w];
  }
  yy = group16_sum(yy);
  float cs[SMAX], x[SMAX];
#pragma unroll
  for (int t = 0; t < SMAX; ++t) {
    cs[t] = 0.f;
    if (t < s) {
      const int i = sel[t] % n1, j = sel[t] / n1;
      float c = 0.f;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int e = sub + kGroup * w;
        if (e < M) c += yl[w] * sD1[e % m1 + m1 * i] * sD2[e / m1 + m2 * j];
      }
      cs[t] = group16_sum(c);
    }
  }
  // Cholesky of the support Gram matrix (packed lower triangle), then L L^T x = cs
  float L[SMAX * (SMAX + 1) / 2];
  bool ok = valid;
#pragma unroll
  for (int t = 0; t < SMAX; ++t) {
    if (t < s) {
      const int it = sel[t] % n1, jt = sel[t] / n1;
#pragma unroll
      for (int u = 0; u <= t; ++u) {
        const int iu = sel[u] % n1, ju = sel[u] / n1;
        float g = sG1[it + n1 * iu] * sG2[jt + n2 * ju];
#pragma unroll
        for (int l = 0; l < u; ++l) g -= L[t * (t + 1) / 2 + l] * L[u * (u + 1) / 2 + l];
        if (u < t) {
          L[t * (t + 1) / 2 + u] = g / L[u * (u + 1) / 2 + u];
        } else {
          const float gaa = sG1[it + n1 * it] * sG2[jt + n2 * jt];
          ok = ok && g > 1e-6f * gaa;
          L[t * (t + 1) / 2 + t] = g > 0.f ? sqrtf(g) : 1.f;
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < SMAX; ++t) {
    x[t] = 0.f;
    if (t < s) {
      float b = cs[t];
#pragma unroll
      for (int l = 0; l < t; ++l) b -= L[t * (t + 1) / 2 + l] * x[l];
      x[t] = b / L[t * (t + 1) / 2 + t];
    }
  }
#pragma unroll
  for (int t = SMAX - 1; t >= 0; --t) {
    if (t < s) {
      float b = x[t];
#pragma unroll
      for (int l = t + 1; l < SMAX; ++l)
        if (l < s) b -= L[l * (l + 1) / 2 + t] * x[l];
      x[t] = b / L[t * (t + 1) / 2 + t];
    }
  }
  float rr = 0.f;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const int e = sub + kGroup * w;
    if (e < M) {
      float r = yl[w];
#pragma unroll
      for (int t = 0; t < SMAX; ++t)
        if (t < s) r -= x[t] * sD1[e % m1 + m1 * (sel[t] % n1)] * sD2[e / m1 + m2 * (sel[t] / n1)];
      rr += r * r;
    }
  }
  rr = group16_sum(rr);
  if (valid) {
#pragma unroll
    for (int t = 0; t < SMAX; ++t) {
      if (t < s && t % kGroup == sub) {
        a.supp[k * s + t] = sel[t];
        a.coef[k * s + t] = ok ? x[t] : 0.f;
      }
    }
    if (sub == 0) {
      if (a.res2) a.res2[k] = rr;
      a.accept[k] = (ok && (double)rr <= a.tau * (double)yy) ? 1 : 0;
    }
  }
}

constexpr int kCompact = 1024;  // signals per compaction block

__global__ void __launch_bounds__(kCompact) compact_count_kernel(const int32_t* accept, int64_t N, int32_t* blkcount) {
  __shared__ int wc[kCompact / 64];
  const int64_t k = (int64_t)blockIdx.x * kCompact + threadIdx.x;
  const bool rej = k < N && accept[k] == 0;
  const unsigned long long b = __ballot(rej);
  if (threadIdx.x % 64 == 0) wc[threadIdx.x / 64] = __popcll(b);
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kCompact / 64; ++w) t += wc[w];
    blkcount[blockIdx.x] = t;
  }
}

__global__ void compact_scan_kernel(int32_t* blkcount, int nblk, int32_t* count) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int run = 0;
  for (int b = 0; b < nblk; ++b) {
    const int c = blkcount[b];
    blkcount[b] = run;
    run += c;
  }
  *count = run;
}

__global__ void __launch_bounds__(kCompact) compact_write_kernel(const int32_t* accept, int64_t N, const int32_t* offs,
                                                                 int32_t* list) {
  __shared__ int wc[kCompact / 64];
  const int64_t k = (int64_t)blockIdx.x * kCompact + threadIdx.x;
  const bool rej = k < N && accept[k] == 0;
  const unsigned long long b = __ballot(rej);
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  if (lane == 0) wc[w] = __popcll(b);
  __syncthreads();
  int base = offs[blockIdx.x];
  for (int q = 0; q < w; ++q) base += wc[q];
  if (rej) list[base + __popcll(b & ((1ull << lane) - 1ull))] = (int32_t)k;
}

template <int VPL, int SMAX>
hipError_t launch_vs(const ProposeArgs& a, hipStream_t st) {
  const size_t lds = sizeof(float) * (a.n1 * a.n1 + a.n2 * a.n2 + a.m1 * a.n1 + a.m2 * a.n2);
  const int64_t blocks = (a.N + 15) / 16;
  hipLaunchKernelGGL((propose_kernel<VPL, SMAX>), dim3((unsigned)blocks), dim3(256), lds, st, a);
  return hipGetLastError();
}

}  // namespace

bool propose_supported(int n1, int n2, int s) {
  const int A = n1 * n2;
  return (A == 256 || A == 144) && s >= 1 && s <= 16 && n1 <= 64 && n2 <= 64;
}

hipError_t launch_propose(const ProposeArgs& a, hipStream_t st) {
  if (a.N == 0) return hipSuccess;
  if (a.m1 * a.m2 > 4 * kGroup) return hipErrorInvalidValue;
  const int A = a.n1 * a.n2;
  if (A == 256) return a.s <= 8 ? launch_vs<16, 8>(a, st) : launch_vs<16, 16>(a, st);
  if (A == 144) return a.s <= 8 ? launch_vs<9, 8>(a, st) : launch_vs<9, 16>(a, st);
  return hipErrorInvalidValue;
}

int compact_blocks(int64_t N) { return (int)((N + kCompact - 1) / kCompact); }

hipError_t launch_compact_rejected(const int32_t* accept, int64_t N, int32_t* blkcount, int32_t* list, int32_t* count,
                                   hipStream_t st) {
  const int nblk = compact_blocks(N);
  if (nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(compact_count_kernel, dim3(nblk), dim3(kCompact), 0, st, accept, N, blkcount);
  hipLaunchKernelGGL(compact_scan_kernel, dim3(1), dim3(64), 0, st, blkcount, nblk, count);
  hipLaunchKernelGGL(compact_write_kernel, dim3(nblk), dim3(kCompact), 0, st, accept, N, blkcount, list);
  return hipGetLastError();
}

}  // namespace sdl
