// Orthonormal variant of the method (Remark 1): square dictionaries with orthonormal columns
// (n1 = m1, n2 = m2).  Sparse coding needs no least squares: X_k = T_s(D1^T Y_k D2), the s
// entries of largest magnitude.  The dictionary update is the orthogonal Procrustes solution:
// the polar factor U V^T of the update's B sum (sum_k Y_k D2 X_k^T for D1, sum_k Y_k^T D1 X_k
// for D2), here by one-sided Jacobi rotations on one wave in FP64.
//
// Codes: a wave codes four signals, sixteen lanes per signal.  The signals are staged in LDS;
// V = Y D2 and C = D1^T V are formed entry by entry (lane l of the signal owns entries
// e = l + 16 u), C stays in registers, and s rounds of a 16-lane argmax (exact magnitude
// comparison, ties to the smaller atom) take the largest entries in decreasing order.  The
// residual energy comes from the explicit residual, as in the oracle.
#include <limits.h>
#include <math.h>

#include "sdl_internal.h"

namespace sdl {
namespace {

constexpr int kOWaves = 4;
constexpr int kOLanes = 16;  // lanes per signal
constexpr int kOSigs = 4;    // signals per wave
constexpr int kOMaxPer = 16;  // entries of C per lane (m1 m2 <= 256)
constexpr int kOMaxBlocks = 4096;

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ inline T sig_load(const OmpArgs<T>& a, int64_t e) {
  return a.Y[e];
}

// Cross-lane moves inside a row of 16 lanes by DPP (no LDS round trip): quad swaps (lane xor 1,
// xor 2), half-row mirror (lane i <-> 7 - i within each 8) and row mirror (i <-> 15 - i).  After
// the four steps of a commutative, associative combine every lane of the row holds the row's
// result.
constexpr int kDppX1 = 0xB1, kDppX2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;
template <int CTRL>
__device__ inline int dpp_int(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL, typename U>
__device__ inline U dpp_move(U v) {
  if constexpr (sizeof(U) == 4) {
    return __builtin_bit_cast(U, dpp_int<CTRL>(__builtin_bit_cast(int, v)));
  } else {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = dpp_int<CTRL>((int)(b & 0xffffffffll)), hi = dpp_int<CTRL>((int)(b >> 32));
    return __builtin_bit_cast(U, ((long long)hi << 32) | (unsigned int)lo);
  }
}
template <typename U>
__device__ inline U row16_sum(U v) {
  v += dpp_move<kDppX1>(v);
  v += dpp_move<kDppX2>(v);
  v += dpp_move<kDppHalfMirror>(v);
  v += dpp_move<kDppMirror>(v);
  return v;
}
// (value, index) maximum over the row, ties to the smaller index
template <int CTRL, typename U>
__device__ inline void argmax_step(U& v, int& idx) {
  const U ov = dpp_move<CTRL>(v);
  const int oi = dpp_int<CTRL>(idx);
  const bool take = ov > v || (ov == v && oi < idx);
  v = take ? ov : v;
  idx = take ? oi : idx;
}
template <typename U>
__device__ inline void row16_argmax(U& v, int& idx) {
  argmax_step<kDppX1>(v, idx);
  argmax_step<kDppX2>(v, idx);
  argmax_step<kDppHalfMirror>(v, idx);
  argmax_step<kDppMirror>(v, idx);
}
template <typename U>
__device__ inline U lane_value(U v, int k) {  // value of lane k (k uniform)
  if constexpr (sizeof(U) == 4) {
    return __builtin_bit_cast(U, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), k));
  } else {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __builtin_bit_cast(U, ((long long)hi << 32) | (unsigned int)lo);
  }
}

template <typename T>
__global__ void __launch_bounds__(kWave* kOWaves) ortho_code_kernel(OmpArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int m1 = a.m1, m2 = a.m2, M = m1 * m2, s = a.s;
  T* sD1 = reinterpret_cast<T*>(smem_raw);  // m1 x m1
  T* sD2 = sD1 + m1 * m1;                    // m2 x m2
  T* wsY = sD2 + m2 * m2;                    // [kOWaves][kOSigs][M] signals
  T* wsV = wsY + (size_t)kOWaves * kOSigs * M;  // [kOWaves][kOSigs][M] Y D2
  T* wsC = wsV + (size_t)kOWaves * kOSigs * M;  // [kOWaves][kOSigs][32] chosen values
  int* wsA = reinterpret_cast<int*>(wsC + (size_t)kOWaves * kOSigs * 32);  // [..][32] chosen atoms
  const int tid = threadIdx.x, wv = tid / kWave, lane = tid % kWave;
  const int g = lane / kOLanes, l = lane % kOLanes;
  for (int e = tid; e < m1 * m1; e += blockDim.x) sD1[e] = a.D1[e];
  for (int e = tid; e < m2 * m2; e += blockDim.x) sD2[e] = a.D2[e];
  __syncthreads();
  T* ys = wsY + (size_t)(wv * kOSigs + g) * M;
  T* vs = wsV + (size_t)(wv * kOSigs + g) * M;
  T* cs = wsC + (size_t)(wv * kOSigs + g) * 32;
  int* as = wsA + (size_t)(wv * kOSigs + g) * 32;
  const int64_t ngroups = (a.N + kOSigs - 1) / kOSigs;
  const int nper = (M + kOLanes - 1) / kOLanes;
  for (int64_t grp = (int64_t)blockIdx.x * kOWaves + wv; grp < ngroups; grp += (int64_t)gridDim.x * kOWaves) {
    const int64_t k = grp * kOSigs + g;
    const bool valid = k < a.N;
    for (int e = l; e < M; e += kOLanes) ys[e] = valid ? sig_load(a, k * M + e) : T(0);
    wave_sync();
    // V = Y D2: entry (p, j) at p + m1 j
    for (int e = l; e < M; e += kOLanes) {
      const int p = e % m1, j = e / m1;
      T v = 0;
      for (int q = 0; q < m2; ++q) v += ys[p + m1 * q] * sD2[q + m2 * j];
      vs[e] = v;
    }
    wave_sync();
    // C = D1^T V: entry (i, j), atom a = i + m1 j, owned by lane a % 16
    T cv[kOMaxPer];
#pragma unroll
    for (int u = 0; u < kOMaxPer; ++u) {
      const int e = l + kOLanes * u;
      T v = 0;
      if (u < nper && e < M) {
        const int i = e % m1, j = e / m1;
        for (int p = 0; p < m1; ++p) v += sD1[p + m1 * i] * vs[p + m1 * j];
      }
      cv[u] = v;
    }
    unsigned taken = 0u;  // bit u: entry u of this lane already chosen
    for (int t = 0; t < s; ++t) {
      // this lane's largest remaining |C| (ties: smaller atom, i.e. smaller u)
      T best = T(-1);
      int ba = INT_MAX;
#pragma unroll
      for (int u = 0; u < kOMaxPer; ++u) {
        const int e = l + kOLanes * u;
        const T m = fabs(cv[u]);
        const bool ok = u < nper && e < M && !((taken >> u) & 1u) && m > best;
        best = ok ? m : best;
        ba = ok ? e : ba;
      }
      // across the signal's 16 lanes (one DPP row)
      row16_argmax(best, ba);
      // the owner lane marks it and provides the signed value
      T val = 0;
      if (ba != INT_MAX && ba % kOLanes == l) {
        const int u = ba / kOLanes;
#pragma unroll
        for (int uu = 0; uu < kOMaxPer; ++uu) val = uu == u ? cv[uu] : val;
        taken |= 1u << u;
      }
      val = row16_sum(val);  // only the owner is nonzero
      if (valid && l == 0) {
        a.supp[k * s + t] = ba == INT_MAX ? -1 : ba;
        a.coef[k * s + t] = ba == INT_MAX ? T(0) : val;
      }
      // the chosen values for the residual
      if (l == 0) {
        cs[t] = val;
        as[t] = ba == INT_MAX ? -1 : ba;
      }
    }
    wave_sync();
    // explicit residual energy
    T rr = 0;
    for (int e = l; e < M; e += kOLanes) {
      const int p = e % m1, q = e / m1;
      T r = ys[e];
      for (int t = 0; t < s; ++t) {
        const int at = as[t];
        if (at >= 0) r -= cs[t] * sD1[p + m1 * (at % m1)] * sD2[q + m2 * (at / m1)];
      }
      rr += r * r;
    }
    rr = row16_sum(rr);
    if (valid && l == 0 && a.res2) a.res2[k] = rr;
    wave_sync();
  }
}

// One wave: the last stage of the fixed-order reduction of the partial rows (row stride ld),
// then the polar factor of B (the n x n block of the sums after A) by one-sided Jacobi
// rotations (n <= 8: four disjoint column pairs at a time in round-robin order; larger n: lane x
// holds row x, pairs in cyclic row order as the oracle), and the new dictionary D = U V^T with
// its compute-type copy and Gram matrix.  A rank-deficient B
// leaves the dictionary unchanged and sets the singular status.
template <typename T>
__global__ void __launch_bounds__(kWave) procrustes_kernel(const double* __restrict__ src, int nrow, int ld, int n,
                                                           double* D, T* Dc, double* G64, T* Gc, int* status,
                                                           unsigned long long* counters) {
  __shared__ double W[SDL_ORTHO_MAX_N * SDL_ORTHO_MAX_N];  // column-major n x n
  __shared__ double V[SDL_ORTHO_MAX_N * SDL_ORTHO_MAX_N];
  __shared__ double Dn[SDL_ORTHO_MAX_N * SDL_ORTHO_MAX_N];
  __shared__ double sig[SDL_ORTHO_MAX_N];
  const int x = threadIdx.x;
  const int nent = n * n;
  for (int e = x; e < nent; e += kWave) {
    // B follows A in the row; eight rows' loads in flight, added in row order
    double v = 0.0;
    int b = 0;
    for (; b + 8 <= nrow; b += 8) {
      double q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) q[u] = src[(size_t)(b + u) * ld + nent + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) v += q[u];
    }
    for (; b < nrow; ++b) v += src[(size_t)b * ld + nent + e];
    W[e] = v;
    V[e] = (e % n) == (e / n) ? 1.0 : 0.0;
  }
  wave_sync();
  const bool row = x < n;
  if (n <= 8) {
    // Up to four disjoint column pairs rotated at once (round-robin order: n' - 1 rounds of n' / 2
    // pairs cover every pair once per sweep, n' = n rounded up to even, pairs with the dummy
    // column n skipped); lane 8 q + r holds row r for the q-th pair of the round.  The polar
    // factor is unique for a full-rank B, so the order of the rotations changes only rounding.
    const int np = n + (n & 1), q = x / 8, r = x % 8;
    for (int sweep = 0; sweep < 60; ++sweep) {
      bool rotated = false;
      for (int round = 0; round < np - 1; ++round) {
        int i = -1, j = -1;
        if (q < np / 2) {
          if (q == 0) {
            i = np - 1;
            j = round;
          } else {
            i = (round + q) % (np - 1);
            j = (round - q + np - 1) % (np - 1);
          }
          if (i > j) { const int tmp = i; i = j; j = tmp; }
        }
        const bool act = j >= 0 && j < n;  // a real pair (the dummy column is n)
        double pa = 0.0, pb = 0.0, pg = 0.0;
        if (act && r < n) {
          const double wi = W[r + n * i], wj = W[r + n * j];
          pa = wi * wi;
          pb = wj * wj;
          pg = wi * wj;
        }
        // sums over the pair's eight lanes (quad swaps and the half-row mirror)
        pa += dpp_move<kDppX1>(pa);
        pb += dpp_move<kDppX1>(pb);
        pg += dpp_move<kDppX1>(pg);
        pa += dpp_move<kDppX2>(pa);
        pb += dpp_move<kDppX2>(pb);
        pg += dpp_move<kDppX2>(pg);
        pa += dpp_move<kDppHalfMirror>(pa);
        pb += dpp_move<kDppHalfMirror>(pb);
        pg += dpp_move<kDppHalfMirror>(pg);
        const bool rot = act && !(fabs(pg) <= 1e-15 * sqrt(pa * pb) || pg == 0.0);
        if (rot) {
          const double zeta = (pb - pa) / (2.0 * pg);
          const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
          if (r < n) {
            const double wi = W[r + n * i], wj = W[r + n * j];
            W[r + n * i] = c * wi - sn * wj;
            W[r + n * j] = sn * wi + c * wj;
            const double vi = V[r + n * i], vj = V[r + n * j];
            V[r + n * i] = c * vi - sn * vj;
            V[r + n * j] = sn * vi + c * vj;
          }
        }
        rotated = rotated || rot;
        wave_sync();
      }
      if (__ballot(rotated) == 0ull) break;
    }
  } else for (int sweep = 0; sweep < 60; ++sweep) {
    int rotated = 0;
    for (int i = 0; i < n - 1; ++i)
      for (int j = i + 1; j < n; ++j) {
        double pa = 0.0, pb = 0.0, pg = 0.0;
        if (row) {
          const double wi = W[x + n * i], wj = W[x + n * j];
          pa = wi * wi;
          pb = wj * wj;
          pg = wi * wj;
        }
        // sums over the n <= 32 rows in a fixed order: each 16-lane row by DPP, then rows 0 and
        // 1 added from their first lanes (uniform values: every lane takes the same decision)
        pa = row16_sum(pa);
        pb = row16_sum(pb);
        pg = row16_sum(pg);
        pa = n > 16 ? lane_value(pa, 0) + lane_value(pa, 16) : lane_value(pa, 0);
        pb = n > 16 ? lane_value(pb, 0) + lane_value(pb, 16) : lane_value(pb, 0);
        pg = n > 16 ? lane_value(pg, 0) + lane_value(pg, 16) : lane_value(pg, 0);
        if (fabs(pg) <= 1e-15 * sqrt(pa * pb) || pg == 0.0) continue;
        rotated = 1;
        const double zeta = (pb - pa) / (2.0 * pg);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
        if (row) {
          const double wi = W[x + n * i], wj = W[x + n * j];
          W[x + n * i] = c * wi - sn * wj;
          W[x + n * j] = sn * wi + c * wj;
          const double vi = V[x + n * i], vj = V[x + n * j];
          V[x + n * i] = c * vi - sn * vj;
          V[x + n * j] = sn * vi + c * vj;
        }
        wave_sync();
      }
    if (!rotated) break;
  }
  wave_sync();
  if (row) {
    double v = 0.0;
    for (int r = 0; r < n; ++r) v += W[r + n * x] * W[r + n * x];
    sig[x] = sqrt(v);
  }
  wave_sync();
  double smax = 0.0;
  for (int i = 0; i < n; ++i) smax = fmax(smax, sig[i]);
  bool ok = true;
  for (int i = 0; i < n; ++i) ok = ok && sig[i] > 1e-12 * smax;
  if (!ok) {
    if (x == 0) {
      atomicOr(status, kStatusSingular);
      atomicAdd(&counters[kCtrSingular], 1ull);
    }
    return;
  }
  // D[x][c] = sum_i (W[x][i] / sigma_i) V[c][i]
  if (row)
    for (int c = 0; c < n; ++c) {
      double v = 0.0;
      for (int i = 0; i < n; ++i) v += (W[x + n * i] / sig[i]) * V[c + n * i];
      Dn[x + n * c] = v;
      D[x + n * c] = v;
      Dc[x + n * c] = (T)v;
    }
  wave_sync();
  if (row)
    for (int c = 0; c < n; ++c) {
      double v = 0.0;
      for (int r = 0; r < n; ++r) v += Dn[r + n * x] * Dn[r + n * c];
      G64[x + n * c] = v;
      Gc[x + n * c] = (T)v;
    }
}

size_t ortho_lds(int m1, int m2, size_t elem) {
  const int M = m1 * m2;
  return elem * ((size_t)m1 * m1 + (size_t)m2 * m2 + 2 * (size_t)kOWaves * kOSigs * M + (size_t)kOWaves * kOSigs * 32) +
         4 * (size_t)kOWaves * kOSigs * 32;
}

}  // namespace

bool ortho_supported(int m1, int m2, int n1, int n2, int s) {
  return n1 == m1 && n2 == m2 && m1 <= SDL_ORTHO_MAX_N && m2 <= SDL_ORTHO_MAX_N && m1 * m2 <= kOLanes * kOMaxPer &&
         s <= 32 && s <= m1 * m2;
}

template <typename T>
hipError_t launch_ortho_code(const OmpArgs<T>& a, hipStream_t st) {
  if (a.N == 0) return hipSuccess;
  const int64_t ngroups = (a.N + kOSigs - 1) / kOSigs;
  int64_t blocks = (ngroups + kOWaves - 1) / kOWaves;
  if (blocks > kOMaxBlocks) blocks = kOMaxBlocks;
  hipLaunchKernelGGL(ortho_code_kernel<T>, dim3((unsigned)blocks), dim3(kWave * kOWaves), ortho_lds(a.m1, a.m2, sizeof(T)),
                     st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_procrustes(const double* src, int nrow, int ld, int n, double* D, T* Dc, double* G64, T* Gc,
                             int* status, unsigned long long* counters, hipStream_t st) {
  hipLaunchKernelGGL(procrustes_kernel<T>, dim3(1), dim3(kWave), 0, st, src, nrow, ld, n, D, Dc, G64, Gc, status,
                     counters);
  return hipGetLastError();
}

hipError_t ortho_init_device() {
  const int bytes = 160 * 1024;  // at most ortho_lds(32, 8, 8), about 75 KiB
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&ortho_code_kernel<float>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&ortho_code_kernel<double>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template hipError_t launch_ortho_code<float>(const OmpArgs<float>&, hipStream_t);
template hipError_t launch_ortho_code<double>(const OmpArgs<double>&, hipStream_t);
template hipError_t launch_procrustes<float>(const double*, int, int, int, double*, float*, double*, float*, int*,
                                             unsigned long long*, hipStream_t);
template hipError_t launch_procrustes<double>(const double*, int, int, int, double*, double*, double*, double*, int*,
                                              unsigned long long*, hipStream_t);

}  // namespace sdl
