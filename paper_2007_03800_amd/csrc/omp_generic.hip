// 2D-OMP sparse coding, generic shapes: one wave64 per signal, everything in LDS.
//
// Method (Sec. III step 1; Sec. II: 2D-OMP is OMP on D2 (x) D1 without forming it):
// for s steps, choose the unselected atom a = i + n1*j with the largest
// |corr_a| (ties: smallest a), then re-fit all chosen coefficients by least
// squares.  The least squares is carried by an incrementally grown Cholesky
// factor L of the support's Gram matrix, whose entries are G1[i,i'] * G2[j,j']
// with G1 = D1^T D1, G2 = D2^T D2 (the Gram identity stated after Algorithm 1).
//
// Correlations are kept in Gram form: corr starts as C = D1^T Y D2 and, when
// atom a joins with new Cholesky row [w^T, delta] (L w = G_{S,a},
// delta^2 = G_aa - |w|^2), the residual loses its component along the
// orthogonalised atom, so
//     corr <- corr - (corr_a / delta^2) * (G_{:,a} - G_{:,S} v),   v = L^{-T} w,
//     x_S  <- x_S  - (corr_a / delta^2) * v,   x_a = corr_a / delta^2.
// The residual and its squared norm are formed explicitly at the end.
//
// This is the shape-agnostic path (any m1, m2, n1, n2 <= 64, s <= 32 that fits LDS),
// used for FP64 and as the fallback for FP32; the register-resident kernel in
// omp_fast.hip covers the benchmark shapes.
#include <float.h>
#include <limits.h>

#include "sdl_internal.h"

namespace sdl {
namespace {

template <typename T>
struct Lay {
  // element offsets inside the dynamic LDS block (in units of T)
  int d1, d2, g1, g2, y, w, al, L, x, v, wv, end;
};

template <typename T>
__host__ __device__ inline Lay<T> layout(int m1, int m2, int n1, int n2, int s) {
  Lay<T> l;
  int o = 0;
  l.d1 = o; o += m1 * n1;
  l.d2 = o; o += m2 * n2;
  l.g1 = o; o += n1 * n1;
  l.g2 = o; o += n2 * n2;
  l.y = o; o += m1 * m2;
  l.w = o; o += n1 * m2;
  l.al = o; o += n1 * n2;
  l.L = o; o += s * s;
  l.x = o; o += s;
  l.v = o; o += s;
  l.wv = o; o += s;
  l.end = o;
  return l;
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// (value, index) maximum with ties to the smaller index; identical result in every lane.
template <typename T>
__device__ inline void wave_argmax(T& v, int& idx) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T ov = __shfl_xor(v, o, kWave);
    int oi = __shfl_xor(idx, o, kWave);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kWave) omp_generic_kernel(OmpArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int m1 = a.m1, m2 = a.m2, n1 = a.n1, n2 = a.n2, s = a.s;
  const int M = m1 * m2, A = n1 * n2;
  const Lay<T> L = layout<T>(m1, m2, n1, n2, s);
  int* supp_s = reinterpret_cast<int*>(sm + L.end);
  unsigned char* sel = reinterpret_cast<unsigned char*>(supp_s + s);
  const int lane = threadIdx.x;

  for (int e = lane; e < m1 * n1; e += kWave) sm[L.d1 + e] = a.D1[e];
  for (int e = lane; e < m2 * n2; e += kWave) sm[L.d2 + e] = a.D2[e];
  for (int e = lane; e < n1 * n1; e += kWave) sm[L.g1 + e] = a.G1[e];
  for (int e = lane; e < n2 * n2; e += kWave) sm[L.g2 + e] = a.G2[e];
  const T* D1s = sm + L.d1;
  const T* D2s = sm + L.d2;
  const T* G1s = sm + L.g1;
  const T* G2s = sm + L.g2;
  T* ys = sm + L.y;
  T* Ws = sm + L.w;
  T* al = sm + L.al;
  T* Ls = sm + L.L;
  T* xs = sm + L.x;
  T* vs = sm + L.v;
  T* wv = sm + L.wv;

  unsigned n_early = 0;  // early-stopped signals of this wave (lane 0), counted once at the end
  for (int64_t k = blockIdx.x; k < a.N; k += gridDim.x) {
    __syncthreads();
    T yy = 0;
    for (int e = lane; e < M; e += kWave) {
      const T v = a.Yh ? (T)bf16_to_float(a.Yh[k * M + e]) : a.Y[k * M + e];
      ys[e] = v;
      yy += v * v;
    }
    for (int e = lane; e < A; e += kWave) sel[e] = 0;
    const T yy_all = wave_sum(yy);
    const T ynorm = sqrt(yy_all);
    // residual energy, by the OMP recurrence ||r||^2 -= corr_a^2 / pivot per appended atom
    T renergy = yy_all;
    __syncthreads();
    // C = D1^T Y D2, as W = D1^T Y (n1 x m2) then W D2
    for (int e = lane; e < n1 * m2; e += kWave) {
      const int i = e % n1, q = e / n1;
      T v = 0;
      for (int p = 0; p < m1; ++p) v += D1s[p + m1 * i] * ys[p + m1 * q];
      Ws[e] = v;
    }
    __syncthreads();
    for (int e = lane; e < A; e += kWave) {
      const int i = e % n1, j = e / n1;
      T v = 0;
      for (int q = 0; q < m2; ++q) v += Ws[i + n1 * q] * D2s[q + m2 * j];
      al[e] = v;
    }
    __syncthreads();

    int t = 0;
    bool early = false;
    for (; t < s; ++t) {
      // error-driven stop (denoising runs, Sec. IV): no further atom once ||r||^2 <= err2
      if (a.err2 > 0.0 && !(renergy > T(a.err2))) {
        early = true;
        break;
      }
      // greedy choice
      T bv = T(-1);
      int bi = INT_MAX;
      for (int e = lane; e < A; e += kWave) {
        if (sel[e]) continue;
        T v = fabs(al[e]);
        if (v > bv) { bv = v; bi = e; }
      }
      wave_argmax(bv, bi);
      if (bi == INT_MAX || !(bv > T(a.stop_rel) * ynorm)) { early = true; break; }
      const int ia = bi % n1, ja = bi / n1;
      const T gaa = G1s[ia + n1 * ia] * G2s[ja + n2 * ja];
      // new Cholesky row: L w = G_{S,a}   (computed redundantly by every lane)
      T ww = 0;
      for (int q = 0; q < t; ++q) {
        const int iq = supp_s[q] % n1, jq = supp_s[q] / n1;
        T b = G1s[iq + n1 * ia] * G2s[jq + n2 * ja];
        for (int l = 0; l < q; ++l) b -= Ls[q * s + l] * wv[l];
        b /= Ls[q * s + q];
        wv[q] = b;
        ww += b * b;
      }
      T d2 = gaa - ww;
      if (sizeof(T) == 4 && d2 < T(a.pivot_fp64) * gaa) {
        // small pivot: recompute this row in FP64 (cancellation in G_aa - |w|^2)
        double w64[SDL_MAX_S];
        double acc = 0.0;
        for (int q = 0; q < t; ++q) {
          const int iq = supp_s[q] % n1, jq = supp_s[q] / n1;
          double b = (double)G1s[iq + n1 * ia] * (double)G2s[jq + n2 * ja];
          for (int l = 0; l < q; ++l) b -= (double)Ls[q * s + l] * w64[l];
          b /= (double)Ls[q * s + q];
          w64[q] = b;
          acc += b * b;
        }
        for (int q = 0; q < t; ++q) wv[q] = (T)w64[q];
        d2 = (T)((double)gaa - acc);
        if (lane == 0) atomicAdd(&a.counters[kCtrFp64Pivot], 1ull);
      }
      if (!(d2 > T(a.dep_eps) * gaa)) { early = true; break; }
      // v = L^{-T} w
      for (int q = t - 1; q >= 0; --q) {
        T b = wv[q];
        for (int l = q + 1; l < t; ++l) b -= Ls[l * s + q] * vs[l];
        vs[q] = b / Ls[q * s + q];
      }
      const T cstar = al[bi] / d2;
      renergy -= cstar * al[bi];
      __syncthreads();
      if (lane == 0) {
        for (int q = 0; q < t; ++q) {
          Ls[t * s + q] = wv[q];
          xs[q] -= cstar * vs[q];
        }
        Ls[t * s + t] = sqrt(d2);
        xs[t] = cstar;
        supp_s[t] = bi;
        sel[bi] = 1;
      }
      if (t + 1 < s) {
        // corr <- corr - cstar * (G_{:,a} - G_{:,S} v)
        for (int e = lane; e < A; e += kWave) {
          const int i = e % n1, j = e / n1;
          T g = G1s[i + n1 * ia] * G2s[ja + n2 * j];
          for (int q = 0; q < t; ++q) {
            const int iq = supp_s[q] % n1, jq = supp_s[q] / n1;
            g -= vs[q] * G1s[i + n1 * iq] * G2s[jq + n2 * j];
          }
          al[e] -= cstar * g;
        }
      }
      __syncthreads();
    }
    __syncthreads();
    // explicit residual Y - sum_t x_t d1_{i_t} d2_{j_t}^T
    T rr = 0;
    for (int e = lane; e < M; e += kWave) {
      const int p = e % m1, q = e / m1;
      T r = ys[e];
      for (int u = 0; u < t; ++u) {
        const int iu = supp_s[u] % n1, ju = supp_s[u] / n1;
        r -= xs[u] * D1s[p + m1 * iu] * D2s[q + m2 * ju];
      }
      rr += r * r;
    }
    rr = wave_sum(rr);
    if (lane < s) {
      a.supp[k * s + lane] = lane < t ? supp_s[lane] : -1;
      a.coef[k * s + lane] = lane < t ? xs[lane] : T(0);
    }
    if (lane == 0) {
      if (a.res2) a.res2[k] = rr;
      n_early += early ? 1u : 0u;
    }
  }
  if (lane == 0 && n_early) atomicAdd(&a.counters[kCtrEarlyStop], (unsigned long long)n_early);
}

}  // namespace

size_t omp_generic_lds_bytes(int m1, int m2, int n1, int n2, int s, size_t elem) {
  int end = elem == 8 ? layout<double>(m1, m2, n1, n2, s).end : layout<float>(m1, m2, n1, n2, s).end;
  return (size_t)end * elem + sizeof(int) * (size_t)s + (size_t)n1 * n2 + 16;
}

template <typename T>
hipError_t launch_omp_generic(const OmpArgs<T>& a, hipStream_t st) {
  if (a.N == 0) return hipSuccess;
  const size_t lds = omp_generic_lds_bytes(a.m1, a.m2, a.n1, a.n2, a.s, sizeof(T));
  // single-wave workgroups, each striding over the signals; 65,536 of them (a few signals each
  // at 10^5 signals) balance the tail better than fewer, longer ones
  int64_t grid = a.N < 65536 ? a.N : 65536;
  hipLaunchKernelGGL(omp_generic_kernel<T>, dim3((unsigned)grid), dim3(kWave), lds, st, a);
  return hipGetLastError();
}

hipError_t omp_generic_init_device() {
  // allow the dynamic LDS of large shapes (up to the 160 KiB of a gfx950 CU)
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&omp_generic_kernel<float>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&omp_generic_kernel<double>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

template hipError_t launch_omp_generic<float>(const OmpArgs<float>&, hipStream_t);
template hipError_t launch_omp_generic<double>(const OmpArgs<double>&, hipStream_t);

}  // namespace sdl
