// n-dimensional separable dictionary learning (Remark 3): signals are tensors of m_1 x ... x m_n
// entries (first index fastest), the dictionary is D_n (x) ... (x) D_1 and atom
// a = i_1 + n_1 (i_2 + n_2 (...)).  Two kernels:
//
//  * tensor_omp_kernel: OMP on the Kronecker dictionary without forming it, one wave64 per
//    signal, everything in LDS (the n-mode form of the generic two-dimensional kernel).  The
//    first correlations are the successive mode products Y x_1 D_1^T ... x_n D_n^T; Gram entries
//    are products of the per-mode Gram entries prod_d G_d[i_d(a), i_d(b)] (the Gram identity
//    after Algorithm 1, mode by mode); the correlations are refreshed in Gram form with the
//    incrementally grown Cholesky factor, and the residual is formed explicitly at the end.
//  * tensor_sums_kernel: the sums of the mode-d update, A = sum_k W_k(d) W_k(d)^T and
//    B = sum_k Y_k(d) W_k(d)^T with W_k = X_k multiplied along every other mode by its
//    dictionary (Remark 3: Corollary 1 with T = the other modes' Kronecker product).  One wave
//    per workgroup strides over the signals, builds W_k(d) in LDS from the sparse code (support
//    elements added in selection order) and accumulates its products in FP64 in LDS; each
//    workgroup writes one row of partial sums, reduced in fixed order by the two-dimensional
//    path's reduction and solved by its FP64 solve.
#include <float.h>
#include <limits.h>

#include "sdl_internal.h"

namespace sdl {
namespace {

struct TLay {
  int d[kTensorMaxModes], g[kTensorMaxModes], y, b0, b1, al, L, x, v, wv, end;  // offsets in elements of T
  int stage;  // elements of one mode-product buffer
};

__host__ __device__ inline TLay tensor_layout(int nm, const int* m, const int* n, int s) {
  TLay l;
  int o = 0;
  for (int d = 0; d < nm; ++d) { l.d[d] = o; o += m[d] * n[d]; }
  for (int d = 0; d < nm; ++d) { l.g[d] = o; o += n[d] * n[d]; }
  int M = 1, A = 1;
  for (int d = 0; d < nm; ++d) { M *= m[d]; A *= n[d]; }
  // largest intermediate of the mode products: modes < k contracted (n), the rest not (m); the
  // last product (k = nm) goes straight into the correlations
  int st = M;
  for (int k = 1; k < nm; ++k) {
    int e = 1;
    for (int d = 0; d < nm; ++d) e *= d < k ? n[d] : m[d];
    st = e > st ? e : st;
  }
  l.stage = st;
  l.y = o; o += M;
  l.b0 = o; o += st;
  l.b1 = o; o += st;
  l.al = o; o += A;
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

// Gram entry of atoms whose per-mode indices are ia[] and ib[]
template <typename T>
__device__ inline T gram(const T* const* G, const int* n, int nm, const int* ia, const int* ib) {
  T g = G[0][ia[0] + n[0] * ib[0]];
#pragma unroll
  for (int d = 1; d < nm; ++d) g *= G[d][ia[d] + n[d] * ib[d]];
  return g;
}

__device__ inline void split(int a, const int* n, int nm, int* idx) {
#pragma unroll
  for (int d = 0; d < nm; ++d) {
    idx[d] = a % n[d];
    a /= n[d];
  }
}

template <typename T, int NM>
__global__ void __launch_bounds__(kWave) tensor_omp_kernel(TensorArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  constexpr int nm = NM;
  const int s = a.s;
  int m[kTensorMaxModes], n[kTensorMaxModes];
  int M = 1, A = 1;
  for (int d = 0; d < kTensorMaxModes; ++d) {
    m[d] = d < nm ? a.m[d] : 1;
    n[d] = d < nm ? a.n[d] : 1;
    M *= m[d];
    A *= n[d];
  }
  const TLay L = tensor_layout(nm, m, n, s);
  int* supp_s = reinterpret_cast<int*>(sm + L.end);
  int* sidx = supp_s + s;  // per-mode indices of the chosen atoms, [t * kTensorMaxModes + d]
  unsigned char* sel = reinterpret_cast<unsigned char*>(sidx + s * kTensorMaxModes);
  // per-mode indices of every atom, 8 bits each (no integer division in the step loop)
  int* epk = reinterpret_cast<int*>(sel + ((A + 3) & ~3));
  const int lane = threadIdx.x;
  for (int e = lane; e < A; e += kWave) {
    int idx[kTensorMaxModes];
    split(e, n, nm, idx);
    int pk = 0;
#pragma unroll
    for (int d = 0; d < nm; ++d) pk |= idx[d] << (8 * d);
    epk[e] = pk;
  }
  const T* Ds[kTensorMaxModes];
  const T* Gs[kTensorMaxModes];
#pragma unroll
  for (int d = 0; d < nm; ++d) {
    for (int e = lane; e < m[d] * n[d]; e += kWave) sm[L.d[d] + e] = a.D[d][e];
    for (int e = lane; e < n[d] * n[d]; e += kWave) sm[L.g[d] + e] = a.G[d][e];
    Ds[d] = sm + L.d[d];
    Gs[d] = sm + L.g[d];
  }
  for (int d = nm; d < kTensorMaxModes; ++d) {
    Ds[d] = Ds[0];
    Gs[d] = Gs[0];
  }
  T* ys = sm + L.y;
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
      const T v = a.Y[k * M + e];
      ys[e] = v;
      yy += v * v;
    }
    for (int e = lane; e < A; e += kWave) sel[e] = 0;
    const T yy_all = wave_sum(yy);
    const T ynorm = sqrt(yy_all);
    T renergy = yy_all;
    __syncthreads();
    // C = Y x_1 D_1^T x_2 D_2^T ...: mode d contracted into a fresh buffer, the last into al
    {
      const T* cur = ys;
      int ext[kTensorMaxModes];
      for (int d = 0; d < kTensorMaxModes; ++d) ext[d] = m[d];
#pragma unroll
      for (int d = 0; d < nm; ++d) {
        T* out = d == nm - 1 ? al : sm + ((d % 2) ? L.b1 : L.b0);
        int pre = 1, post = 1;
#pragma unroll
        for (int e = 0; e < d; ++e) pre *= ext[e];
#pragma unroll
        for (int e = d + 1; e < nm; ++e) post *= ext[e];
        const int total = pre * n[d] * post;
        for (int e = lane; e < total; e += kWave) {
          const int p0 = e % pre, i = (e / pre) % n[d], q = e / (pre * n[d]);
          const T* src = cur + p0 + pre * m[d] * q;
          const T* dcol = Ds[d] + m[d] * i;
          T v = 0;
          for (int p = 0; p < m[d]; ++p) v += dcol[p] * src[pre * p];
          out[e] = v;
        }
        ext[d] = n[d];
        cur = out;
        __syncthreads();
      }
    }

    int t = 0;
    bool early = false;
    for (; t < s; ++t) {
      if (a.err2 > 0.0 && !(renergy > T(a.err2))) {
        early = true;
        break;
      }
      T bv = T(-1);
      int bi = INT_MAX;
      for (int e = lane; e < A; e += kWave) {
        if (sel[e]) continue;
        const T v = fabs(al[e]);
        if (v > bv) { bv = v; bi = e; }
      }
      wave_argmax(bv, bi);
      if (bi == INT_MAX || !(bv > T(a.stop_rel) * ynorm)) { early = true; break; }
      int ia[kTensorMaxModes];
      split(bi, n, nm, ia);
      for (int d = nm; d < kTensorMaxModes; ++d) ia[d] = 0;
      const T gaa = gram(Gs, n, nm, ia, ia);
      // new Cholesky row L w = G_{S,a} (every lane, redundantly)
      T ww = 0;
      for (int q = 0; q < t; ++q) {
        T b = gram(Gs, n, nm, sidx + q * kTensorMaxModes, ia);
        for (int l = 0; l < q; ++l) b -= Ls[q * s + l] * wv[l];
        b /= Ls[q * s + q];
        wv[q] = b;
        ww += b * b;
      }
      T d2 = gaa - ww;
      if (sizeof(T) == 4 && d2 < T(a.pivot_fp64) * gaa) {
        double w64[SDL_MAX_S];
        double acc = 0.0;
        for (int q = 0; q < t; ++q) {
          const int* iq = sidx + q * kTensorMaxModes;
          double b = 1.0;
#pragma unroll
          for (int d = 0; d < nm; ++d) b *= (double)Gs[d][iq[d] + n[d] * ia[d]];
          for (int l = 0; l < q; ++l) b -= (double)Ls[q * s + l] * w64[l];
          b /= (double)Ls[q * s + q];
          w64[q] = b;
          acc += b * b;
        }
        for (int q = 0; q < t; ++q) wv[q] = (T)w64[q];
        double g64 = 1.0;
#pragma unroll
        for (int d = 0; d < nm; ++d) g64 *= (double)Gs[d][ia[d] + n[d] * ia[d]];
        d2 = (T)(g64 - acc);
        if (lane == 0) atomicAdd(&a.counters[kCtrFp64Pivot], 1ull);
      }
      if (!(d2 > T(a.dep_eps) * gaa)) { early = true; break; }
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
        for (int d = 0; d < kTensorMaxModes; ++d) sidx[t * kTensorMaxModes + d] = ia[d];
        sel[bi] = 1;
      }
      if (t + 1 < s) {
        // corr <- corr - cstar (G_{:,a} - G_{:,S} v)
        for (int e = lane; e < A; e += kWave) {
          int ie[kTensorMaxModes];
          const int pk = epk[e];
#pragma unroll
          for (int d = 0; d < nm; ++d) ie[d] = (pk >> (8 * d)) & 0xFF;
          T g = gram(Gs, n, nm, ie, ia);
          for (int q = 0; q < t; ++q) g -= vs[q] * gram(Gs, n, nm, ie, sidx + q * kTensorMaxModes);
          al[e] -= cstar * g;
        }
      }
      __syncthreads();
    }
    __syncthreads();
    // explicit residual
    T rr = 0;
    for (int e = lane; e < M; e += kWave) {
      int pe[kTensorMaxModes];
      split(e, m, nm, pe);
      T r = ys[e];
      for (int u = 0; u < t; ++u) {
        const int* iu = sidx + u * kTensorMaxModes;
        T prod = xs[u];
#pragma unroll
        for (int d = 0; d < nm; ++d) prod *= Ds[d][pe[d] + m[d] * iu[d]];
        r -= prod;
      }
      rr += r * r;
    }
    rr = wave_sum(rr);
    for (int q = lane; q < s; q += kWave) {
      a.supp[k * s + q] = q < t ? supp_s[q] : -1;
      a.coef[k * s + q] = q < t ? xs[q] : T(0);
    }
    if (lane == 0) {
      if (a.res2) a.res2[k] = rr;
      n_early += early ? 1u : 0u;
    }
  }
  if (lane == 0 && n_early) atomicAdd(&a.counters[kCtrEarlyStop], (unsigned long long)n_early);
}

// ---------------------------------------------------------------- mode-d sums

struct SLay {
  int d[kTensorMaxModes], y, w, end;  // offsets in elements of T
  int mo;                             // columns of the mode-d matricisation
};

__host__ __device__ inline SLay sums_layout(int nm, const int* m, const int* n, int mode) {
  SLay l;
  int o = 0, M = 1;
#pragma unroll
  for (int d = 0; d < nm; ++d) { l.d[d] = o; o += m[d] * n[d]; M *= m[d]; }
  l.mo = M / m[mode];
  l.y = o; o += M;
  l.w = o; o += n[mode] * l.mo;
  l.end = o;
  return l;
}

__host__ __device__ inline size_t sums_lds_bytes(int nm, const int* m, const int* n, int mode, size_t elem) {
  const SLay l = sums_layout(nm, m, n, mode);
  const int nent = n[mode] * n[mode] + m[mode] * n[mode];
  // elements of T, then the columns' packed indices and base offsets, then FP64 accumulators
  return ((size_t)l.end * elem + 15) / 16 * 16 + 2 * sizeof(int) * (size_t)l.mo + sizeof(double) * (size_t)nent + 32;
}

template <typename T, int NM>
__global__ void __launch_bounds__(kWave) tensor_sums_kernel(TensorArgs<T> a, int mode, double* part) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  constexpr int nm = NM;
  const int s = a.s, lane = threadIdx.x;
  int m[kTensorMaxModes], n[kTensorMaxModes];
  int M = 1;
  for (int d = 0; d < kTensorMaxModes; ++d) {
    m[d] = d < nm ? a.m[d] : 1;
    n[d] = d < nm ? a.n[d] : 1;
    M *= m[d];
  }
  const SLay L = sums_layout(nm, m, n, mode);
  const int mo = L.mo, na = n[mode], mr = m[mode];
  const int nent = na * na + mr * na;
  int* cidx = reinterpret_cast<int*>(smem_raw + ((size_t)L.end * sizeof(T) + 15) / 16 * 16);
  int* cbase = cidx + mo;
  double* acc = reinterpret_cast<double*>((reinterpret_cast<uintptr_t>(cbase + mo) + 7) & ~uintptr_t(7));
  const T* Ds[kTensorMaxModes];
#pragma unroll
  for (int d = 0; d < nm; ++d) {
    for (int e = lane; e < m[d] * n[d]; e += kWave) sm[L.d[d] + e] = a.D[d][e];
    Ds[d] = sm + L.d[d];
  }
  // column c of the matricisation: the other modes' pixel indices (packed 8 bits each) and the
  // pixel offset with the mode-d index 0
  int stride[kTensorMaxModes];
  {
    int st = 1;
    for (int d = 0; d < kTensorMaxModes; ++d) {
      stride[d] = st;
      st *= m[d];
    }
  }
  for (int c = lane; c < mo; c += kWave) {
    int r = c, packed = 0, base = 0;
#pragma unroll
    for (int d = 0; d < nm; ++d) {
      if (d == mode) continue;
      const int v = r % m[d];
      r /= m[d];
      packed |= v << (8 * d);
      base += v * stride[d];
    }
    cidx[c] = packed;
    cbase[c] = base;
  }
  for (int e = lane; e < nent; e += kWave) acc[e] = 0.0;
  T* ys = sm + L.y;
  T* W = sm + L.w;  // na x mo, column-major
  for (int64_t k = blockIdx.x; k < a.N; k += gridDim.x) {
    __syncthreads();
    for (int e = lane; e < M; e += kWave) ys[e] = a.Y[k * M + e];
    // W(d)[i, c] = sum over support elements with mode-d index i of x_t prod_{e != d} D_e[c_e, i_e(t)]
    for (int c = lane; c < mo; c += kWave) {
      for (int i = 0; i < na; ++i) W[i + na * c] = T(0);
      const int packed = cidx[c];
      for (int t = 0; t < s; ++t) {
        const int at = a.supp[k * s + t];
        if (at < 0) continue;
        int r = at, id = 0;
        T v = a.coef[k * s + t];
#pragma unroll
        for (int d = 0; d < nm; ++d) {
          const int i = r % n[d];
          r /= n[d];
          if (d == mode) {
            id = i;
          } else {
            const int pc = (packed >> (8 * d)) & 0xFF;
            v *= Ds[d][pc + m[d] * i];
          }
        }
        W[id + na * c] += v;
      }
    }
    __syncthreads();
    for (int e = lane; e < nent; e += kWave) {
      T v = 0;
      if (e < na * na) {
        const int i = e % na, j = e / na;
        for (int c = 0; c < mo; ++c) v += W[i + na * c] * W[j + na * c];
      } else {
        const int f = e - na * na, p = f % mr, i = f / mr;
        for (int c = 0; c < mo; ++c) v += ys[cbase[c] + p * stride[mode]] * W[i + na * c];
      }
      acc[e] += (double)v;
    }
  }
  __syncthreads();
  for (int e = lane; e < nent; e += kWave) part[(size_t)blockIdx.x * nent + e] = acc[e];
}

// Dk[p', j'] = prod_{d>=1} D_d[p_d, i_d] with p' = p_1 + m_1 (p_2 + ...), j' = i_1 + n_1 (i_2 + ...)
__global__ void kron_tail_kernel(TensorArgs<double> d, double* Dk, int mk, int nk) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < mk * nk; e += gridDim.x * blockDim.x) {
    int p = e % mk, j = e / mk;
    double v = 1.0;
    for (int q = 1; q < d.nmodes; ++q) {
      const int pq = p % d.m[q], iq = j % d.n[q];
      p /= d.m[q];
      j /= d.n[q];
      v *= d.D[q][pq + d.m[q] * iq];
    }
    Dk[e] = v;
  }
}

// FP32 mode-d sums on the matrix cores, for n_d <= 16 and m_d <= 16: the signals' W_k(d) and
// Y_k(d) concatenated along their columns form the contraction A = Wcat Wcat^T, B = Ycat Wcat^T,
// run four columns at a time with the 16x16x4 FP32 MFMA (lane l supplies row l % 16 of column
// l / 16 of the slice, which is both operands' value for the A sum).  One wave per workgroup
// strides over the signals, accumulating in FP32; its tiles are written as one FP64 partial row.
typedef float f32x4_t __attribute__((ext_vector_type(4)));
constexpr int kSumsLdw = 17;  // W column stride (odd: the lanes' columns fall in different banks)

__host__ __device__ inline size_t sums_mfma_lds_bytes(int nm, const int* m, const int* n, int mode) {
  int M = 1, dsz = 0;
  for (int d = 0; d < nm; ++d) {
    M *= m[d];
    dsz += m[d] * n[d];
  }
  const int mo = M / m[mode], mo4 = (mo + 3) / 4 * 4;
  return sizeof(float) * ((size_t)dsz + M + (size_t)kSumsLdw * mo4) + 2 * sizeof(int) * (size_t)mo4 +
         2 * sizeof(int) * SDL_MAX_S + 32;
}

template <int NM>
__global__ void __launch_bounds__(kWave) tensor_sums_mfma_kernel(TensorArgs<float> a, int mode, double* part) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* sm = reinterpret_cast<float*>(smem_raw);
  constexpr int nm = NM;
  const int s = a.s, lane = threadIdx.x;
  int m[kTensorMaxModes], n[kTensorMaxModes], stride[kTensorMaxModes];
  int M = 1, dsz = 0;
  for (int d = 0; d < kTensorMaxModes; ++d) {
    m[d] = d < nm ? a.m[d] : 1;
    n[d] = d < nm ? a.n[d] : 1;
    stride[d] = M;
    M *= m[d];
  }
  const float* Ds[kTensorMaxModes];
  int off = 0;
#pragma unroll
  for (int d = 0; d < nm; ++d) {
    for (int e = lane; e < m[d] * n[d]; e += kWave) sm[off + e] = a.D[d][e];
    Ds[d] = sm + off;
    off += m[d] * n[d];
    dsz = off;
  }
  const int na = n[mode], mr = m[mode], mo = M / mr, mo4 = (mo + 3) / 4 * 4;
  float* ys = sm + dsz;
  float* W = ys + M;  // W[i + kSumsLdw c], i < 16, c < mo4 (rows >= na and columns >= mo stay 0)
  int* cidx = reinterpret_cast<int*>(W + kSumsLdw * mo4);
  int* cbase = cidx + mo4;
  unsigned* tpk = reinterpret_cast<unsigned*>(cbase + mo4);  // the signal's code, decoded (below)
  float* tcv = reinterpret_cast<float*>(tpk + SDL_MAX_S);
  for (int c = lane; c < mo4; c += kWave) {
    int r = c, packed = 0, base = 0;
#pragma unroll
    for (int d = 0; d < nm; ++d) {
      if (d == mode) continue;
      const int v = r % m[d];
      r /= m[d];
      packed |= v << (8 * d);
      base += v * stride[d];
    }
    cidx[c] = packed;
    cbase[c] = c < mo ? base : -1;
  }
  const int r16 = lane % 16, kq = lane / 16;
  f32x4_t accA = {0.f, 0.f, 0.f, 0.f}, accB = {0.f, 0.f, 0.f, 0.f};
  for (int64_t k = blockIdx.x; k < a.N; k += gridDim.x) {
    __syncthreads();
    for (int e = lane; e < M; e += kWave) ys[e] = a.Y[k * M + e];
    // the signal's code decoded once: slot t's atom as its per-mode indices (8 bits each) and
    // its coefficient; an unused slot reads (0, 0) and is skipped
    if (lane < s) {
      const int at = a.supp[k * s + lane];
      unsigned pk = 0u;
      float cv = 0.f;
      if (at >= 0) {
        int r = at;
#pragma unroll
        for (int d = 0; d < nm; ++d) {
          pk |= (unsigned)(r % n[d]) << (8 * d);
          r /= n[d];
        }
        cv = a.coef[k * s + lane];
      }
      tpk[lane] = pk;
      tcv[lane] = cv;
    }
    __syncthreads();
    for (int c = lane; c < mo4; c += kWave) {
      float col[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) col[i] = 0.f;
      if (c < mo) {
        const int packed = cidx[c];
        for (int t = 0; t < s; ++t) {
          const unsigned pk = tpk[t];
          float v = tcv[t];
          if (pk == 0u && v == 0.f) continue;
          int id = 0;
#pragma unroll
          for (int d = 0; d < nm; ++d) {
            const int i = (int)((pk >> (8 * d)) & 0xFFu);
            if (d == mode) id = i;
            else v *= Ds[d][((packed >> (8 * d)) & 0xFF) + m[d] * i];
          }
          // selection order within the column: the same sums as adding element by element
#pragma unroll
          for (int i = 0; i < 16; ++i) col[i] += (i == id) ? v : 0.f;
        }
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) W[i + kSumsLdw * c] = col[i];
    }
    __syncthreads();
    for (int c0 = 0; c0 < mo4; c0 += 4) {
      const int c = c0 + kq;
      const float wv = W[r16 + kSumsLdw * c];
      const int cb = cbase[c];
      const float yv = (r16 < mr && cb >= 0) ? ys[cb + r16 * stride[mode]] : 0.f;
      accA = __builtin_amdgcn_mfma_f32_16x16x4f32(wv, wv, accA, 0, 0, 0);
      accB = __builtin_amdgcn_mfma_f32_16x16x4f32(yv, wv, accB, 0, 0, 0);
    }
  }
  // tile element (4 kq + v, r16): A[i][j] with i = 4 kq + v, j = r16; B[p][j] likewise
  const int nent = na * na + mr * na;
  double* row = part + (size_t)blockIdx.x * nent;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 4 * kq + v, j = r16;
    if (i < na && j < na) row[i + na * j] = (double)accA[v];
    if (i < mr && j < na) row[na * na + i + mr * j] = (double)accB[v];
  }
}

template <typename T>
__global__ void tensor_rescale_kernel(int64_t n_el, int div, int na, const int32_t* supp, T* coef, const double* w) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_el) return;
  const int at = supp[e];
  if (at < 0) return;
  coef[e] = (T)((double)coef[e] * w[(at / div) % na]);
}

}  // namespace

size_t tensor_omp_lds_bytes(int nmodes, const int* m, const int* n, int s, size_t elem) {
  const TLay l = tensor_layout(nmodes, m, n, s);
  int A = 1;
  for (int d = 0; d < nmodes; ++d) A *= n[d];
  return (size_t)l.end * elem + sizeof(int) * (size_t)s * (1 + kTensorMaxModes) + (size_t)((A + 3) & ~3) +
         sizeof(int) * (size_t)A + 16;
}

size_t tensor_sums_lds(int nmodes, const int* m, const int* n, int mode, size_t elem) {
  return sums_lds_bytes(nmodes, m, n, mode, elem);
}

int tensor_sums_rows(int64_t N) {
  // one wave per row: 8,192 rows give the mode sums 8 waves per SIMD on 256 CUs (their
  // register limit), which hides each signal's loads (4,096 rows: 4% slower per learning
  // iteration at 100,000 three-mode signals)
  int64_t r = N < 8192 ? N : 8192;
  return (int)(r < 1 ? 1 : r);
}

template <typename T>
hipError_t launch_tensor_omp(const TensorArgs<T>& a, hipStream_t st) {
  if (a.N == 0) return hipSuccess;
  const size_t lds = tensor_omp_lds_bytes(a.nmodes, a.m, a.n, a.s, sizeof(T));
  const int64_t grid = a.N < 65536 ? a.N : 65536;
  if (a.nmodes == 2)
    hipLaunchKernelGGL((tensor_omp_kernel<T, 2>), dim3((unsigned)grid), dim3(kWave), lds, st, a);
  else if (a.nmodes == 3)
    hipLaunchKernelGGL((tensor_omp_kernel<T, 3>), dim3((unsigned)grid), dim3(kWave), lds, st, a);
  else
    hipLaunchKernelGGL((tensor_omp_kernel<T, 4>), dim3((unsigned)grid), dim3(kWave), lds, st, a);
  return hipGetLastError();
}

bool tensor_sums_mfma_ok(int nmodes, const int* m, const int* n, int mode) {
  return n[mode] <= 16 && m[mode] <= 16 && sums_mfma_lds_bytes(nmodes, m, n, mode) <= 64 * 1024;
}

template <typename T>
hipError_t launch_tensor_sums(const TensorArgs<T>& a, int mode, double* part, hipStream_t st) {
  const int rows = tensor_sums_rows(a.N);
  if constexpr (sizeof(T) == 4) {
    if (tensor_sums_mfma_ok(a.nmodes, a.m, a.n, mode)) {
      const size_t lds = sums_mfma_lds_bytes(a.nmodes, a.m, a.n, mode);
      if (a.nmodes == 2)
        hipLaunchKernelGGL((tensor_sums_mfma_kernel<2>), dim3((unsigned)rows), dim3(kWave), lds, st, a, mode, part);
      else if (a.nmodes == 3)
        hipLaunchKernelGGL((tensor_sums_mfma_kernel<3>), dim3((unsigned)rows), dim3(kWave), lds, st, a, mode, part);
      else
        hipLaunchKernelGGL((tensor_sums_mfma_kernel<4>), dim3((unsigned)rows), dim3(kWave), lds, st, a, mode, part);
      return hipGetLastError();
    }
  }
  const size_t lds = sums_lds_bytes(a.nmodes, a.m, a.n, mode, sizeof(T));
  if (a.nmodes == 2)
    hipLaunchKernelGGL((tensor_sums_kernel<T, 2>), dim3((unsigned)rows), dim3(kWave), lds, st, a, mode, part);
  else if (a.nmodes == 3)
    hipLaunchKernelGGL((tensor_sums_kernel<T, 3>), dim3((unsigned)rows), dim3(kWave), lds, st, a, mode, part);
  else
    hipLaunchKernelGGL((tensor_sums_kernel<T, 4>), dim3((unsigned)rows), dim3(kWave), lds, st, a, mode, part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tensor_rescale(const TensorArgs<T>& a, int mode, const double* w, hipStream_t st) {
  const int64_t n_el = a.N * a.s;
  if (n_el == 0) return hipSuccess;
  int div = 1;
  for (int d = 0; d < mode; ++d) div *= a.n[d];
  hipLaunchKernelGGL(tensor_rescale_kernel<T>, dim3((unsigned)((n_el + 255) / 256)), dim3(256), 0, st, n_el, div,
                     a.n[mode], a.supp, a.coef, w);
  return hipGetLastError();
}

hipError_t launch_kron_tail(const TensorArgs<double>& d, double* Dk, hipStream_t st) {
  int mk = 1, nk = 1;
  for (int q = 1; q < d.nmodes; ++q) {
    mk *= d.m[q];
    nk *= d.n[q];
  }
  hipLaunchKernelGGL(kron_tail_kernel, dim3((unsigned)((mk * nk + 255) / 256)), dim3(256), 0, st, d, Dk, mk, nk);
  return hipGetLastError();
}

hipError_t tensor_init_device() {
  const void* fs[] = {
      reinterpret_cast<const void*>(&tensor_omp_kernel<float, 2>), reinterpret_cast<const void*>(&tensor_omp_kernel<float, 3>),
      reinterpret_cast<const void*>(&tensor_omp_kernel<float, 4>), reinterpret_cast<const void*>(&tensor_omp_kernel<double, 2>),
      reinterpret_cast<const void*>(&tensor_omp_kernel<double, 3>), reinterpret_cast<const void*>(&tensor_omp_kernel<double, 4>),
      reinterpret_cast<const void*>(&tensor_sums_kernel<float, 2>), reinterpret_cast<const void*>(&tensor_sums_kernel<float, 3>),
      reinterpret_cast<const void*>(&tensor_sums_kernel<float, 4>), reinterpret_cast<const void*>(&tensor_sums_kernel<double, 2>),
      reinterpret_cast<const void*>(&tensor_sums_kernel<double, 3>), reinterpret_cast<const void*>(&tensor_sums_kernel<double, 4>)};
  for (const void* f : fs) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t launch_tensor_omp<float>(const TensorArgs<float>&, hipStream_t);
template hipError_t launch_tensor_omp<double>(const TensorArgs<double>&, hipStream_t);
template hipError_t launch_tensor_sums<float>(const TensorArgs<float>&, int, double*, hipStream_t);
template hipError_t launch_tensor_sums<double>(const TensorArgs<double>&, int, double*, hipStream_t);
template hipError_t launch_tensor_rescale<float>(const TensorArgs<float>&, int, const double*, hipStream_t);
template hipError_t launch_tensor_rescale<double>(const TensorArgs<double>&, int, const double*, hipStream_t);

}  // namespace sdl
