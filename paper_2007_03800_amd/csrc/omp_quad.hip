// FP32 2D-OMP on matrix-core quadrants: shapes whose correlation block is too large for
// four lanes per signal (omp_mfma.hip) but small enough that a whole wave per signal
// (omp_wave.hip) leaves most of the wave's work per step idle.
//
// Same method and recurrences as omp_mfma.hip (2D-OMP, Sec. III step 1; Gram-form
// refresh with G1[i,i'] G2[j,j'], text after Algorithm 1); what changes is the mapping:
//
//  * Sixteen lanes own a signal and a wave codes 4 signals.  The signal's n1 x n2
//    correlations (padded with zeros to multiples of 8) are split into 2 x 2 quadrants;
//    each quadrant is one block of the 4x4x1 16-block FP32 MFMA and holds its
//    (n1/8) x (n2/8) tiles of 4x4 in that instruction's result layout.  A refresh term
//    gamma_k G1[:,i_k] G2[j_k,:] is then one MFMA per tile of a quadrant, fed by n1/8 + n2/8
//    LDS reads per lane.
//  * Largest |corr| on packed keys as in omp_mfma.hip (|corr| with the low 6 mantissa
//    bits replaced by the position inside the lane, a lane's positions in increasing atom
//    order), then across the signal's 16 lanes (one DPP row) by quad swaps, half-row
//    mirror and row mirror on (magnitude, atom) pairs, ties to the smaller atom.
//  * The chosen atom's correlation is recomputed exactly (d1_i^T Y d2_j minus the
//    support's contribution) and the greedy step is branch-free (results committed with
//    selects), as in omp_mfma.hip.  The least squares carries the inverse Cholesky factor
//    (in LDS), so both triangular products of a step are independent dot products: with
//    only four signals per wave, substitution chains would leave the SIMD idle.
//  * No sums epilogue: dictionary updates use the standalone sums kernel.
#include <limits.h>

#include "sdl_internal.h"

namespace sdl {
namespace {

constexpr int kQWaves = 4;        // waves per workgroup
constexpr int kQMaxBlocks = 4096;
constexpr int kQLanes = 16;       // lanes per signal: four 4x4x1 MFMA blocks (quadrants)
constexpr int kQSigs = 4;         // signals per wave

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int M1_, int M2_, int N1_, int N2_, int S_>
struct QCfg {
  static constexpr int M1 = M1_, M2 = M2_, N1 = N1_, N2 = N2_, S = S_;
  static constexpr int NP1 = (N1 + 7) / 8 * 8, NP2 = (N2 + 7) / 8 * 8;  // two quadrants of 4x4 tiles
  static constexpr int TI = NP1 / 8, TJ = NP2 / 8;                        // tiles per quadrant
  static constexpr int M = M1 * M2, NL = S * (S + 1) / 2;
  // odd LDS strides: the four signals of a wave (and the atoms they pick) fall into
  // different banks
  static constexpr int YS = M + 1, LD1 = M1 + 1, LD2 = M2 + 1, NLP = NL + 1;
  static_assert(TI * TJ * 4 <= 64, "at most 64 correlations per lane (6-bit position in the keys)");
  static_assert(M % 16 == 0 && M1 % 4 == 0, "staging, residual split and 4x4 tiles of Y D2");
  static_assert(M2 <= kQLanes && S <= kQLanes, "one lane per column of Y / per support element");
};

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL>
__device__ inline int dpp(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ inline float dppf(float v) {
  return __builtin_bit_cast(float, dpp<CTRL>(__builtin_bit_cast(int, v)));
}

// Sum over the 16 lanes of a DPP row (quad swaps, half-row mirror, row mirror); every
// lane of the row ends with the same value.
__device__ inline float row_sum(float v) {
  v += dppf<0xB1>(v);
  v += dppf<0x4E>(v);
  v += dppf<0x141>(v);
  v += dppf<0x140>(v);
  return v;
}

template <int CTRL>
__device__ inline void row_argmax_stage(unsigned& key, int& atom) {
  const unsigned ok = (unsigned)dpp<CTRL>((int)key);
  const int oa = dpp<CTRL>(atom);
  const bool take = ok > key || (ok == key && oa < atom);
  key = take ? ok : key;
  atom = take ? oa : atom;
}

__device__ inline unsigned umax3(unsigned a, unsigned b, unsigned c) { return max(max(a, b), c); }

constexpr int tri(int k, int l) { return k * (k + 1) / 2 + l; }  // L[k][l], l <= k

template <class C>
__global__ void __launch_bounds__(kWave* kQWaves) __attribute__((amdgpu_waves_per_eu(2, 2))) omp_quad_kernel(OmpArgs<float> a) {
  constexpr int M1 = C::M1, M2 = C::M2, N1 = C::N1, N2 = C::N2, S = C::S, M = C::M;
  constexpr int NP1 = C::NP1, NP2 = C::NP2, TI = C::TI, TJ = C::TJ;
  __shared__ float sG1[NP1 * NP1];                  // G1[i, i'] at i + NP1 i' (zero padding)
  __shared__ float sG2[NP2 * NP2];                  // G2[j, j'] at j + NP2 j'
  __shared__ __align__(16) float sG1P[NP1 * NP1];   // [ik][qi][c][bi] = G1[4 (qi TI + bi) + c, ik]
  __shared__ __align__(16) float sG2P[NP2 * NP2];   // [jk][qj][c][bj] = G2[jk, 4 (qj TJ + bj) + c]
  __shared__ float sD1[C::LD1 * NP1];               // D1[p, i] at p + LD1 i
  __shared__ __align__(16) float sD1P[M1 * NP1];    // [p][qi][c][bi] = D1[p, 4 (qi TI + bi) + c]
  __shared__ float sD2[C::LD2 * NP2];               // D2[q, j] at q + LD2 j
  __shared__ __align__(16) float sY[kQWaves][kQSigs * C::YS];
  __shared__ float sL[kQWaves][kQSigs * C::NLP];

  const int tid = threadIdx.x, wv = tid / kWave, lane = tid % kWave;
  const int g = lane / kQLanes, cs = lane % kQLanes;  // signal of the wave, lane of the signal
  const int qb = cs / 4, c = cs % 4, qi = qb / 2, qj = qb % 2;
  auto g1v = [&](int i, int ik) { return i < N1 && ik < N1 ? a.G1[i + N1 * ik] : 0.f; };
  auto g2v = [&](int j, int jk) { return j < N2 && jk < N2 ? a.G2[j + N2 * jk] : 0.f; };
  auto d1v = [&](int p, int i) { return i < N1 ? a.D1[p + M1 * i] : 0.f; };
  auto d2v = [&](int q, int j) { return j < N2 ? a.D2[q + M2 * j] : 0.f; };
  for (int e = tid; e < NP1 * NP1; e += blockDim.x) {
    sG1[e] = g1v(e % NP1, e / NP1);
    const int ik = e / NP1, r = e % NP1, rq = r / (4 * TI), rc = (r % (4 * TI)) / TI, rb = r % TI;
    sG1P[e] = g1v(4 * (rq * TI + rb) + rc, ik);
  }
  for (int e = tid; e < NP2 * NP2; e += blockDim.x) {
    sG2[e] = g2v(e % NP2, e / NP2);
    const int jk = e / NP2, r = e % NP2, rq = r / (4 * TJ), rc = (r % (4 * TJ)) / TJ, rb = r % TJ;
    sG2P[e] = g2v(4 * (rq * TJ + rb) + rc, jk);  // G2 is symmetric
  }
  for (int e = tid; e < M1 * NP1; e += blockDim.x) {
    sD1[e % M1 + C::LD1 * (e / M1)] = d1v(e % M1, e / M1);
    const int p = e / NP1, r = e % NP1, rq = r / (4 * TI), rc = (r % (4 * TI)) / TI, rb = r % TI;
    sD1P[e] = d1v(p, 4 * (rq * TI + rb) + rc);
  }
  for (int e = tid; e < M2 * NP2; e += blockDim.x) sD2[e % M2 + C::LD2 * (e / M2)] = d2v(e % M2, e / M2);
  __syncthreads();

  const float stop_rel = (float)a.stop_rel, dep_eps = (float)a.dep_eps, piv = (float)a.pivot_fp64;
  const int64_t nsig = a.N;
  const int64_t ngroups = (nsig + kQSigs - 1) / kQSigs;
  float* ys = sY[wv];
  const float* G1q = sG1P + qi * 4 * TI + c * TI;  // + ik NP1: G1[4 (qi TI + bi) + c, ik], bi < TI
  const float* G2q = sG2P + qj * 4 * TJ + c * TJ;  // + jk NP2: G2[jk, 4 (qj TJ + bj) + c], bj < TJ

  unsigned n_early = 0;  // early-stopped signals seen by this lane, counted once at the end
  for (int64_t grp = (int64_t)blockIdx.x * kQWaves + wv; grp < ngroups; grp += (int64_t)gridDim.x * kQWaves) {
    const int64_t k0 = grp * kQSigs;
    const int nvalid = (int)((nsig - k0) < kQSigs ? (nsig - k0) : kQSigs);
    {
      // signal b of the group at ys + b * YS
      const int nchunk = nvalid * M / 4;
      for (int e = lane; e < kQSigs * M / 4; e += kWave) {
        const int b = e / (M / 4), off = e % (M / 4);
        const float4 v = e < nchunk ? load_signal4(a, (k0 + b) * M + 4 * off) : make_float4(0.f, 0.f, 0.f, 0.f);
        float* d = ys + b * C::YS + 4 * off;
        d[0] = v.x;
        d[1] = v.y;
        d[2] = v.z;
        d[3] = v.w;
      }
    }
    wave_sync();
    const float* y = ys + g * C::YS;
    const bool valid = g < nvalid;
    float yy = 0.f;
#pragma unroll
    for (int u = 0; u < M / kQLanes; ++u) {
      const float v = y[cs + kQLanes * u];
      yy += v * v;
    }
    const float ynorm = sqrtf(row_sum(yy));

    // ---- C = D1^T (Y D2) for this lane's quadrant, on the matrix cores
    f32x4 al[TI][TJ];
#pragma unroll
    for (int bi = 0; bi < TI; ++bi)
#pragma unroll
      for (int bj = 0; bj < TJ; ++bj) al[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
    // V = Y D2 in 4x4 tiles (rows 4bp + v, the quadrant's columns), one row block bp at a
    // time: register v of tile bj in lane c is V[4bp + v, 4 (qj TJ + bj) + c], the B operand
    // of C = D1^T V for rows p = 4bp + v
#pragma unroll
    for (int bp = 0; bp < M1 / 4; ++bp) {
      f32x4 vt[TJ];
#pragma unroll
      for (int bj = 0; bj < TJ; ++bj) vt[bj] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < M2; ++q) {
        const float ya = y[(4 * bp + c) + M1 * q];
#pragma unroll
        for (int bj = 0; bj < TJ; ++bj)
          vt[bj] = __builtin_amdgcn_mfma_f32_4x4x1f32(ya, sD2[q + C::LD2 * (4 * (qj * TJ + bj) + c)], vt[bj], 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = 4 * bp + v;
        const float* d1p = sD1P + p * NP1 + qi * 4 * TI + c * TI;  // D1[p, 4 (qi TI + bi) + c]
#pragma unroll
        for (int bi = 0; bi < TI; ++bi) {
          const float av = d1p[bi];
#pragma unroll
          for (int bj = 0; bj < TJ; ++bj) {
            const float vb = vt[bj][v];  // by value
            al[bi][bj] = __builtin_amdgcn_mfma_f32_4x4x1f32(av, vb, al[bi][bj], 0, 0, 0);
          }
        }
      }
    }

    // ---- greedy loop
    float* L = sL[wv] + g * C::NLP;
    float x[S];
    int ia[S], ja[S];
#pragma unroll
    for (int k = 0; k < S; ++k) {
      x[k] = 0.f;
      ia[k] = 0;
      ja[k] = 0;
    }
    bool active = valid;
    int nsel = 0;
    const float stop_thr = stop_rel * ynorm;

#pragma unroll
    for (int t = 0; t < S; ++t) {
      // packed keys, position e = (bj TI + bi) 4 + v (increasing atom order in the lane);
      // elements are read by value
      unsigned bacc[TI];
#pragma unroll
      for (int bi = 0; bi < TI; ++bi) bacc[bi] = 0u;
#pragma unroll
      for (int bj = 0; bj < TJ; ++bj)
#pragma unroll
        for (int bi = 0; bi < TI; ++bi)
#pragma unroll
          for (int v = 0; v < 4; v += 2) {
            const int e0 = (bj * TI + bi) * 4 + v;
            const float c0 = al[bi][bj][v], c1 = al[bi][bj][v + 1];
            const unsigned k0v = (__float_as_uint(c0) & 0x7FFFFFC0u) | (unsigned)(63 - e0);
            const unsigned k1v = (__float_as_uint(c1) & 0x7FFFFFC0u) | (unsigned)(63 - (e0 + 1));
            bacc[bi] = umax3(bacc[bi], k0v, k1v);
          }
      unsigned best = bacc[0];
#pragma unroll
      for (int bi = 1; bi + 1 < TI; bi += 2) best = umax3(best, bacc[bi], bacc[bi + 1]);
      if (TI % 2 == 0) best = max(best, bacc[TI - 1]);
      int atom;
      {
        const int epos = 63 - (int)(best & 63u);
        const int v_ = epos & 3, tile = epos >> 2;
        const int bi_ = tile % TI, bj_ = tile / TI;
        atom = (4 * (qi * TI + bi_) + v_) + N1 * (4 * (qj * TJ + bj_) + c);
      }
      unsigned bkey = best & ~63u;
      row_argmax_stage<0xB1>(bkey, atom);
      row_argmax_stage<0x4E>(bkey, atom);
      row_argmax_stage<0x141>(bkey, atom);
      row_argmax_stage<0x140>(bkey, atom);
      const int it = atom % N1, jt = atom / N1;
      const float babs = __builtin_bit_cast(float, bkey);
      bool stop = !(babs > stop_thr);
#pragma unroll
      for (int k = 0; k < t; ++k) stop = stop || (atom == ia[k] + N1 * ja[k]);
      if (stop) active = false;
      // The step runs in every lane (a stopped signal computes values it never commits):
      // results are committed with selects below.
      // L^{-1} (rows with the diagonal, in LDS) instead of L: with g = G_{S,a}, w = L^{-1} g
      // and v = L^{-T} w are independent dot products, delta^2 = G_aa - |w|^2, and the new
      // row of L^{-1} is [-v^T, 1] / delta
      float w[S > 1 ? S - 1 : 1], gv[S > 1 ? S - 1 : 1];
      const float gaa = sG1[it + NP1 * it] * sG2[jt + NP2 * jt];
      float d2;
      {
#pragma unroll
        for (int k = 0; k < t; ++k) gv[k] = sG1[ia[k] + NP1 * it] * sG2[ja[k] + NP2 * jt];
        float ww = 0.f;
#pragma unroll
        for (int k = 0; k < t; ++k) {
          float b = 0.f;
#pragma unroll
          for (int l = 0; l <= k; ++l) b += L[tri(k, l)] * gv[l];
          w[k] = b;
          ww += b * b;
        }
        d2 = gaa - ww;
        if (active && d2 < piv * gaa) {
          // small pivot: w and |w|^2 again in FP64 (cancellation in G_aa - |w|^2)
          double accd = 0.0;
#pragma unroll
          for (int k = 0; k < t; ++k) {
            double b = 0.0;
#pragma unroll
            for (int l = 0; l <= k; ++l)
              b += (double)L[tri(k, l)] * ((double)sG1[ia[l] + NP1 * it] * (double)sG2[ja[l] + NP2 * jt]);
            w[k] = (float)b;
            accd += b * b;
          }
          d2 = (float)((double)gaa - accd);
          if (cs == 0) atomicAdd(&a.counters[kCtrFp64Pivot], 1ull);
        }
        if (!(d2 > dep_eps * gaa)) active = false;
      }
      // exact correlation of the chosen atom with the residual: d1^T Y d2 - G_{a,S} x_S,
      // one column q = cs of Y per lane
      float cor;
      {
        float part = 0.f;
        if (cs < M2) {
          float col = 0.f;
#pragma unroll
          for (int p = 0; p < M1; ++p) col += sD1[p + C::LD1 * it] * y[p + M1 * cs];
          part = col * sD2[cs + C::LD2 * jt];
        }
        cor = row_sum(part);
#pragma unroll
        for (int k = 0; k < t; ++k) cor -= gv[k] * x[k];
      }
      {
        float vv[S > 1 ? S - 1 : 1];
#pragma unroll
        for (int l = 0; l < t; ++l) {
          float b = 0.f;
#pragma unroll
          for (int k = l; k < t; ++k) b += L[tri(k, l)] * w[k];
          vv[l] = b;
        }
        const float cst = cor / d2;
        const float dinv = rsqrtf(d2);
        // the signal's lanes write the same row: no divergent store
#pragma unroll
        for (int k = 0; k < t; ++k) {
          L[tri(t, k)] = -vv[k] * dinv;
          x[k] = active ? x[k] - cst * vv[k] : x[k];
        }
        L[tri(t, t)] = dinv;
        x[t] = active ? cst : 0.f;
        ia[t] = active ? it : 0;
        ja[t] = active ? jt : 0;
        nsel = active ? t + 1 : nsel;
        if (t + 1 < S) {
          // corr += sum_k (-gamma_k G1[:, i_k]) (x) G2[j_k, :], gamma_t = cst, gamma_k = -cst v_k
#pragma unroll
          for (int k = 0; k <= t; ++k) {
            const float gk = k == t ? -cst : cst * vv[k < t ? k : 0];
            const int ik = k == t ? it : ia[k];
            const int jk = k == t ? jt : ja[k];
            const float* g1p = G1q + ik * NP1;
            const float* g2p = G2q + jk * NP2;
            float av[TI], bv[TJ];
#pragma unroll
            for (int bi = 0; bi < TI; ++bi) av[bi] = gk * g1p[bi];
#pragma unroll
            for (int bj = 0; bj < TJ; ++bj) bv[bj] = g2p[bj];
#pragma unroll
            for (int bi = 0; bi < TI; ++bi)
#pragma unroll
              for (int bj = 0; bj < TJ; ++bj)
                al[bi][bj] = __builtin_amdgcn_mfma_f32_4x4x1f32(av[bi], bv[bj], al[bi][bj], 0, 0, 0);
          }
        }
      }
      // no wave sync here: each lane reads back only the L rows it wrote itself
    }

    // ---- explicit residual and outputs
    float rr = 0.f;
#pragma unroll
    for (int u = 0; u < M / kQLanes; ++u) {
      const int e = cs + kQLanes * u;
      const int p = e % M1, q = e / M1;
      float r = y[e];
#pragma unroll
      for (int k = 0; k < S; ++k) r -= x[k] * sD1[p + C::LD1 * ia[k]] * sD2[q + C::LD2 * ja[k]];
      rr += r * r;
    }
    rr = row_sum(rr);
    if (valid) {
      const int64_t k = k0 + g;
#pragma unroll
      for (int t = 0; t < S; ++t) {
        if (t == cs) {
          a.supp[k * S + t] = t < nsel ? ia[t] + N1 * ja[t] : -1;
          a.coef[k * S + t] = t < nsel ? x[t] : 0.f;
        }
      }
      if (cs == 0) {
        if (a.res2) a.res2[k] = rr;
        n_early += nsel < S ? 1u : 0u;
      }
    }
    wave_sync();  // the next group's staging overwrites ys
  }
  if (n_early) atomicAdd(&a.counters[kCtrEarlyStop], (unsigned long long)n_early);
}

template <class C>
hipError_t launch_qcfg(const OmpArgs<float>& a, hipStream_t st) {
  const int64_t ngroups = (a.N + kQSigs - 1) / kQSigs;
  int64_t blocks = (ngroups + kQWaves - 1) / kQWaves;
  if (blocks > kQMaxBlocks) blocks = kQMaxBlocks;
  hipLaunchKernelGGL(omp_quad_kernel<C>, dim3((unsigned)blocks), dim3(kWave * kQWaves), 0, st, a);
  return hipGetLastError();
}

struct QuadVariant {
  int m1, m2, n1, n2, s;
  hipError_t (*f)(const OmpArgs<float>&, hipStream_t);
};

// Shapes with a quadrant kernel: (m1, m2, n1, n2, s)
#define SDL_QUAD_SHAPES(X) X(12, 12, 24, 24, 12) X(12, 12, 20, 20, 10)

const QuadVariant kQuadVariants[] = {
#define X(A_, B_, C_, D_, E_) {A_, B_, C_, D_, E_, &launch_qcfg<QCfg<A_, B_, C_, D_, E_>>},
    SDL_QUAD_SHAPES(X)
#undef X
};

const QuadVariant* find_quad(int m1, int m2, int n1, int n2, int s) {
  for (const QuadVariant& v : kQuadVariants)
    if (v.m1 == m1 && v.m2 == m2 && v.n1 == n1 && v.n2 == n2 && v.s == s) return &v;
  return nullptr;
}

}  // namespace

bool omp_quad_supported(int m1, int m2, int n1, int n2, int s) { return find_quad(m1, m2, n1, n2, s) != nullptr; }

hipError_t launch_omp_quad(const OmpArgs<float>& a, hipStream_t st) {
  const QuadVariant* v = find_quad(a.m1, a.m2, a.n1, a.n2, a.s);
  if (!v || a.index || a.sums_side) return hipErrorInvalidValue;
  if (a.N == 0) return hipSuccess;
  return v->f(a, st);
}

}  // namespace sdl
