// Register-resident FP32 2D-OMP for fixed shapes (the image-patch workloads).
//
// Same method and Gram-form recurrences as omp_generic.hip (2D-OMP, Sec. III
// step 1; Gram entries G1[i,i'] G2[j,j'], text after Algorithm 1), mapped for
// CDNA4 throughput instead of generality:
//
//  * A group of LG = LR*LC consecutive lanes owns one signal; SPW = 64/LG signals
//    run side by side in one wave64.  Lane (sr, sc) of a group holds the
//    correlations of atoms (i, j) with i = sr + LR*ri, j = sc + LC*cj in
//    registers (E = N1*N2/LG values), so the correlation refresh, the largest
//    |corr| search and the first correlation are plain register arithmetic.
//  * The Cholesky factor of the support Gram matrix, the coefficients and the
//    support live in registers of every lane of the group (computed
//    redundantly: free in SIMD); the shape and s are template parameters so the
//    greedy loop is fully unrolled and every register index is static.
//  * G1, G2, D1, D2 sit in LDS once per workgroup, with G1/G2 also stored in a
//    lane-permuted order so each refresh term is two contiguous LDS reads.
//  * Each signal's 2D block is staged through LDS with 16-byte coalesced loads.
//  * Selected atoms are not masked explicitly: after the least-squares re-fit
//    their correlation with the residual is zero up to rounding, so they cannot
//    win while any unselected atom has a correlation above rounding level; if
//    the search ever returns a selected atom the signal stops (same as the
//    stop rule).  The FP64 reference masks explicitly; both agree whenever the
//    stop threshold is above rounding level.
//  * Pivots below pivot_fp64 * G_aa are recomputed in FP64 (cancellation in
//    G_aa - |w|^2).
#include <limits.h>

#include <iterator>
#include <vector>

#include "sdl_internal.h"

namespace sdl {
namespace {

constexpr int kFastWaves = 4;  // waves per workgroup
constexpr int kFastMaxBlocks = 1024;

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int M1_, int M2_, int N1_, int N2_, int S_, int LR_, int LC_, int WPE_>
struct Cfg {
  static constexpr int M1 = M1_, M2 = M2_, N1 = N1_, N2 = N2_, S = S_, LR = LR_, LC = LC_;
  static constexpr int WPE = WPE_;  // register budget: target waves per SIMD (1 = unconstrained)
  static constexpr int LG = LR * LC;
  static constexpr int SPW = 64 / LG;
  static constexpr int NRI = N1 / LR, NCJ = N2 / LC, E = NRI * NCJ;
  static constexpr int M = M1 * M2;
  // first correlation association: (D1^T Y) D2 when lanes split rows, D1^T (Y D2) when they split columns
  static constexpr bool ROWFIRST = (NRI * M2 * M1 + E * M2) <= (NCJ * M1 * M2 + E * M1);
  static constexpr int NL = S * (S + 1) / 2;
  // epilogue TMOD sums: tiles over either side's atoms / signal rows, signals per MFMA pass
  static constexpr int NAX = N1 > N2 ? N1 : N2, MRX = M1 > M2 ? M1 : M2;
  static constexpr int TPX = (NAX + 15) / 16, TRX = (MRX + 15) / 16, NPX = 16 * TPX + 1;
  // signals per epilogue pass: keep the per-wave Tcat near 8 KiB
  static constexpr int SUB = (SPW * MRX * NPX <= 2048) ? SPW
                             : (SPW / 2 * MRX * NPX <= 2048 || SPW / 2 <= 1) ? (SPW / 2 > 0 ? SPW / 2 : 1)
                             : (SPW / 4 * MRX * NPX <= 2048 || SPW / 4 <= 1) ? (SPW / 4 > 0 ? SPW / 4 : 1)
                             : (SPW / 8 > 0 ? SPW / 8 : 1);
  // per-wave LDS work area: the Cholesky factors during the greedy loop, Tcat in the epilogue
  static constexpr int WORK = SPW * NL > SUB * MRX * NPX ? SPW * NL : SUB * MRX * NPX;
  // epilogue accumulators live in LDS between groups: (TPX*TPX + TRX*TPX) tiles x 4 values x 64 lanes
  static constexpr int NTILE = TPX * TPX + TRX * TPX;
  // block reduction buffer (kFastWaves rows of the largest side's entry count + 1), aliased on the staging area
  static constexpr int NENTX = NAX * NAX + MRX * NAX + 1;
  static constexpr int STAGE = (SPW * M * 4 > NENTX * 4) ? SPW * M : NENTX;
  static_assert(N1 % LR == 0 && N2 % LC == 0 && 64 % LG == 0, "lane split must tile the atoms");
  static_assert(M % 4 == 0, "signals are staged in 16-byte chunks");
};

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int LG>
__device__ inline float group_sum(float v) {
#pragma unroll
  for (int o = 1; o < LG; o <<= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

constexpr int tri(int k, int l) { return k * (k + 1) / 2 + l; }  // packed lower-triangular index

template <class C>
__global__ void __launch_bounds__(kWave* kFastWaves) __attribute__((amdgpu_waves_per_eu(C::WPE, C::WPE)))
    omp_fast_kernel(OmpArgs<float> a) {
  constexpr int M1 = C::M1, M2 = C::M2, N1 = C::N1, N2 = C::N2, S = C::S, LR = C::LR, LC = C::LC;
  constexpr int LG = C::LG, SPW = C::SPW, NRI = C::NRI, NCJ = C::NCJ, E = C::E, M = C::M;
  __shared__ float sG1[N1 * N1];
  __shared__ float sG2[N2 * N2];
  __shared__ __align__(16) float sG1P[N1 * N1];  // [ik][sr][ri] = G1[sr + LR*ri, ik]
  __shared__ __align__(16) float sG2P[N2 * N2];  // [jk][sc][cj] = G2[jk, sc + LC*cj]
  __shared__ __align__(16) float sD1[M1 * N1];
  __shared__ __align__(16) float sD2[M2 * N2];
  __shared__ __align__(16) float sY[kFastWaves][C::STAGE];
  // per wave: packed lower-triangular Cholesky factors of its signals (greedy loop), then
  // Tcat with one column per (signal, c) (epilogue); the two phases are separated by a wave sync
  __shared__ float sWork[kFastWaves][C::WORK];
  __shared__ float sAcc[kFastWaves][C::NTILE * 4 * kWave];  // epilogue accumulators, lane-major
  __shared__ double sRacc[kFastWaves];

  const int tid = threadIdx.x, wv = tid / kWave, lane = tid % kWave;
  const int g = lane / LG, sub = lane % LG, sr = sub / LC, sc = sub % LC;

  for (int e = tid; e < N1 * N1; e += blockDim.x) {
    sG1[e] = a.G1[e];
    const int ik = e / N1, rem = e % N1, r_sr = rem / NRI, ri = rem % NRI;
    sG1P[e] = a.G1[(r_sr + LR * ri) + N1 * ik];
  }
  for (int e = tid; e < N2 * N2; e += blockDim.x) {
    sG2[e] = a.G2[e];
    const int jk = e / N2, rem = e % N2, r_sc = rem / NCJ, cj = rem % NCJ;
    sG2P[e] = a.G2[jk + N2 * (r_sc + LC * cj)];
  }
  for (int e = tid; e < M1 * N1; e += blockDim.x) sD1[e] = a.D1[e];
  for (int e = tid; e < M2 * N2; e += blockDim.x) sD2[e] = a.D2[e];
  __syncthreads();

  const int lane_base = sr + N1 * sc;  // atom index of local element (ri, cj) = lane_base + LR*ri + N1*LC*cj
  const float stop_rel = (float)a.stop_rel, dep_eps = (float)a.dep_eps, piv = (float)a.pivot_fp64;

  const int64_t nsig = a.index ? (int64_t)*a.count : a.N;  // signals to code
  const int64_t ngroups = (nsig + SPW - 1) / SPW;
  float* ys = sY[wv];
  // epilogue accumulators (the next dictionary update's sums and sum of res2)
  const int eside = a.sums_side;
  const int ena = eside == 2 ? N2 : N1, emr = eside == 2 ? M2 : M1, emc = eside == 2 ? M1 : M2;
  const float* eDo = eside == 2 ? sD1 : sD2;  // fixed dictionary: emc x (other atoms), column-major
  f32x4* acc = reinterpret_cast<f32x4*>(sAcc[wv]) + lane;  // tile q of this lane at acc[q * kWave]
#pragma unroll
  for (int q = 0; q < C::NTILE; ++q) acc[q * kWave] = f32x4{0.f, 0.f, 0.f, 0.f};
  double racc = 0.0;
  unsigned n_early = 0;  // early-stopped signals seen by this lane, counted once at the end
  for (int64_t grp = (int64_t)blockIdx.x * kFastWaves + wv; grp < ngroups; grp += (int64_t)gridDim.x * kFastWaves) {
    const int64_t k0 = grp * SPW;
    const int nvalid = (int)((nsig - k0) < SPW ? (nsig - k0) : SPW);
    // ---- stage the wave's signals through LDS, 16-byte chunks (contiguous, or gathered by index)
    {
      float4* dst = reinterpret_cast<float4*>(ys);
      const int nchunk = nvalid * M / 4;
      for (int e = lane; e < SPW * M / 4; e += kWave) {
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (e < nchunk) {
          const int b = e / (M / 4), off = e % (M / 4);
          const int64_t k = a.index ? (int64_t)a.index[k0 + b] : k0 + b;
          v = load_signal4(a, k * M + 4 * off);
        }
        dst[e] = v;
      }
    }
    wave_sync();
    const float* y = ys + g * M;
    const bool valid = g < nvalid;

    // ---- ||Y||_F and first correlation C = D1^T Y D2 (registers)
    float yy = 0.f;
#pragma unroll
    for (int e = sub; e < M; e += LG) yy += y[e] * y[e];  // (runtime start; M/LG iterations)
    const float ynorm = sqrtf(group_sum<LG>(yy));
    float al[E];
#pragma unroll
    for (int e = 0; e < E; ++e) al[e] = 0.f;
    if constexpr (C::ROWFIRST) {
      // W = D1^T Y for this lane's rows (NRI x M2), then al = W D2
#pragma unroll
      for (int q = 0; q < M2; ++q) {
        float w[NRI];
#pragma unroll
        for (int ri = 0; ri < NRI; ++ri) w[ri] = 0.f;
#pragma unroll
        for (int p = 0; p < M1; ++p) {
          const float yv = y[p + M1 * q];
#pragma unroll
          for (int ri = 0; ri < NRI; ++ri) w[ri] += sD1[p + M1 * (sr + LR * ri)] * yv;
        }
#pragma unroll
        for (int cj = 0; cj < NCJ; ++cj) {
          const float d = sD2[q + M2 * (sc + LC * cj)];
#pragma unroll
          for (int ri = 0; ri < NRI; ++ri) al[cj * NRI + ri] += w[ri] * d;
        }
      }
    } else {
      // V = Y D2 for this lane's columns (M1 x NCJ), then al = D1^T V
#pragma unroll
      for (int p = 0; p < M1; ++p) {
        float v[NCJ];
#pragma unroll
        for (int cj = 0; cj < NCJ; ++cj) v[cj] = 0.f;
#pragma unroll
        for (int q = 0; q < M2; ++q) {
          const float yv = y[p + M1 * q];
#pragma unroll
          for (int cj = 0; cj < NCJ; ++cj) v[cj] += yv * sD2[q + M2 * (sc + LC * cj)];
        }
#pragma unroll
        for (int ri = 0; ri < NRI; ++ri) {
          const float d = sD1[p + M1 * (sr + LR * ri)];
#pragma unroll
          for (int cj = 0; cj < NCJ; ++cj) al[cj * NRI + ri] += d * v[cj];
        }
      }
    }

    // ---- greedy loop, fully unrolled over the support size
    float* L = sWork[wv] + g * C::NL;  // packed lower-triangular factor (diagonal unused; dinv holds 1/L_kk)
    float dinv[S];
    float x[S];
    int ia[S], ja[S];
#pragma unroll
    for (int k = 0; k < S; ++k) { x[k] = 0.f; ia[k] = 0; ja[k] = 0; dinv[k] = 0.f; }
    bool active = valid;
    int nsel = 0;
    const float stop_thr = stop_rel * ynorm;

#pragma unroll
    for (int t = 0; t < S; ++t) {
      // largest |corr| in this lane, scanning in increasing atom index (ties -> smallest)
      float bv = -1.f, bs = 0.f;
      int ba = 0;
#pragma unroll
      for (int cj = 0; cj < NCJ; ++cj)
#pragma unroll
        for (int ri = 0; ri < NRI; ++ri) {
          const float v = al[cj * NRI + ri];
          const float av = fabsf(v);
          const bool c = av > bv;
          bv = c ? av : bv;
          bs = c ? v : bs;
          ba = c ? (LR * ri + N1 * LC * cj) : ba;
        }
      ba += lane_base;
#pragma unroll
      for (int o = 1; o < LG; o <<= 1) {
        const float ov = __shfl_xor(bv, o, kWave);
        const float os = __shfl_xor(bs, o, kWave);
        const int oa = __shfl_xor(ba, o, kWave);
        const bool c = ov > bv || (ov == bv && oa < ba);
        bv = c ? ov : bv;
        bs = c ? os : bs;
        ba = c ? oa : ba;
      }
      bool stop = !(bv > stop_thr);
#pragma unroll
      for (int k = 0; k < t; ++k) stop = stop || (ba == ia[k] + N1 * ja[k]);
      if (stop) active = false;
      const int it = ba % N1, jt = ba / N1;
      // The step runs in every lane (a stopped signal computes values it never commits), so
      // the common path has no branches: results are committed with selects below.
      float w[S > 1 ? S - 1 : 1];
      float d2;
      {
        const float gaa = sG1[it + N1 * it] * sG2[jt + N2 * jt];
        float ww = 0.f;
#pragma unroll
        for (int k = 0; k < t; ++k) {
          float b = sG1[ia[k] + N1 * it] * sG2[ja[k] + N2 * jt];
#pragma unroll
          for (int l = 0; l < k; ++l) b -= L[tri(k, l)] * w[l];
          w[k] = b * dinv[k];
          ww += w[k] * w[k];
        }
        d2 = gaa - ww;
        if (active && d2 < piv * gaa) {
          // small pivot: this row again in FP64
          double w64[S > 1 ? S - 1 : 1];
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < t; ++k) {
            double b = (double)sG1[ia[k] + N1 * it] * (double)sG2[ja[k] + N2 * jt];
#pragma unroll
            for (int l = 0; l < k; ++l) b -= (double)L[tri(k, l)] * w64[l];
            w64[k] = b * (double)dinv[k];
            acc += w64[k] * w64[k];
          }
#pragma unroll
          for (int k = 0; k < t; ++k) w[k] = (float)w64[k];
          d2 = (float)((double)gaa - acc);
          if (sub == 0) atomicAdd(&a.counters[kCtrFp64Pivot], 1ull);
        }
        if (!(d2 > dep_eps * gaa)) active = false;
      }
      {
        // v = L^{-T} w ; coefficients x_S -= c v, x_t = c with c = corr_a / delta^2
        float v[S > 1 ? S - 1 : 1];
#pragma unroll
        for (int k = t - 1; k >= 0; --k) {
          float b = w[k];
#pragma unroll
          for (int l = k + 1; l < t; ++l) b -= L[tri(l, k)] * v[l];
          v[k] = b * dinv[k];
        }
        const float cst = bs / d2;
        // every lane of the group writes the same row: no divergent store
#pragma unroll
        for (int k = 0; k < t; ++k) {
          L[tri(t, k)] = w[k];
          x[k] = active ? x[k] - cst * v[k] : x[k];
        }
        dinv[t] = rsqrtf(d2);
        x[t] = active ? cst : 0.f;
        ia[t] = active ? it : 0;
        ja[t] = active ? jt : 0;
        nsel = active ? t + 1 : nsel;
        if (t + 1 < S) {
          // corr <- corr - c * (G_{:,a} - G_{:,S} v): t+1 rank-one terms gamma_k g1_k g2_k^T
#pragma unroll
          for (int k = 0; k <= t; ++k) {
            const float gk = k == t ? cst : -cst * v[k < t ? k : 0];
            const int ik = k == t ? it : ia[k];
            const int jk = k == t ? jt : ja[k];
            float u[NRI], g2v[NCJ];
            const float* g1p = sG1P + ik * N1 + sr * NRI;
            const float* g2p = sG2P + jk * N2 + sc * NCJ;
#pragma unroll
            for (int ri = 0; ri < NRI; ++ri) u[ri] = gk * g1p[ri];
#pragma unroll
            for (int cj = 0; cj < NCJ; ++cj) g2v[cj] = g2p[cj];
#pragma unroll
            for (int cj = 0; cj < NCJ; ++cj)
#pragma unroll
              for (int ri = 0; ri < NRI; ++ri) al[cj * NRI + ri] -= u[ri] * g2v[cj];
          }
        }
      }
      // no wave sync here: each lane reads back only the L rows it wrote itself
    }

    // ---- explicit residual and outputs
    float rr = 0.f;
#pragma unroll
    for (int e0 = 0; e0 < M; e0 += LG) {
      const int e = e0 + sub;
      if (e < M) {
        const int p = e % M1, q = e / M1;
        float r = y[e];
#pragma unroll
        for (int k = 0; k < S; ++k) r -= x[k] * sD1[p + M1 * ia[k]] * sD2[q + M2 * ja[k]];
        rr += r * r;
      }
    }
    rr = group_sum<LG>(rr);
    if (valid) {
      const int64_t k = a.index ? (int64_t)a.index[k0 + g] : k0 + g;
#pragma unroll
      for (int t = 0; t < S; ++t) {
        if (t % LG == sub) {
          a.supp[k * S + t] = t < nsel ? ia[t] + N1 * ja[t] : -1;
          a.coef[k * S + t] = t < nsel ? x[t] : 0.f;
        }
      }
      if (sub == 0) {
        if (a.res2) a.res2[k] = rr;
        n_early += nsel < S ? 1u : 0u;
        racc += (double)rr;
      }
    }
    if (eside) {
      // Tcat = [T_1 .. T_SUB] for side 1 (T = X D2^T) or side 2 (T = (D1 X)^T), one
      // column per (signal, c); then A += Tcat Tcat^T, B += Ycat Tcat^T on the matrix cores
      const int r16 = lane % 16, kq = lane / 16;
      float* tc = sWork[wv];
      f32x4 accP[C::TPX][C::TPX], accR[C::TRX][C::TPX];
#pragma unroll
      for (int i = 0; i < C::TPX; ++i)
#pragma unroll
        for (int j = 0; j < C::TPX; ++j) accP[i][j] = acc[(i * C::TPX + j) * kWave];
#pragma unroll
      for (int i = 0; i < C::TRX; ++i)
#pragma unroll
        for (int j = 0; j < C::TPX; ++j) accR[i][j] = acc[(C::TPX * C::TPX + i * C::TPX + j) * kWave];
#pragma unroll
      for (int pass = 0; pass < SPW; pass += C::SUB) {
        if (g >= pass && g < pass + C::SUB) {
          for (int c = sub; c < emc; c += LG) {
            float* col = tc + ((g - pass) * emc + c) * C::NPX;
            for (int r = 0; r < C::NPX; ++r) col[r] = 0.f;
#pragma unroll
            for (int t = 0; t < S; ++t) {
              const int ra = eside == 1 ? ia[t] : ja[t], rb = eside == 1 ? ja[t] : ia[t];
              col[ra] += x[t] * eDo[c + emc * rb];
            }
          }
        }
        wave_sync();
        for (int kk = 0; kk < C::SUB * emc; kk += 4) {
          const int kx = kk + kq;
          const int b = pass + kx / emc, c = kx % emc;
          float at[C::TPX], ay[C::TRX];
#pragma unroll
          for (int i = 0; i < C::TPX; ++i) at[i] = tc[kx * C::NPX + 16 * i + r16];
#pragma unroll
          for (int i = 0; i < C::TRX; ++i) {
            const int row = 16 * i + r16;
            ay[i] = row < emr ? (eside == 1 ? ys[b * M + c * M1 + row] : ys[b * M + c + M1 * row]) : 0.f;
          }
#pragma unroll
          for (int i = 0; i < C::TPX; ++i)
#pragma unroll
            for (int j = 0; j < C::TPX; ++j)
              accP[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(at[i], at[j], accP[i][j], 0, 0, 0);
#pragma unroll
          for (int i = 0; i < C::TRX; ++i)
#pragma unroll
            for (int j = 0; j < C::TPX; ++j)
              accR[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ay[i], at[j], accR[i][j], 0, 0, 0);
        }
        wave_sync();
      }
#pragma unroll
      for (int i = 0; i < C::TPX; ++i)
#pragma unroll
        for (int j = 0; j < C::TPX; ++j) acc[(i * C::TPX + j) * kWave] = accP[i][j];
#pragma unroll
      for (int i = 0; i < C::TRX; ++i)
#pragma unroll
        for (int j = 0; j < C::TPX; ++j) acc[(C::TPX * C::TPX + i * C::TPX + j) * kWave] = accR[i][j];
    }
    wave_sync();  // the staging buffer is rewritten by the next group
  }
  if (n_early) atomicAdd(&a.counters[kCtrEarlyStop], (unsigned long long)n_early);
  if (eside) {
    // one partial row per workgroup: [A (na x na) | B (mr x na)] column-major, then sum of
    // res2; the four waves' values are added in wave order
    const int nent = ena * ena + emr * ena;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) racc += __shfl_xor(racc, o, kWave);
    if (lane == 0) sRacc[wv] = racc;
    __syncthreads();  // every wave is done with its staging area
    float* red = sY[0];  // kFastWaves x nent, spans the staging areas
    const int col = lane % 16;
#pragma unroll
    for (int i = 0; i < C::TPX; ++i)
#pragma unroll
      for (int j = 0; j < C::TPX; ++j) {
        const f32x4 v4 = acc[(i * C::TPX + j) * kWave];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * i + 4 * (lane / 16) + v, c = 16 * j + col;
          if (r < ena && c < ena) red[wv * nent + r + ena * c] = v4[v];
        }
      }
#pragma unroll
    for (int i = 0; i < C::TRX; ++i)
#pragma unroll
      for (int j = 0; j < C::TPX; ++j) {
        const f32x4 v4 = acc[(C::TPX * C::TPX + i * C::TPX + j) * kWave];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * i + 4 * (lane / 16) + v, c = 16 * j + col;
          if (r < emr && c < ena) red[wv * nent + ena * ena + r + emr * c] = v4[v];
        }
      }
    __syncthreads();
    double* row = a.sums_part + (size_t)blockIdx.x * (nent + 1);
    for (int e = tid; e < nent; e += blockDim.x) {
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < kFastWaves; ++q) v += (double)red[q * nent + e];
      row[e] = v;
    }
    if (tid == 0) row[nent] = ((sRacc[0] + sRacc[1]) + sRacc[2]) + sRacc[3];
  }
}

int g_num_cus = 256;

// persistent grid: one workgroup per SIMD slot the variant's register budget allows
int64_t fast_blocks(int64_t N, int spw, int wpe) {
  const int64_t ngroups = (N + spw - 1) / spw;
  int64_t blocks = (ngroups + kFastWaves - 1) / kFastWaves;
  const int64_t cap = (int64_t)g_num_cus * (wpe > 1 ? wpe : 1);
  if (blocks > cap) blocks = cap;
  if (blocks > kFastMaxBlocks) blocks = kFastMaxBlocks;
  if (blocks < 1) blocks = 1;
  return blocks;
}

template <class C>
hipError_t launch_cfg(const OmpArgs<float>& a, hipStream_t st) {
  const int64_t blocks = fast_blocks(a.N, C::SPW, C::WPE);
  hipLaunchKernelGGL(omp_fast_kernel<C>, dim3((unsigned)blocks), dim3(kWave * kFastWaves), 0, st, a);
  return hipGetLastError();
}

// Register-resident instantiations: shape (m1, m2, n1, n2, s) and the variants the
// autotuner chooses from (lane split LR x LC, register budget in waves per SIMD).
#define SDL_FAST_VARIANTS(X)                                                        \
  X(8, 8, 16, 16, 8, 1, 4, 1) X(8, 8, 16, 16, 8, 1, 4, 2) X(8, 8, 16, 16, 8, 2, 4, 2) \
  X(8, 8, 16, 16, 8, 2, 4, 3) X(8, 8, 16, 16, 6, 1, 4, 2) X(8, 8, 16, 16, 6, 2, 4, 3) \
  X(8, 8, 12, 12, 4, 1, 4, 3) X(12, 12, 20, 20, 10, 1, 4, 1) X(12, 12, 20, 20, 10, 2, 4, 2) \
  X(12, 12, 24, 24, 12, 2, 4, 1) X(12, 12, 24, 24, 12, 4, 4, 2) \
  X(16, 16, 32, 32, 16, 4, 4, 1) X(16, 16, 32, 32, 16, 4, 8, 2)

struct Variant {
  int m1, m2, n1, n2, s, lr, lc, wpe, mfma;
  hipError_t (*launch)(const OmpArgs<float>&, hipStream_t);
};

const Variant kValuVariants[] = {
#define X(A_, B_, C_, D_, E_, F_, G_, H_) {A_, B_, C_, D_, E_, F_, G_, H_, 0, &launch_cfg<Cfg<A_, B_, C_, D_, E_, F_, G_, H_>>},
    SDL_FAST_VARIANTS(X)
#undef X
};

// all variants: the VALU layouts above, then the matrix-core layouts (lanes 1 x 4)
const std::vector<Variant>& variants() {
  static const std::vector<Variant> v = [] {
    std::vector<Variant> out(std::begin(kValuVariants), std::end(kValuVariants));
    for (int i = 0; i < mfma_variants_count; ++i) {
      const MfmaVariant& m = mfma_variants_table[i];
      out.push_back(Variant{m.m1, m.m2, m.n1, m.n2, m.s, 1, 4, m.wpe, 1, m.launch});
    }
    return out;
  }();
  return v;
}

}  // namespace

template <>
bool omp_fast_supported<float>(int m1, int m2, int n1, int n2, int s) {
  return omp_fast_variants(m1, m2, n1, n2, s, nullptr, 0) > 0;
}

template <>
bool omp_fast_supported<double>(int, int, int, int, int) {
  return false;
}

int omp_fast_partial_rows(int64_t N, int m1, int m2, int n1, int n2, int s) {
  const int id = omp_fast_choice(m1, m2, n1, n2, s);
  if (id < 0) return 0;
  const Variant& x = variants()[id];
  if (x.mfma) return (int)mfma_partial_rows(N, x.wpe);
  return (int)fast_blocks(N, 64 / (x.lr * x.lc), x.wpe);
}

int omp_fast_max_partial_rows() { return kFastMaxBlocks; }

hipError_t omp_fast_init_device() {
  int dev = 0, n = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess && n > 0) {
    g_num_cus = n;
    mfma_set_cus(n);
    tmod_set_cus(n);
    tmod_bf16_set_cus(n);
  }
  return e;
}

int omp_fast_variants(int m1, int m2, int n1, int n2, int s, int* ids, int cap) {
  int n = 0;
  const std::vector<Variant>& vs = variants();
  for (int v = 0; v < (int)vs.size(); ++v) {
    const Variant& x = vs[v];
    if (x.m1 == m1 && x.m2 == m2 && x.n1 == n1 && x.n2 == n2 && x.s == s) {
      if (ids && n < cap) ids[n] = v;
      ++n;
    }
  }
  return n;
}

void omp_fast_variant_info(int id, int* lr, int* lc, int* wpe, int* mfma) {
  const Variant& x = variants()[id];
  *lr = x.lr;
  *lc = x.lc;
  *wpe = x.wpe;
  if (mfma) *mfma = x.mfma;
}

hipError_t launch_omp_fast_variant(int id, const OmpArgs<float>& a, hipStream_t st) {
  if (id < 0 || id >= (int)variants().size()) return hipErrorInvalidValue;
  if (a.N == 0) return hipSuccess;
  return variants()[id].launch(a, st);
}

template <>
hipError_t launch_omp_fast<float>(const OmpArgs<float>& a, hipStream_t st) {
  return launch_omp_fast_variant(omp_fast_choice(a.m1, a.m2, a.n1, a.n2, a.s), a, st);
}

template <>
hipError_t launch_omp_fast<double>(const OmpArgs<double>&, hipStream_t) {
  return hipErrorInvalidValue;
}

}  // namespace sdl
