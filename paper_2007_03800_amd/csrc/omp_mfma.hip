// FP32 2D-OMP with the correlation refresh on the matrix cores (shapes with n1, n2
// multiples of 4 and small tile counts).
//
// Same method as omp_fast.hip (2D-OMP, Sec. III step 1; Gram-form refresh with
// G1[i,i'] G2[j,j'], text after Algorithm 1); what changes is the mapping:
//
//  * Four lanes own a signal and a wave codes 16 signals.  The n1 x n2 correlations of
//    a signal are held as (n1/4)(n2/4) tiles of 4x4 in exactly the result layout of
//    the 4x4x1 16-block FP32 MFMA (block = signal, lane c of the block holds column c
//    of each tile), so each rank-one refresh term gamma_k G1[:,i_k] G2[j_k,:] of the
//    Gram-form update is one MFMA per tile, and the first correlation
//    C = D1^T (Y D2) is m1 more rank-one terms, with Y D2 itself formed in the same
//    layout (m2 rank-one terms per 4x4 tile).
//  * Largest |corr| search on packed keys: |corr| with its low 6 mantissa bits
//    replaced by the element's position inside the lane, reduced with 3-input max
//    and two DPP quad permutes.  Correlations within 2^-17 relative of each other
//    are ordered by position instead of value (a near-tie band below FP32's own
//    rounding of the refreshed correlations).
//  * The chosen atom's correlation is recomputed exactly as d1_i^T Y d2_j minus the
//    support's contribution (the Gram entries of the new Cholesky row times x), so
//    coefficients do not inherit the key truncation.
//  * Support, coefficients and the Cholesky factor as in omp_fast.hip; the epilogue
//    accumulates the next dictionary update's sums on the matrix cores.
#include <limits.h>

#include "sdl_internal.h"

namespace sdl {
namespace {

constexpr int kWaves = 4;
constexpr int kMaxBlocks = 1024;
constexpr int kLanes = 4;      // lanes per signal
constexpr int kSigs = 16;      // signals per wave

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int M1_, int M2_, int N1_, int N2_, int S_, int WPE_>
struct MCfg {
  static constexpr int M1 = M1_, M2 = M2_, N1 = N1_, N2 = N2_, S = S_, WPE = WPE_;
  static constexpr int TI = N1 / 4, TJ = N2 / 4, NT = TI * TJ;  // 4x4 tiles
  static constexpr int M = M1 * M2;
  static constexpr int NL = S * (S + 1) / 2;
  // LDS strides padded to odd word counts, so that the 16 signals of a wave (and the
  // atoms they picked) fall into different banks
  static constexpr int YS = M + 1, LD1 = M1 + 1, LD2 = M2 + 1, NLP = NL + 1;
  static constexpr int NAX = N1 > N2 ? N1 : N2, MRX = M1 > M2 ? M1 : M2;
  static constexpr int TPX = (NAX + 15) / 16, TRX = (MRX + 15) / 16, NPX = 16 * TPX + 1;
  // signals per epilogue pass: all 16 at the occupancy of 2 waves per SIMD (LDS is not the
  // limit there), half of them at higher occupancies
  static constexpr int SUB = WPE <= 2 ? kSigs : kSigs / 2;
  static constexpr int WORK = kSigs * NLP > SUB * MRX * NPX ? kSigs * NLP : SUB * MRX * NPX;
  static constexpr int NTILE = TPX * TPX + TRX * TPX;
  static constexpr int NENTX = NAX * NAX + MRX * NAX + 1;
  static constexpr int STAGE = kSigs * YS > NENTX ? kSigs * YS : NENTX;
  static_assert(N1 % 4 == 0 && N2 % 4 == 0, "4x4 tiles");
  static_assert(NT * 4 <= 64, "at most 64 correlations per lane (6-bit position in the keys)");
  static_assert(M % 4 == 0 && M1 % 4 == 0 && M2 % 4 == 0, "staging and 4x4 tiles of Y D2 and of the residual");
};

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// lane xor 1 / xor 2 inside a quad (DPP quad_perm), no LDS round trip
__device__ inline int dpp_x1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true); }
__device__ inline int dpp_x2(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true); }
__device__ inline float dpp_x1f(float v) { return __builtin_bit_cast(float, dpp_x1(__builtin_bit_cast(int, v))); }
__device__ inline float dpp_x2f(float v) { return __builtin_bit_cast(float, dpp_x2(__builtin_bit_cast(int, v))); }
__device__ inline float quad_sum(float v) {
  v += dpp_x1f(v);
  v += dpp_x2f(v);
  return v;
}

constexpr int tri(int k, int l) { return k * (k + 1) / 2 + l; }

__device__ inline unsigned umax3(unsigned a, unsigned b, unsigned c) { return max(max(a, b), c); }

// Epilogue of one group: the group's contribution to the next dictionary update's sums
// (Corollary 1 for SIDE 1, Result 1 for SIDE 2), accumulated on the matrix cores.
// Each signal's T = X D2^T (SIDE 1) or Z^T = (D1 X)^T (SIDE 2) is built column by
// column in LDS (tc): the lane owning a column adds every support element to its row in
// selection order.  Then P += T T^T and R^T += Yt T^T with
// 16x16x4 MFMA over (signal, column) pairs; acc (LDS) carries the accumulators between
// groups.
template <class C, int SIDE>
__device__ inline void sums_epilogue(f32x4* acc, float* tc, const float* ys, const float* Do, const float (&x)[C::S],
                                     const int (&ia)[C::S], const int (&ja)[C::S], int g, int c, int lane) {
  constexpr int M1 = C::M1, S = C::S, TPX = C::TPX, TRX = C::TRX, NPX = C::NPX;
  constexpr int EMC = SIDE == 2 ? C::M1 : C::M2;  // columns of T per signal
  constexpr int EMR = SIDE == 2 ? C::M2 : C::M1;  // rows of the right-hand side
  constexpr int ELD = SIDE == 2 ? C::LD1 : C::LD2;
  static_assert(EMC % kLanes == 0, "columns split over the signal's lanes");
  const int r16 = lane % 16, kq = lane / 16;
  int ra[S];
#pragma unroll
  for (int t = 0; t < S; ++t) ra[t] = SIDE == 1 ? ia[t] : ja[t];
  // NA independent accumulator sets (summed at the end): consecutive 16x16x4 MFMA then do
  // not wait for each other's results
  constexpr int NA = 4;
  f32x4 accP[NA][TPX][TPX], accR[NA][TRX][TPX];
#pragma unroll
  for (int q = 0; q < NA; ++q) {
#pragma unroll
    for (int i = 0; i < TPX; ++i)
#pragma unroll
      for (int j = 0; j < TPX; ++j) accP[q][i][j] = q == 0 ? acc[(i * TPX + j) * kWave] : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < TRX; ++i)
#pragma unroll
      for (int j = 0; j < TPX; ++j)
        accR[q][i][j] = q == 0 ? acc[(TPX * TPX + i * TPX + j) * kWave] : f32x4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int pass = 0; pass < kSigs; pass += C::SUB) {
    if (g >= pass && g < pass + C::SUB) {
#pragma unroll
      for (int u2 = 0; u2 < EMC / kLanes; ++u2) {
        const int cc = c + kLanes * u2;
        float* col = tc + ((g - pass) * EMC + cc) * NPX;
#pragma unroll
        for (int r = 0; r < NPX; ++r) col[r] = 0.f;
#pragma unroll
        for (int t = 0; t < S; ++t) col[ra[t]] += x[t] * Do[cc + ELD * (SIDE == 1 ? ja[t] : ia[t])];
      }
    }
    wave_sync();
    static_assert((C::SUB * EMC) % (4 * NA) == 0, "whole rounds of the accumulator sets");
    for (int kk = 0; kk < C::SUB * EMC; kk += 4 * NA) {
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const int kx = kk + 4 * q + kq;
        const int b = pass + kx / EMC, cc = kx % EMC;
        float at[TPX], ay[TRX];
#pragma unroll
        for (int i = 0; i < TPX; ++i) at[i] = tc[kx * NPX + 16 * i + r16];
#pragma unroll
        for (int i = 0; i < TRX; ++i) {
          const int row = 16 * i + r16;
          ay[i] = row < EMR ? (SIDE == 1 ? ys[b * C::YS + cc * M1 + row] : ys[b * C::YS + cc + M1 * row]) : 0.f;
        }
#pragma unroll
        for (int i = 0; i < TPX; ++i)
#pragma unroll
          for (int j = 0; j < TPX; ++j)
            accP[q][i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(at[i], at[j], accP[q][i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < TRX; ++i)
#pragma unroll
          for (int j = 0; j < TPX; ++j)
            accR[q][i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ay[i], at[j], accR[q][i][j], 0, 0, 0);
      }
    }
    wave_sync();
  }
#pragma unroll
  for (int i = 0; i < TPX; ++i)
#pragma unroll
    for (int j = 0; j < TPX; ++j)
      acc[(i * TPX + j) * kWave] = (accP[0][i][j] + accP[1][i][j]) + (accP[2][i][j] + accP[3][i][j]);
#pragma unroll
  for (int i = 0; i < TRX; ++i)
#pragma unroll
    for (int j = 0; j < TPX; ++j)
      acc[(TPX * TPX + i * TPX + j) * kWave] = (accR[0][i][j] + accR[1][i][j]) + (accR[2][i][j] + accR[3][i][j]);
}

template <class C, bool ORTHO = false>
__global__ void __launch_bounds__(kWave* kWaves) __attribute__((amdgpu_waves_per_eu(C::WPE, C::WPE)))
    omp_mfma_kernel(OmpArgs<float> a) {
  constexpr int M1 = C::M1, M2 = C::M2, N1 = C::N1, N2 = C::N2, S = C::S;
  constexpr int TI = C::TI, TJ = C::TJ, NT = C::NT, M = C::M;
  __shared__ float sG1[N1 * N1];
  __shared__ float sG2[N2 * N2];
  __shared__ __align__(16) float sG1P[N1 * N1];  // [ik][c][bi] = G1[4bi + c, ik]
  __shared__ __align__(16) float sG2P[N2 * N2];  // [jk][c][bj] = G2[jk, 4bj + c]
  __shared__ __align__(16) float sD1[C::LD1 * N1];  // D1[p, i] at p + LD1 i
  __shared__ __align__(16) float sD1P[M1 * N1];  // [p][c][bi] = D1[p, 4bi + c]
  __shared__ __align__(16) float sD2[C::LD2 * N2];  // D2[q, j] at q + LD2 j
  __shared__ __align__(16) float sY[kWaves][C::STAGE];
  __shared__ float sWork[kWaves][C::WORK];
  __shared__ float sAcc[kWaves][C::NTILE * 4 * kWave];
  __shared__ double sRacc[kWaves];

  const int tid = threadIdx.x, wv = tid / kWave, lane = tid % kWave;
  const int g = lane / kLanes, c = lane % kLanes;

  for (int e = tid; e < N1 * N1; e += blockDim.x) {
    sG1[e] = a.G1[e];
    const int ik = e / N1, rem = e % N1, cc = rem / TI, bi = rem % TI;
    sG1P[e] = a.G1[(4 * bi + cc) + N1 * ik];
  }
  for (int e = tid; e < N2 * N2; e += blockDim.x) {
    sG2[e] = a.G2[e];
    const int jk = e / N2, rem = e % N2, cc = rem / TJ, bj = rem % TJ;
    sG2P[e] = a.G2[jk + N2 * (4 * bj + cc)];
  }
  for (int e = tid; e < M1 * N1; e += blockDim.x) {
    sD1[e % M1 + C::LD1 * (e / M1)] = a.D1[e];
    const int p = e / N1, rem = e % N1, cc = rem / TI, bi = rem % TI;
    sD1P[e] = a.D1[p + M1 * (4 * bi + cc)];
  }
  for (int e = tid; e < M2 * N2; e += blockDim.x) sD2[e % M2 + C::LD2 * (e / M2)] = a.D2[e];
  __syncthreads();

  const float stop_rel = (float)a.stop_rel, dep_eps = (float)a.dep_eps, piv = (float)a.pivot_fp64;
  const int64_t nsig = a.index ? (int64_t)*a.count : a.N;
  const int64_t ngroups = (nsig + kSigs - 1) / kSigs;
  float* ys = sY[wv];
  const int eside = a.sums_side;
  const int ena = eside == 2 ? N2 : N1, emr = eside == 2 ? M2 : M1;
  f32x4* acc = reinterpret_cast<f32x4*>(sAcc[wv]) + lane;
#pragma unroll
  for (int q = 0; q < C::NTILE; ++q) acc[q * kWave] = f32x4{0.f, 0.f, 0.f, 0.f};
  double racc = 0.0;

  unsigned n_early = 0;  // early-stopped signals seen by this lane, counted once at the end
  for (int64_t grp = (int64_t)blockIdx.x * kWaves + wv; grp < ngroups; grp += (int64_t)gridDim.x * kWaves) {
    const int64_t k0 = grp * kSigs;
    const int nvalid = (int)((nsig - k0) < kSigs ? (nsig - k0) : kSigs);
    {
      // signal b of the group at ys + b * YS
      const int nchunk = nvalid * M / 4;
      for (int e = lane; e < kSigs * M / 4; e += kWave) {
        const int b = e / (M / 4), off = e % (M / 4);
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (e < nchunk) {
          const int64_t k = a.index ? (int64_t)a.index[k0 + b] : k0 + b;
          v = load_signal4(a, k * M + 4 * off);
        }
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

    // ---- ||Y|| and C = D1^T (Y D2) into the tile registers
    float yy = 0.f;
#pragma unroll
    for (int u = 0; u < M / kLanes; ++u) {
      const float v = y[c * (M / kLanes) + u];
      yy += v * v;
    }
    const float ynorm = sqrtf(quad_sum(yy));
    f32x4 al[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) al[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    // V = Y D2 on the matrix cores, in 4x4 tiles (rows 4bp + v, columns 4bj + c): lane c
    // supplies Y[4bp + c, q] and D2[q, 4bj + c] for each rank-one term q.  Register v of tile
    // (bp, bj) in lane c is then V[4bp + v, 4bj + c], exactly the B operand the second stage
    // C = D1^T V needs for row p = 4bp + v.
    f32x4 vt[M1 / 4][TJ];
#pragma unroll
    for (int bp = 0; bp < M1 / 4; ++bp)
#pragma unroll
      for (int bj = 0; bj < TJ; ++bj) vt[bp][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < M2; ++q) {
      float ya[M1 / 4], db[TJ];
#pragma unroll
      for (int bp = 0; bp < M1 / 4; ++bp) ya[bp] = y[(4 * bp + c) + M1 * q];
#pragma unroll
      for (int bj = 0; bj < TJ; ++bj) db[bj] = sD2[q + C::LD2 * (4 * bj + c)];
#pragma unroll
      for (int bp = 0; bp < M1 / 4; ++bp)
#pragma unroll
        for (int bj = 0; bj < TJ; ++bj)
          vt[bp][bj] = __builtin_amdgcn_mfma_f32_4x4x1f32(ya[bp], db[bj], vt[bp][bj], 0, 0, 0);
    }
#pragma unroll
    for (int p = 0; p < M1; ++p) {
      const float* d1p = sD1P + p * N1 + c * TI;  // D1[p, 4bi + c]
#pragma unroll
      for (int bi = 0; bi < TI; ++bi) {
        const float av = d1p[bi];
#pragma unroll
        for (int bj = 0; bj < TJ; ++bj) {
          const float vb = vt[p / 4][bj][p % 4];  // by value (see the argmax keys)
          al[bi * TJ + bj] = __builtin_amdgcn_mfma_f32_4x4x1f32(av, vb, al[bi * TJ + bj], 0, 0, 0);
        }
      }
    }

    float x[S];
    int ia[S], ja[S];
#pragma unroll
    for (int k = 0; k < S; ++k) { x[k] = 0.f; ia[k] = 0; ja[k] = 0; }
    int nsel = 0;
    if constexpr (ORTHO) {
      // ---- Remark 1's codes: the s largest |C| in decreasing order (ties: smaller atom), exact.
      // Key of an element: its |C| bits above 16 bits holding 65535 - atom, compared as 64-bit
      // integers; chosen elements drop out through the lane's taken mask.
      unsigned taken = 0u;
#pragma unroll
      for (int t = 0; t < S; ++t) {
        unsigned long long best = 0ull;
#pragma unroll
        for (int bj = 0; bj < TJ; ++bj)
#pragma unroll
          for (int bi = 0; bi < TI; ++bi)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int e = (bj * TI + bi) * 4 + v;
              const float cv = al[bi * TJ + bj][v];  // by value
              const int atom = (4 * bi + v) + N1 * (4 * bj + c);
              const unsigned long long key =
                  ((unsigned long long)(__float_as_uint(cv) & 0x7FFFFFFFu) << 16) | (unsigned)(0xFFFF - atom);
              const bool ok = !((taken >> e) & 1u) && key > best;
              best = ok ? key : best;
            }
        // the signal's four lanes: quad swaps on both halves of the key
#pragma unroll
        for (int o = 0; o < 2; ++o) {
          const unsigned lo = (unsigned)best, hi = (unsigned)(best >> 32);
          const unsigned olo = (unsigned)(o == 0 ? dpp_x1((int)lo) : dpp_x2((int)lo));
          const unsigned ohi = (unsigned)(o == 0 ? dpp_x1((int)hi) : dpp_x2((int)hi));
          const unsigned long long ok = ((unsigned long long)ohi << 32) | olo;
          best = ok > best ? ok : best;
        }
        const int atom = 0xFFFF - (int)(best & 0xFFFFull);
        const int it = atom % N1, jt = atom / N1;
        const int eo = ((jt / 4) * TI + it / 4) * 4 + it % 4;  // element index in the owner lane
        const bool owner = (jt % 4) == c;
        float val = 0.f;
#pragma unroll
        for (int bj = 0; bj < TJ; ++bj)
#pragma unroll
          for (int bi = 0; bi < TI; ++bi)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int e = (bj * TI + bi) * 4 + v;
              const float cv = al[bi * TJ + bj][v];
              val = (owner && e == eo) ? cv : val;
            }
        taken |= owner ? (1u << eo) : 0u;
        val = quad_sum(val);  // only the owner's value is nonzero
        x[t] = val;
        ia[t] = it;
        ja[t] = jt;
      }
      nsel = valid ? S : 0;
    } else {
    // ---- greedy loop
    float* L = sWork[wv] + g * C::NLP;
    float dinv[S];
#pragma unroll
    for (int k = 0; k < S; ++k) dinv[k] = 0.f;
    bool active = valid;
    const float stop_thr = stop_rel * ynorm;

#pragma unroll
    for (int t = 0; t < S; ++t) {
      // packed keys: |corr| bits with the low 6 bits = 63 - position (position = (bj, bi, v))
      // independent max chains (one per tile row bi), merged at the end: short dependency depth
      unsigned bacc[TI];
#pragma unroll
      for (int bi = 0; bi < TI; ++bi) bacc[bi] = 0u;
#pragma unroll
      for (int bj = 0; bj < TJ; ++bj)
#pragma unroll
        for (int bi = 0; bi < TI; ++bi)
#pragma unroll
          for (int v = 0; v < 4; v += 2) {
            // elements are read by value: a bit cast of a vector-element lvalue reads
            // element 0 with this compiler
            const int e0 = (bj * TI + bi) * 4 + v;
            const float c0 = al[bi * TJ + bj][v], c1 = al[bi * TJ + bj][v + 1];
            const unsigned k0v = (__float_as_uint(c0) & 0x7FFFFFC0u) | (unsigned)(63 - (e0 & 63));
            const unsigned k1v = (__float_as_uint(c1) & 0x7FFFFFC0u) | (unsigned)(63 - ((e0 + 1) & 63));
            bacc[bi] = umax3(bacc[bi], k0v, k1v);
          }
      unsigned best = bacc[0];
#pragma unroll
      for (int bi = 1; bi + 1 < TI; bi += 2) best = umax3(best, bacc[bi], bacc[bi + 1]);
      if (TI % 2 == 0) best = max(best, bacc[TI - 1]);
      // cross-lane: larger key, ties -> smaller lane (c) ; pack lane into a second word
      unsigned bkey = best;
      int blane = c;
      {
        const unsigned ok = (unsigned)dpp_x1((int)bkey);
        const int ol = dpp_x1(blane);
        const bool take = ok > bkey || (ok == bkey && ol < blane);
        bkey = take ? ok : bkey;
        blane = take ? ol : blane;
      }
      {
        const unsigned ok = (unsigned)dpp_x2((int)bkey);
        const int ol = dpp_x2(blane);
        const bool take = ok > bkey || (ok == bkey && ol < blane);
        bkey = take ? ok : bkey;
        blane = take ? ol : blane;
      }
      const int epos = 63 - (int)(bkey & 63u);
      const int v_ = epos & 3, tile = epos >> 2;
      const int bi_ = tile % TI, bj_ = tile / TI;
      const int it = 4 * bi_ + v_, jt = 4 * bj_ + blane;
      const int ba = it + N1 * jt;
      const float babs = __builtin_bit_cast(float, bkey & 0x7FFFFFC0u);
      bool stop = !(babs > stop_thr);
#pragma unroll
      for (int k = 0; k < t; ++k) stop = stop || (ba == ia[k] + N1 * ja[k]);
      if (stop) active = false;
      // The step runs in every lane (a stopped signal computes values it never commits), so
      // the common path has no branches: results are committed with selects below.
      float w[S > 1 ? S - 1 : 1];
      const float gaa = sG1[it + N1 * it] * sG2[jt + N2 * jt];
      float d2;
      {
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
          double w64[S > 1 ? S - 1 : 1];
          double accd = 0.0;
#pragma unroll
          for (int k = 0; k < t; ++k) {
            double b = (double)sG1[ia[k] + N1 * it] * (double)sG2[ja[k] + N2 * jt];
#pragma unroll
            for (int l = 0; l < k; ++l) b -= (double)L[tri(k, l)] * w64[l];
            w64[k] = b * (double)dinv[k];
            accd += w64[k] * w64[k];
          }
#pragma unroll
          for (int k = 0; k < t; ++k) w[k] = (float)w64[k];
          d2 = (float)((double)gaa - accd);
          if (c == 0) atomicAdd(&a.counters[kCtrFp64Pivot], 1ull);
        }
        if (!(d2 > dep_eps * gaa)) active = false;
      }
      // exact correlation of the chosen atom with the residual: d1^T Y d2 - G_{a,S} x_S
      float cor;
      {
        float part = 0.f;
#pragma unroll
        for (int u = 0; u < M2 / kLanes; ++u) {
          const int q = c + kLanes * u;
          float col = 0.f;
#pragma unroll
          for (int p = 0; p < M1; ++p) col += sD1[p + C::LD1 * it] * y[p + M1 * q];
          part += col * sD2[q + C::LD2 * jt];
        }
        cor = quad_sum(part);
#pragma unroll
        for (int k = 0; k < t; ++k) cor -= sG1[ia[k] + N1 * it] * sG2[ja[k] + N2 * jt] * x[k];
      }
      {
        float vv[S > 1 ? S - 1 : 1];
#pragma unroll
        for (int k = t - 1; k >= 0; --k) {
          float b = w[k];
#pragma unroll
          for (int l = k + 1; l < t; ++l) b -= L[tri(l, k)] * vv[l];
          vv[k] = b * dinv[k];
        }
        const float cst = cor / d2;
        // the signal's four lanes write the same row: no divergent store
#pragma unroll
        for (int k = 0; k < t; ++k) {
          L[tri(t, k)] = w[k];
          x[k] = active ? x[k] - cst * vv[k] : x[k];
        }
        dinv[t] = rsqrtf(d2);
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
            const float* g1p = sG1P + ik * N1 + c * TI;  // G1[4bi + c, ik]
            const float* g2p = sG2P + jk * N2 + c * TJ;  // G2[jk, 4bj + c]
            float av[TI], bv[TJ];
#pragma unroll
            for (int bi = 0; bi < TI; ++bi) av[bi] = gk * g1p[bi];
#pragma unroll
            for (int bj = 0; bj < TJ; ++bj) bv[bj] = g2p[bj];
#pragma unroll
            for (int bi = 0; bi < TI; ++bi)
#pragma unroll
              for (int bj = 0; bj < TJ; ++bj)
                al[bi * TJ + bj] = __builtin_amdgcn_mfma_f32_4x4x1f32(av[bi], bv[bj], al[bi * TJ + bj], 0, 0, 0);
          }
        }
      }
      // no wave sync here: each lane reads back only the L rows it wrote itself
    }
    }  // greedy loop

    // ---- explicit residual and outputs
    // D1 X D2^T on the matrix cores: S rank-one terms x_k d1_{i_k} d2_{j_k}^T per 4x4 tile
    // (register v of tile (bp, bq) in lane c: row 4bp + v, column 4bq + c); unused slots add 0
    f32x4 dx[M1 / 4][M2 / 4];
#pragma unroll
    for (int bp = 0; bp < M1 / 4; ++bp)
#pragma unroll
      for (int bq = 0; bq < M2 / 4; ++bq) dx[bp][bq] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < S; ++k) {
      float av[M1 / 4], bv[M2 / 4];
#pragma unroll
      for (int bp = 0; bp < M1 / 4; ++bp) av[bp] = x[k] * sD1[(4 * bp + c) + C::LD1 * ia[k]];
#pragma unroll
      for (int bq = 0; bq < M2 / 4; ++bq) bv[bq] = sD2[(4 * bq + c) + C::LD2 * ja[k]];
#pragma unroll
      for (int bp = 0; bp < M1 / 4; ++bp)
#pragma unroll
        for (int bq = 0; bq < M2 / 4; ++bq)
          dx[bp][bq] = __builtin_amdgcn_mfma_f32_4x4x1f32(av[bp], bv[bq], dx[bp][bq], 0, 0, 0);
    }
    float rr = 0.f;
#pragma unroll
    for (int bp = 0; bp < M1 / 4; ++bp)
#pragma unroll
      for (int bq = 0; bq < M2 / 4; ++bq)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float r = y[(4 * bp + v) + M1 * (4 * bq + c)] - dx[bp][bq][v];
          rr += r * r;
        }
    rr = quad_sum(rr);
    if (valid) {
      const int64_t k = a.index ? (int64_t)a.index[k0 + g] : k0 + g;
#pragma unroll
      for (int t = 0; t < S; ++t) {
        if (t % kLanes == c) {
          a.supp[k * S + t] = t < nsel ? ia[t] + N1 * ja[t] : -1;
          a.coef[k * S + t] = t < nsel ? x[t] : 0.f;
        }
      }
      if (c == 0) {
        if (a.res2) a.res2[k] = rr;
        n_early += nsel < S ? 1u : 0u;
        racc += (double)rr;
      }
    }
    if (eside == 1)
      sums_epilogue<C, 1>(acc, sWork[wv], ys, sD2, x, ia, ja, g, c, lane);
    else if (eside == 2)
      sums_epilogue<C, 2>(acc, sWork[wv], ys, sD1, x, ia, ja, g, c, lane);
    wave_sync();
  }
  if (n_early) atomicAdd(&a.counters[kCtrEarlyStop], (unsigned long long)n_early);
  if (eside) {
    const int nent = ena * ena + emr * ena;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) racc += __shfl_xor(racc, o, kWave);
    if (lane == 0) sRacc[wv] = racc;
    __syncthreads();
    float* red = sY[0];
    const int col = lane % 16;
#pragma unroll
    for (int i = 0; i < C::TPX; ++i)
#pragma unroll
      for (int j = 0; j < C::TPX; ++j) {
        const f32x4 v4 = acc[(i * C::TPX + j) * kWave];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * i + 4 * (lane / 16) + v, cc = 16 * j + col;
          if (r < ena && cc < ena) red[wv * nent + r + ena * cc] = v4[v];
        }
      }
#pragma unroll
    for (int i = 0; i < C::TRX; ++i)
#pragma unroll
      for (int j = 0; j < C::TPX; ++j) {
        const f32x4 v4 = acc[(C::TPX * C::TPX + i * C::TPX + j) * kWave];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * i + 4 * (lane / 16) + v, cc = 16 * j + col;
          if (r < emr && cc < ena) red[wv * nent + ena * ena + r + emr * cc] = v4[v];
        }
      }
    __syncthreads();
    double* row = a.sums_part + (size_t)blockIdx.x * (nent + 1);
    for (int e = tid; e < nent; e += blockDim.x) {
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < kWaves; ++q) v += (double)red[q * nent + e];
      row[e] = v;
    }
    if (tid == 0) row[nent] = ((sRacc[0] + sRacc[1]) + sRacc[2]) + sRacc[3];
  }
}

int g_cus = 256;

int64_t mfma_blocks(int64_t N, int wpe) {
  const int64_t ngroups = (N + kSigs - 1) / kSigs;
  int64_t blocks = (ngroups + kWaves - 1) / kWaves;
  const int64_t cap = (int64_t)g_cus * (wpe > 1 ? wpe : 1);
  if (blocks > cap) blocks = cap;
  if (blocks > kMaxBlocks) blocks = kMaxBlocks;
  if (blocks < 1) blocks = 1;
  return blocks;
}

template <class C>
hipError_t launch_mcfg(const OmpArgs<float>& a, hipStream_t st) {
  const int64_t blocks = mfma_blocks(a.N, C::WPE);
  hipLaunchKernelGGL(omp_mfma_kernel<C>, dim3((unsigned)blocks), dim3(kWave * kWaves), 0, st, a);
  return hipGetLastError();
}

}  // namespace

// Matrix-core variants: (m1, m2, n1, n2, s, waves per SIMD)
#define SDL_MFMA_VARIANTS(X) \
  X(8, 8, 16, 16, 8, 2) X(8, 8, 16, 16, 8, 3) X(8, 8, 16, 16, 8, 4) X(8, 8, 16, 16, 6, 3) X(8, 8, 12, 12, 4, 4)

MfmaVariant mfma_variants_table[] = {
#define X(A_, B_, C_, D_, E_, F_) {A_, B_, C_, D_, E_, F_, &launch_mcfg<MCfg<A_, B_, C_, D_, E_, F_>>},
    SDL_MFMA_VARIANTS(X)
#undef X
};
const int mfma_variants_count = sizeof(mfma_variants_table) / sizeof(mfma_variants_table[0]);

int64_t mfma_partial_rows(int64_t N, int wpe) { return mfma_blocks(N, wpe); }

// Remark 1's orthonormal variant on the same layout: first correlation on the matrix cores,
// exact top-s selection, explicit residual, and the update sums in the epilogue (the B block
// is what the Procrustes update reads).  (m1, m2, s, waves per SIMD); n1 = m1, n2 = m2.
// Three waves per SIMD fit its registers (149) and, with the epilogue in two passes, its LDS:
// 6% faster per orthonormal iteration than two.
#define SDL_ORTHO_MFMA_VARIANTS(X) X(8, 8, 8, 3)

struct OrthoMfmaVariant {
  int m1, m2, s, wpe;
  hipError_t (*launch)(const OmpArgs<float>&, hipStream_t);
};

template <class C>
hipError_t launch_ortho_cfg(const OmpArgs<float>& a, hipStream_t st) {
  const int64_t blocks = mfma_blocks(a.N, C::WPE);
  hipLaunchKernelGGL((omp_mfma_kernel<C, true>), dim3((unsigned)blocks), dim3(kWave * kWaves), 0, st, a);
  return hipGetLastError();
}

const OrthoMfmaVariant kOrthoMfma[] = {
#define X(A_, B_, S_, W_) {A_, B_, S_, W_, &launch_ortho_cfg<MCfg<A_, B_, A_, B_, S_, W_>>},
    SDL_ORTHO_MFMA_VARIANTS(X)
#undef X
};

bool ortho_mfma_supported(int m1, int m2, int n1, int n2, int s) {
  for (const OrthoMfmaVariant& v : kOrthoMfma)
    if (v.m1 == m1 && v.m2 == m2 && n1 == m1 && n2 == m2 && v.s == s) return true;
  return false;
}

int64_t ortho_mfma_partial_rows(int64_t N, int m1, int m2, int s) {
  for (const OrthoMfmaVariant& v : kOrthoMfma)
    if (v.m1 == m1 && v.m2 == m2 && v.s == s) return mfma_blocks(N, v.wpe);
  return 0;
}

hipError_t launch_ortho_mfma(const OmpArgs<float>& a, hipStream_t st) {
  if (a.N == 0) return hipSuccess;
  for (const OrthoMfmaVariant& v : kOrthoMfma)
    if (v.m1 == a.m1 && v.m2 == a.m2 && a.n1 == a.m1 && a.n2 == a.m2 && v.s == a.s) return v.launch(a, st);
  return hipErrorInvalidValue;
}

void mfma_set_cus(int n) {
  if (n > 0) g_cus = n;
}

}  // namespace sdl
