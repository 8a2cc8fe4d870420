// 2D-OMP for large shapes: one wave64 per signal, correlations in registers.
//
// Same method and Gram-form recurrences as omp_generic.hip (2D-OMP, Sec. III step 1;
// Gram entries G1[i,i'] G2[j,j'], text after Algorithm 1), for shapes whose n1 x n2
// correlations do not fit the multi-signal layouts of omp_fast.hip / omp_mfma.hip
// (hundreds to ~2000 atoms, s up to 32):
//
//  * FP64 (omp_wave_kernel): lane (sr, sc) of an LR x LC grid (LR*LC <= 64) holds the
//    correlations of atoms i = sr + LR*ri, j = sc + LC*cj in E = (n1/LR)(n2/LC) registers,
//    so each Gram-form refresh term gamma_k G1[:, i_k] G2[j_k, :] is an E-element rank-one
//    update from NRI + NCJ contiguous LDS reads.  FP32 (omp_wave_mfma_kernel): the
//    correlations sit in 16x16 tiles of the 16x16x4 MFMA result layout (see that kernel).
//  * The least squares is carried by the inverse of the Cholesky factor, L^{-1}, kept
//    in LDS (packed rows with the diagonal).  Appending atom a with Gram column g = G_{S,a}
//    needs w = L^{-1} g (the new row of L), v = L^{-T} w and delta^2 = G_aa - |w|^2; the
//    new row of L^{-1} is [-v^T, 1] / delta.  Both products are matrix-vector products
//    spread over lanes (lane k holds element k of the support, its coefficient and its
//    Gram entry), so a step has no serial triangular solve.
//  * Each step writes the refresh coefficients gamma_q and the support atoms to LDS; the
//    refresh reads them four terms at a time (padding terms have gamma = 0), so their
//    LDS latencies overlap.
//  * Loops over the greedy step and the support are runtime loops: code size does not
//    grow with s.  In FP64 chosen atoms are masked explicitly (one bit per register
//    element), as in the generic kernel and the FP64 reference; in FP32 a repeated pick
//    stops the signal, as in the other FP32 kernels.
//  * FP32 pivots below pivot_fp64 * G_aa are recomputed in FP64.
//  * The error-driven stop (sdl_options.err2, the denoising runs of Sec. IV) tracks the
//    residual energy by the OMP recurrence ||r||^2 -= corr_a^2 / delta^2 from ||Y||^2 and
//    takes no further atom once it is <= err2, as the generic kernel does.
// No TMOD sums epilogue: with this kernel the dictionary updates use the standalone
// sums kernel.  FP32 shapes compiled in omp_quad.hip are dispatched there instead.
#include <limits.h>

#include "sdl_internal.h"

namespace sdl {
namespace {

constexpr int kWaveMaxBlocks = 4096;

typedef float f32x4 __attribute__((ext_vector_type(4)));

// WPB_: signals (waves) per workgroup, chosen per shape so that the dictionary tables
// shared by a workgroup plus its waves' buffers leave room for as many waves per CU as
// the registers allow
// MF_: FP32 on the matrix cores (omp_wave_mfma_kernel) instead of the vector ALUs
template <int M1_, int M2_, int N1_, int N2_, int S_, int LR_, int LC_, int WPB_, bool MF_>
struct WCfg {
  static constexpr int M1 = M1_, M2 = M2_, N1 = N1_, N2 = N2_, S = S_, LR = LR_, LC = LC_, WPB = WPB_;
  static constexpr bool MF = MF_;
  static constexpr int LG = LR * LC, NRI = N1 / LR, NCJ = N2 / LC, E = NRI * NCJ;
  static constexpr int M = M1 * M2;
  static constexpr int NLI = S * (S + 1) / 2;   // packed rows of L^{-1} with the diagonal
  static constexpr int SP = (S + 2 + 3) / 4 * 4;  // support arrays, padded for 4-term batches
  static constexpr int WS = N1 * M2;            // first-correlation staging
  static constexpr int PW = M + WS + NLI + 5 * SP + 1;  // per-wave LDS words (+1: odd stride)
  // occupancy target (waves per SIMD) that bounds the registers of the 4-term refresh
  static constexpr int WPE = E <= 16 ? 4 : (E <= 32 ? 3 : 2);
  static_assert(N1 % LR == 0 && N2 % LC == 0 && LG <= 64, "lane grid must tile the atoms");
  static_assert(E <= 64, "one mask bit per register element");
  static_assert(S <= LG, "support element k lives in lane k of the grid");
};

constexpr int trow(int k) { return k * (k + 1) / 2; }  // row k of packed L^{-1}

template <typename U>
__device__ inline U wave_sum(U v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Appends atom a = (ia, ja) with refreshed correlation bs to the support held by the wave
// (lane k holds support element k: its atom my_i, my_j and coefficient my_x).  With the
// Gram column g = G_{S,a}: w = L^{-1} g, v = L^{-T} w, delta^2 = G_aa - |w|^2 (again in FP64
// below pivot_fp64 G_aa for FP32), c = bs / delta^2; then x_S -= c v, x_a = c, the new row
// of L^{-1} is [-v^T, 1] / delta, and the refresh terms become gamma_q = c v_q (q < t),
// gamma_t = -c.  Returns false, changing nothing, when delta^2 <= dep_eps G_aa (the atom
// is numerically in the span of the support).  Ends with a wave sync: gam, supi, supj
// and the new row are visible to the whole wave.
template <typename T, class C, class G1f, class G2f>
__device__ inline bool append_atom(int t, int lane, int ia, int ja, T bs, G1f g1, G2f g2, T* Li, T* gam, T* supi,
                                   T* supj, T* xg, T* xw, T& my_x, int& my_i, int& my_j, const OmpArgs<T>& a,
                                   T& cst_out) {
  const T gaa = g1(ia, ia) * g2(ja, ja);
  // w = L^{-1} g, lane k < t taking row k
  if (lane < t) xg[lane] = g1(my_i, ia) * g2(ja, my_j);
  wave_sync();
  T w = 0;
  if (lane < t) {
    const T* row = Li + trow(lane);
    T p0 = 0, p1 = 0;
    int l = 0;
    for (; l + 1 <= lane; l += 2) {
      p0 += row[l] * xg[l];
      p1 += row[l + 1] * xg[l + 1];
    }
    if (l <= lane) p0 += row[l] * xg[l];
    w = p0 + p1;
    xw[lane] = w;
  }
  wave_sync();
  // |w|^2 in every lane, v = L^{-T} w in lane l < t (column l of L^{-1})
  T ww = 0, v = 0;
#pragma unroll 4
  for (int k = 0; k < t; ++k) {
    const T wk = xw[k];
    ww += wk * wk;
    if (lane <= k) v += Li[trow(k) + lane] * wk;
  }
  T d2 = gaa - ww;
  if (sizeof(T) == 4 && d2 < (T)a.pivot_fp64 * gaa) {
    // small pivot: w and |w|^2 again in FP64 (cancellation in G_aa - |w|^2)
    double w64 = 0.0;
    if (lane < t) {
      const T* row = Li + trow(lane);
      for (int l = 0; l <= lane; ++l)
        w64 += (double)row[l] * ((double)g1((int)supi[l], ia) * (double)g2(ja, (int)supj[l]));
    }
    const double ww64 = wave_sum(lane < t ? w64 * w64 : 0.0);
    wave_sync();
    if (lane < t) xw[lane] = (T)w64;
    wave_sync();
    v = 0;
    for (int k = 0; k < t; ++k)
      if (lane <= k) v += Li[trow(k) + lane] * xw[k];
    d2 = (T)((double)gaa - ww64);
    if (lane == 0) atomicAdd(&a.counters[kCtrFp64Pivot], 1ull);
  }
  if (!(d2 > (T)a.dep_eps * gaa)) return false;
  const T cst = bs / d2;
  cst_out = cst;
  const T dinv = (T)1 / sqrt(d2);
  T* rowt = Li + trow(t);
  if (lane < t) {
    rowt[lane] = -v * dinv;
    my_x -= cst * v;
    gam[lane] = cst * v;
  }
  if (lane == t) {
    rowt[t] = dinv;
    my_x = cst;
    my_i = ia;
    my_j = ja;
    gam[t] = -cst;
    supi[t] = (T)ia;
    supj[t] = (T)ja;
  }
  wave_sync();
  return true;
}

template <typename T, class C>
__global__ void __launch_bounds__(kWave* C::WPB)
    omp_wave_kernel(OmpArgs<T> a) {
  constexpr int M1 = C::M1, M2 = C::M2, N1 = C::N1, N2 = C::N2, S = C::S, LR = C::LR;
  constexpr int NRI = C::NRI, NCJ = C::NCJ, E = C::E, M = C::M;
  __shared__ T sD1[M1 * N1];                  // D1[p, i] at p + M1 i
  __shared__ T sD2[M2 * N2];                  // D2[q, j] at q + M2 j
  __shared__ __align__(16) T sG1P[N1 * N1];   // [ik][sr][ri] = G1[sr + LR ri, ik]
  __shared__ __align__(16) T sG2P[N2 * N2];   // [jk][sc][cj] = G2[jk, sc + LC cj]
  __shared__ T sW[C::WPB][C::PW];

  const int tid = threadIdx.x, wv = tid / kWave, lane = tid % kWave;
  for (int e = tid; e < M1 * N1; e += blockDim.x) sD1[e] = a.D1[e];
  for (int e = tid; e < M2 * N2; e += blockDim.x) sD2[e] = a.D2[e];
  for (int e = tid; e < N1 * N1; e += blockDim.x) {
    const int ik = e / N1, rem = e % N1, r = rem / NRI, ri = rem % NRI;
    sG1P[e] = a.G1[(r + LR * ri) + N1 * ik];
  }
  for (int e = tid; e < N2 * N2; e += blockDim.x) {
    const int jk = e / N2, rem = e % N2, c = rem / NCJ, cj = rem % NCJ;
    sG2P[e] = a.G2[jk + N2 * (c + C::LC * cj)];
  }
  __syncthreads();

  const bool act = lane < C::LG;
  const int sr = lane % LR, sc = (lane / LR) % C::LC;
  T* ys = sW[wv];
  T* Ws = ys + M;
  T* Li = Ws + C::WS;        // L^{-1}, packed rows with the diagonal
  T* gam = Li + C::NLI;      // refresh coefficients gamma_q (zero beyond the support)
  T* supi = gam + C::SP;     // support atoms i_q, j_q (exact small integers)
  T* supj = supi + C::SP;
  T* xg = supj + C::SP;      // exchange vectors: Gram column g, then w
  T* xw = xg + C::SP;
  // G1[i, i'] and G2[j, j'] from the permuted tables (both are symmetric)
  auto g1 = [&](int i, int ik) { return sG1P[ik * N1 + (i % LR) * NRI + i / LR]; };
  auto g2 = [&](int jk, int j) { return sG2P[jk * N2 + (j % C::LC) * NCJ + j / C::LC]; };

  unsigned n_early = 0;  // early-stopped signals of this wave (lane 0), counted once at the end
  for (int64_t k = (int64_t)blockIdx.x * C::WPB + wv; k < a.N; k += (int64_t)gridDim.x * C::WPB) {
    T yy = 0;
    for (int e = lane; e < M; e += kWave) {
      const T v = a.Yh ? (T)bf16_to_float(a.Yh[k * M + e]) : a.Y[k * M + e];
      ys[e] = v;
      yy += v * v;
    }
    const T yy_all = wave_sum(yy);
    const T ynorm = sqrt(yy_all);
    // residual energy by the OMP recurrence ||r||^2 -= corr_a^2 / pivot (error-driven stop)
    T renergy = yy_all;
    wave_sync();
    // C = (D1^T Y) D2: W = D1^T Y staged in LDS, then each lane's block of C
    for (int e = lane; e < C::WS; e += kWave) {
      const int i = e % N1, q = e / N1;
      T v = 0;
      for (int p = 0; p < M1; ++p) v += sD1[p + M1 * i] * ys[p + M1 * q];
      Ws[e] = v;
    }
    wave_sync();
    // C[i, j] = sum_q W[i, q] D2[q, j] as m2 rank-one updates of the lane's block: the
    // live set stays at the block plus one column and one row
    T corr[E];
#pragma unroll
    for (int e = 0; e < E; ++e) corr[e] = 0;
    if (act) {
#pragma unroll 2
      for (int q = 0; q < M2; ++q) {
        T wi[NRI];
#pragma unroll
        for (int ri = 0; ri < NRI; ++ri) wi[ri] = Ws[(sr + LR * ri) + N1 * q];
#pragma unroll
        for (int cj = 0; cj < NCJ; ++cj) {
          const T d = sD2[q + M2 * (sc + C::LC * cj)];
#pragma unroll
          for (int ri = 0; ri < NRI; ++ri) corr[ri * NCJ + cj] += wi[ri] * d;
        }
      }
    }
    for (int e = lane; e < 3 * C::SP; e += kWave) gam[e] = 0;  // gam, supi, supj
    wave_sync();
    unsigned long long used = 0ull;  // bit e: register element e is a chosen atom
    // support element k lives in lane k
    T my_x = 0;
    int my_i = 0, my_j = 0;
    int t = 0;
    bool early = false;
    const T stop_thr = (T)a.stop_rel * ynorm;
#pragma unroll 1
    for (; t < S; ++t) {
      // error-driven stop (denoising runs, Sec. IV): no further atom once ||r||^2 <= err2
      if (a.err2 > 0.0 && !(renergy > (T)a.err2)) {
        early = true;
        break;
      }
      // largest |corr| over the unselected atoms; ties to the smaller atom index.  A lane
      // scans its atoms in increasing index order (cj, then ri), so a strict comparison
      // keeps the first of equal values.
      T bv = T(-1), bs = 0;
      int ba = INT_MAX;
      if (act) {
        const int base = sr + N1 * sc;
#pragma unroll
        for (int cj = 0; cj < NCJ; ++cj)
#pragma unroll
          for (int ri = 0; ri < NRI; ++ri) {
            const int e = ri * NCJ + cj;
            const T v = fabs(corr[e]);
            const bool take = !((used >> e) & 1ull) && v > bv;
            bv = take ? v : bv;
            bs = take ? corr[e] : bs;
            ba = take ? base + LR * ri + N1 * C::LC * cj : ba;
          }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const T ov = __shfl_xor(bv, o, kWave), os = __shfl_xor(bs, o, kWave);
        const int oa = __shfl_xor(ba, o, kWave);
        const bool take = ov > bv || (ov == bv && oa < ba);
        bv = take ? ov : bv;
        bs = take ? os : bs;
        ba = take ? oa : ba;
      }
      if (ba == INT_MAX || !(bv > stop_thr)) {
        early = true;
        break;
      }
      const int ia = ba % N1, ja = ba / N1;
      T cst = 0;
      if (!append_atom<T, C>(t, lane, ia, ja, bs, g1, g2, Li, gam, supi, supj, xg, xw, my_x, my_i, my_j, a, cst)) {
        early = true;
        break;
      }
      renergy -= cst * bs;
      if (act && sr == ia % LR && sc == ja % C::LC) used |= 1ull << ((ia / LR) * NCJ + ja / C::LC);
      if (t + 1 < S && act) {
        // corr <- corr - cst (G_{:,a} - G_{:,S} v): terms gamma_q G1[:, i_q] G2[j_q, :],
        // four at a time (terms beyond t have gamma = 0 and atom 0)
#pragma unroll 1
        for (int q0 = 0; q0 <= t; q0 += 4) {
          T gq[4];
          int iq[4], jq[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            gq[u] = gam[q0 + u];
            iq[u] = (int)supi[q0 + u];
            jq[u] = (int)supj[q0 + u];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const T* p1 = sG1P + iq[u] * N1 + sr * NRI;
            const T* p2 = sG2P + jq[u] * N2 + sc * NCJ;
            T u1[NRI];
#pragma unroll
            for (int ri = 0; ri < NRI; ++ri) u1[ri] = gq[u] * p1[ri];
#pragma unroll
            for (int cj = 0; cj < NCJ; ++cj) {
              const T u2 = p2[cj];
#pragma unroll
              for (int ri = 0; ri < NRI; ++ri) corr[ri * NCJ + cj] += u1[ri] * u2;
            }
          }
        }
      }
    }
    // explicit residual Y - sum_q x_q d1_{i_q} d2_{j_q}^T, the support read back from LDS
    // (coefficients staged in the exchange vector, atoms in supi / supj)
    wave_sync();
    if (lane < t) xg[lane] = my_x;
    wave_sync();
    T rr = 0;
    for (int e = lane; e < M; e += kWave) {
      const int p = e % M1, q = e / M1;
      T r = ys[e];
      for (int u = 0; u < t; ++u) r -= xg[u] * sD1[p + M1 * (int)supi[u]] * sD2[q + M2 * (int)supj[u]];
      rr += r * r;
    }
    rr = wave_sum(rr);
    if (lane < S) {
      a.supp[k * S + lane] = lane < t ? my_i + N1 * my_j : -1;
      a.coef[k * S + lane] = lane < t ? my_x : T(0);
    }
    if (lane == 0) {
      if (a.res2) a.res2[k] = rr;
      n_early += early ? 1u : 0u;
    }
    wave_sync();
  }
  // one atomic per workgroup: atomics on one address from every wave serialise
  __shared__ unsigned sEarly[C::WPB];
  if (lane == 0) sEarly[wv] = n_early;
  __syncthreads();
  if (tid == 0) {
    unsigned tot = 0;
    for (int w = 0; w < C::WPB; ++w) tot += sEarly[w];
    if (tot) atomicAdd(&a.counters[kCtrEarlyStop], (unsigned long long)tot);
  }
}

// Largest (key, atom) pair of the wave, ties to the smaller atom; the result is uniform.
// Keys are magnitudes as bit patterns (non-negative floats order like unsigned integers).
// Within each row of 16 lanes: DPP quad swaps, half-row mirror and row mirror leave every
// lane with its row's best; two DPP row broadcasts then merge the rows into lane 63.
template <int CTRL>
__device__ inline void argmax_dpp_stage(unsigned& key, int& atom) {
  const unsigned ok = (unsigned)__builtin_amdgcn_update_dpp(0, (int)key, CTRL, 0xF, 0xF, false);
  const int oa = __builtin_amdgcn_update_dpp(0, atom, CTRL, 0xF, 0xF, false);
  const bool take = ok > key || (ok == key && oa < atom);
  key = take ? ok : key;
  atom = take ? oa : atom;
}

// the same merge from a DPP row broadcast, in the rows of ROWS only (other rows keep theirs)
template <int CTRL, int ROWS>
__device__ inline void argmax_bcast_stage(unsigned& key, int& atom) {
  const unsigned ok = (unsigned)__builtin_amdgcn_update_dpp((int)key, (int)key, CTRL, ROWS, 0xF, false);
  const int oa = __builtin_amdgcn_update_dpp(atom, atom, CTRL, ROWS, 0xF, false);
  const bool take = ok > key || (ok == key && oa < atom);
  key = take ? ok : key;
  atom = take ? oa : atom;
}

__device__ inline void wave_argmax_key(unsigned& key, int& atom) {
  argmax_dpp_stage<0xB1>(key, atom);   // quad_perm [1,0,3,2]
  argmax_dpp_stage<0x4E>(key, atom);   // quad_perm [2,3,0,1]
  argmax_dpp_stage<0x141>(key, atom);  // row_half_mirror
  argmax_dpp_stage<0x140>(key, atom);  // row_mirror
  // every lane now holds its row's best: rows 1 and 3 take in lane 15 / 47 (row_bcast:15), then
  // rows 2 and 3 take in lane 31 (row_bcast:31), so lane 63 holds the wave's best
  argmax_bcast_stage<0x142, 0xA>(key, atom);
  argmax_bcast_stage<0x143, 0xC>(key, atom);
  key = (unsigned)__builtin_amdgcn_readlane((int)key, 63);
  atom = __builtin_amdgcn_readlane(atom, 63);
}

// FP32 variant on the matrix cores.  The n1 x n2 correlations (padded to multiples of 16)
// live in 16x16 tiles in the output layout of the 16x16x4 FP32 MFMA: register v of tile
// (ti, tj) in lane l is C[16 ti + 4 (l / 16) + v, 16 tj + l % 16].  Four refresh terms are
// one MFMA per tile: lane l supplies gamma_q G1[16 ti + l % 16, i_q] and G2[j_q, 16 tj + l % 16]
// for q = q0 + l / 16, i.e. one LDS read per tile row and per tile column for four terms.
// The first correlation runs the same way in two products, W = D1^T Y (k = m1) and
// C = W D2 (k = m2).  Padding rows and columns are zero and never selected.
// L^{-1} is kept twice, by rows and by columns, in float4 chunks (16-byte aligned, zero
// outside the lower triangle of the rows written so far), so w = L^{-1} g, |w|^2 and
// v = L^{-T} w are float4 loops whose loads all issue at once.  For long supports
// (s >= 24, the error-driven caps) both copies are packed: row k holds its entries
// l < 4 (k/4 + 1), column l its entries k >= 4 (l/4), about half the LDS of square
// storage (at s = 32 a wave's buffer drops from 10.5 KB to 5.9 KB, and LDS no longer
// caps the waves per CU below the register limit: 6 instead of 3 per SIMD).  Shorter
// supports keep square copies: there the packed form saves no waves and its per-lane
// chunk bounds cost registers.
template <class C>
struct MLay {
  static constexpr int TR = (C::N1 + 15) / 16, TC = (C::N2 + 15) / 16, TQ = (C::M2 + 15) / 16;
  static constexpr int P1 = 16 * TR, P2 = 16 * TC;
  static constexpr int YQ = 16 * TQ + 1;  // Y^T staging stride (odd: conflict-free writes)
  static constexpr int P1W = P1 + 1;      // W staging stride (odd: conflict-free writes)
  static constexpr int SP = C::SP;        // multiple of 4
  static constexpr int YT = (YQ * C::M1 + 3) / 4 * 4;
  static constexpr int WSM = P1W * C::M2;
  static constexpr int C4 = (C::S + 3) / 4;        // float4 chunks of a full row of L^{-1}
  static constexpr bool PK = C::S >= 24;             // packed copies of L^{-1}
  // waves per SIMD the registers must allow: with packed copies LDS allows 6, and the
  // compiler's own choice lands one register above that (12 bytes per lane spill instead)
  static constexpr int MINW = PK ? 6 : 1;
  static constexpr int LPK = PK ? 8 * C4 * (C4 + 1) : C::S * SP;  // one copy (rows or columns)
  static constexpr int SCR = 2 * LPK + 5 * SP;       // L^{-1} by rows and by columns, gam, supi, supj, g, w
  static constexpr int UNI = ((WSM > SCR ? WSM : SCR) + 3) / 4 * 4;  // W staging aliases the scratch
  static constexpr int PW = YT + UNI;
  static_assert(C::M1 % 4 == 0 && C::M2 % 4 == 0, "m1 and m2 are the k of the first-correlation MFMAs");
  static_assert(TR * TC * 4 <= 64, "one mask bit per register element");
};

// append_atom for the square, zero-padded L^{-1} storage of the matrix-core kernel (same
// arithmetic, same return and same visibility guarantee).
// Offsets of the rows and columns of L^{-1}.  Packed (C4 chunks of four in a full row):
// row k = 4c + r starts at 4 (c + 1)(2c + r), column l = 4c + r at
// 16 (c C4 - c (c - 1) / 2) + 4 r (C4 - c) and holds entries k = 4c, 4c + 1, ...
// Square: row k at k SP, column l at l SP, holding entries k = 0, 1, ...
template <class Lay>
__device__ inline int lrow(int k) {
  if constexpr (!Lay::PK) return k * Lay::SP;
  const int c = k >> 2, r = k & 3;
  return 4 * (c + 1) * (2 * c + r);
}
template <class Lay>
__device__ inline int lcol(int l) {
  if constexpr (!Lay::PK) return l * Lay::SP;
  constexpr int C4 = Lay::C4;
  const int c = l >> 2, r = l & 3;
  return 16 * (c * C4 - c * (c - 1) / 2) + 4 * r * (C4 - c);
}
// first entry index held by column l
template <class Lay>
__device__ inline int lcol0(int l) {
  return Lay::PK ? 4 * (l >> 2) : 0;
}

template <class C, class G1f, class G2f>
__device__ inline bool append_atom_sq(int t, int lane, int ia, int ja, float bs, G1f g1, G2f g2, float* LiR,
                                      float* LiT, float* gam, float* supi, float* supj, float* xg, float* xw,
                                      float& my_x, int& my_i, int& my_j, const OmpArgs<float>& a,
                                      float& cst_out) {
  using L = MLay<C>;
  constexpr int S = C::S, NC = L::C4;
  constexpr bool PK = L::PK;
  // chunks of four past the support (index t and beyond) hold zeros: skip them
  const int nc = (t + 4) / 4;
  const float gaa = g1(ia, ia) * g2(ja, ja);
  if (lane < t) xg[lane] = g1(my_i, ia) * g2(ja, my_j);
  wave_sync();
  // w = L^{-1} g in lane k < t (row k: its chunks c <= k/4; entries past the diagonal
  // and rows not yet written are zero, as are g and w past t)
  const int rw = lane < S ? lane : S - 1;
  const int cl = rw >> 2;  // packed: last chunk of row rw, first chunk of column rw
  const float4* row = reinterpret_cast<const float4*>(LiR + lrow<L>(rw));
  const float4* g4 = reinterpret_cast<const float4*>(xg);
  float p0 = 0.f, p1 = 0.f;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (c >= nc) break;
    // past its last chunk a row's storage holds the next rows: this lane stops there
    if (PK && c > cl) break;
    const float4 r = row[c], gg = g4[c];
    p0 += r.x * gg.x;
    p1 += r.y * gg.y;
    p0 += r.z * gg.z;
    p1 += r.w * gg.w;
  }
  if (lane < t) xw[lane] = p0 + p1;
  wave_sync();
  // |w|^2 in every lane, v = L^{-T} w in lane l < t (column l of L^{-1})
  const float4* w4 = reinterpret_cast<const float4*>(xw);
  // (packed, column rw holds chunks cl, cl + 1, ...: before cl its entries are zero)
  const float4* col = reinterpret_cast<const float4*>(LiT + lcol<L>(rw) - lcol0<L>(rw));
  float q0 = 0.f, q1 = 0.f, v0 = 0.f, v1 = 0.f;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (c >= nc) break;
    const float4 w = w4[c];
    q0 += w.x * w.x;
    q1 += w.y * w.y;
    q0 += w.z * w.z;
    q1 += w.w * w.w;
    if (!PK || c >= cl) {  // before its first chunk a column's entries are zero
      const float4 cc = col[c];
      v0 += cc.x * w.x;
      v1 += cc.y * w.y;
      v0 += cc.z * w.z;
      v1 += cc.w * w.w;
    }
  }
  float v = v0 + v1;
  float d2 = gaa - (q0 + q1);
  if (d2 < (float)a.pivot_fp64 * gaa) {
    // small pivot: w and |w|^2 again in FP64 (cancellation in G_aa - |w|^2)
    double w64 = 0.0;
    if (lane < t)
      for (int l = 0; l <= lane; ++l)
        w64 += (double)LiR[lrow<L>(lane) + l] * ((double)g1((int)supi[l], ia) * (double)g2(ja, (int)supj[l]));
    const double ww64 = wave_sum(lane < t ? w64 * w64 : 0.0);
    wave_sync();
    if (lane < t) xw[lane] = (float)w64;
    wave_sync();
    v0 = 0.f;
    v1 = 0.f;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (c >= nc) break;
      if (!PK || c >= cl) {
        const float4 w = w4[c], cc = col[c];
        v0 += cc.x * w.x;
        v1 += cc.y * w.y;
        v0 += cc.z * w.z;
        v1 += cc.w * w.w;
      }
    }
    v = v0 + v1;
    d2 = (float)((double)gaa - ww64);
    if (lane == 0) atomicAdd(&a.counters[kCtrFp64Pivot], 1ull);
  }
  if (!(d2 > (float)a.dep_eps * gaa)) return false;
  const float cst = bs / d2;
  cst_out = cst;
  const float dinv = 1.f / sqrtf(d2);
  if (lane < t) {
    LiR[lrow<L>(t) + lane] = -v * dinv;
    LiT[lcol<L>(lane) + t - lcol0<L>(lane)] = -v * dinv;
    my_x -= cst * v;
    gam[lane] = cst * v;
  }
  if (lane == t) {
    LiR[lrow<L>(t) + t] = dinv;
    LiT[lcol<L>(t) + t - lcol0<L>(t)] = dinv;
    my_x = cst;
    my_i = ia;
    my_j = ja;
    gam[t] = -cst;
    supi[t] = (float)ia;
    supj[t] = (float)ja;
  }
  wave_sync();
  return true;
}

template <class C>
__global__ void __launch_bounds__(kWave* C::WPB) __attribute__((amdgpu_waves_per_eu(MLay<C>::MINW)))
    omp_wave_mfma_kernel(OmpArgs<float> a) {
  using L = MLay<C>;
  constexpr int M1 = C::M1, M2 = C::M2, N1 = C::N1, N2 = C::N2, S = C::S, M = C::M, SP = C::SP;
  constexpr int TR = L::TR, TC = L::TC, TQ = L::TQ, P1 = L::P1, P2 = L::P2, YQ = L::YQ, P1W = L::P1W;
  __shared__ __align__(16) float sD1T[P1 * M1];  // D1[p, i] at i + P1 p, zero for i >= n1
  __shared__ __align__(16) float sD2T[P2 * M2];  // D2[q, j] at j + P2 q, zero for j >= n2
  __shared__ __align__(16) float sG1P[P1 * N1];  // G1[i, ik] at i + P1 ik, zero for i >= n1
  __shared__ __align__(16) float sG2P[P2 * N2];  // G2[jk, j] at j + P2 jk, zero for j >= n2
  __shared__ __align__(16) float sW[C::WPB][L::PW];

  const int tid = threadIdx.x, wv = tid / kWave, lane = tid % kWave;
  const int r16 = lane % 16, k4 = lane / 16;
  for (int e = tid; e < P1 * M1; e += blockDim.x) {
    const int i = e % P1, p = e / P1;
    sD1T[e] = i < N1 ? a.D1[p + M1 * i] : 0.f;
  }
  for (int e = tid; e < P2 * M2; e += blockDim.x) {
    const int j = e % P2, q = e / P2;
    sD2T[e] = j < N2 ? a.D2[q + M2 * j] : 0.f;
  }
  for (int e = tid; e < P1 * N1; e += blockDim.x) {
    const int i = e % P1, ik = e / P1;
    sG1P[e] = i < N1 ? a.G1[i + N1 * ik] : 0.f;
  }
  for (int e = tid; e < P2 * N2; e += blockDim.x) {
    const int j = e % P2, jk = e / P2;
    sG2P[e] = j < N2 ? a.G2[jk + N2 * j] : 0.f;
  }
  float* ysT = sW[wv];          // Y[p, q] at q + YQ p; columns m2 .. 16 TQ - 1 stay zero
  float* Ws = ysT + L::YT;      // W[i, q] at i + P1W q (first correlation only)
  float* LiR = Ws;              // L^{-1}[k, l] at lrow(k) + l (greedy loop; aliases W)
  float* LiT = LiR + L::LPK;    // L^{-1}[k, l] at lcol(l) + k - 4 (l / 4)
  float* gam = LiT + L::LPK;    // refresh coefficients gamma_q (zero beyond the support)
  float* supi = gam + SP;       // support atoms i_q, j_q (exact small integers)
  float* supj = supi + SP;
  float* xg = supj + SP;        // exchange vectors: Gram column g, then w
  float* xw = xg + SP;
  if constexpr (16 * TQ > M2) {
    for (int e = lane; e < (16 * TQ - M2) * M1; e += kWave) {
      const int q = M2 + e % (16 * TQ - M2), p = e / (16 * TQ - M2);
      ysT[q + YQ * p] = 0.f;
    }
  }
  __syncthreads();
  // G1 and G2 are symmetric: G1[i, ik] and G2[jk, j] from the padded tables
  auto g1 = [&](int i, int ik) { return sG1P[i + P1 * ik]; };
  auto g2 = [&](int jk, int j) { return sG2P[j + P2 * jk]; };
  // register elements outside the n1 x n2 block stay exactly zero (zero rows and columns
  // in every table), so they are never selected

  unsigned n_early = 0;  // early-stopped signals of this wave (lane 0), counted once at the end
  for (int64_t k = (int64_t)blockIdx.x * C::WPB + wv; k < a.N; k += (int64_t)gridDim.x * C::WPB) {
    float yy = 0.f;
    for (int e = lane; e < M; e += kWave) {
      const float v = a.Yh ? bf16_to_float(a.Yh[k * M + e]) : a.Y[k * M + e];
      ysT[e / M1 + YQ * (e % M1)] = v;
      yy += v * v;
    }
    const float yy_all = wave_sum(yy);
    const float ynorm = sqrtf(yy_all);
    float renergy = yy_all;  // ||r||^2 by the OMP recurrence (error-driven stop)
    wave_sync();
    {
      // W = D1^T Y, rows padded with zeros to P1
      f32x4 wt[TR][TQ];
#pragma unroll
      for (int ti = 0; ti < TR; ++ti)
#pragma unroll
        for (int tq = 0; tq < TQ; ++tq) wt[ti][tq] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
      for (int p0 = 0; p0 < M1; p0 += 4) {
        const int p = p0 + k4;
        float av[TR], bv[TQ];
#pragma unroll
        for (int ti = 0; ti < TR; ++ti) av[ti] = sD1T[16 * ti + r16 + P1 * p];
#pragma unroll
        for (int tq = 0; tq < TQ; ++tq) bv[tq] = ysT[16 * tq + r16 + YQ * p];
#pragma unroll
        for (int ti = 0; ti < TR; ++ti)
#pragma unroll
          for (int tq = 0; tq < TQ; ++tq)
            wt[ti][tq] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ti], bv[tq], wt[ti][tq], 0, 0, 0);
      }
#pragma unroll
      for (int ti = 0; ti < TR; ++ti)
#pragma unroll
        for (int tq = 0; tq < TQ; ++tq) {
          const int q = 16 * tq + r16;
          if (q < M2) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const float wvv = wt[ti][tq][v];  // by value
              Ws[16 * ti + 4 * k4 + v + P1W * q] = wvv;
            }
          }
        }
    }
    wave_sync();
    f32x4 acc[TR][TC];
#pragma unroll
    for (int ti = 0; ti < TR; ++ti)
#pragma unroll
      for (int tj = 0; tj < TC; ++tj) acc[ti][tj] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int q0 = 0; q0 < M2; q0 += 4) {
      const int q = q0 + k4;
      float av[TR], bv[TC];
#pragma unroll
      for (int ti = 0; ti < TR; ++ti) av[ti] = Ws[16 * ti + r16 + P1W * q];
#pragma unroll
      for (int tj = 0; tj < TC; ++tj) bv[tj] = sD2T[16 * tj + r16 + P2 * q];
#pragma unroll
      for (int ti = 0; ti < TR; ++ti)
#pragma unroll
        for (int tj = 0; tj < TC; ++tj) acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ti], bv[tj], acc[ti][tj], 0, 0, 0);
    }
    wave_sync();  // W is read: the scratch it aliases is cleared next
    for (int e = lane; e < L::SCR; e += kWave) LiR[e] = 0.f;
    wave_sync();

    float my_x = 0.f;
    int my_i = 0, my_j = 0;
    int t = 0;
    bool early = false;
    const float stop_thr = (float)a.stop_rel * ynorm;
#pragma unroll 1
    for (; t < S; ++t) {
      if (a.err2 > 0.0 && !(renergy > (float)a.err2)) {
        early = true;
        break;
      }
      // largest |corr| over the unselected atoms, ties to the smaller atom index; a lane's
      // atoms in (tj, ti, v) order have increasing indices, so a strict comparison keeps
      // the first of equal values.  Elements are read by value.
      unsigned bk = 0u;
      float bs = 0.f;
      int ba = INT_MAX;
#pragma unroll
      for (int tj = 0; tj < TC; ++tj)
#pragma unroll
        for (int ti = 0; ti < TR; ++ti)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float cv = acc[ti][tj][v];
            const unsigned kv = __float_as_uint(cv) & 0x7FFFFFFFu;  // |cv|
            const bool take = kv > bk;
            bk = take ? kv : bk;
            bs = take ? cv : bs;
            ba = take ? (16 * ti + 4 * k4 + v) + N1 * (16 * tj + r16) : ba;
          }
      wave_argmax_key(bk, ba);
      if (ba == INT_MAX || !(__uint_as_float(bk) > stop_thr)) {
        early = true;
        break;
      }
      const int ia = ba % N1, ja = ba / N1;
      // no explicit masking: a chosen atom's correlation is zero up to rounding after the
      // re-fit, so picking it again means every correlation is at rounding level: stop
      if (__ballot(lane < t && my_i == ia && my_j == ja) != 0ull) {
        early = true;
        break;
      }
      // the signed correlation from the lane that holds the atom
      bs = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, bs), 16 * ((ia % 16) / 4) + ja % 16));
      float cst = 0.f;
      if (!append_atom_sq<C>(t, lane, ia, ja, bs, g1, g2, LiR, LiT, gam, supi, supj, xg, xw, my_x, my_i, my_j, a,
                             cst)) {
        early = true;
        break;
      }
      renergy -= cst * bs;
      if (t + 1 < S) {
        // corr <- corr - cst (G_{:,a} - G_{:,S} v), four terms gamma_q G1[:, i_q] G2[j_q, :]
        // per MFMA (terms beyond t have gamma = 0 and atom 0)
#pragma unroll 1
        for (int q0 = 0; q0 <= t; q0 += 4) {
          const int q = q0 + k4;
          const float gq = gam[q];
          const int iq = (int)supi[q], jq = (int)supj[q];
          float av[TR], bv2[TC];
#pragma unroll
          for (int ti = 0; ti < TR; ++ti) av[ti] = gq * sG1P[16 * ti + r16 + P1 * iq];
#pragma unroll
          for (int tj = 0; tj < TC; ++tj) bv2[tj] = sG2P[16 * tj + r16 + P2 * jq];
#pragma unroll
          for (int ti = 0; ti < TR; ++ti)
#pragma unroll
            for (int tj = 0; tj < TC; ++tj)
              acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ti], bv2[tj], acc[ti][tj], 0, 0, 0);
        }
      }
    }
    // explicit residual Y - D1_S diag(x) D2_S^T on the matrix cores: four support terms per
    // 16x16x4 MFMA (terms beyond t have x = 0; support atoms beyond t are atom 0)
    wave_sync();
    if (lane < SP) xg[lane] = lane < t ? my_x : 0.f;
    wave_sync();
    constexpr int RP = (M1 + 15) / 16;
    f32x4 dx[RP][TQ];
#pragma unroll
    for (int tp = 0; tp < RP; ++tp)
#pragma unroll
      for (int tq = 0; tq < TQ; ++tq) dx[tp][tq] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int u0 = 0; u0 < t; u0 += 4) {
      const int u = u0 + k4;
      const float xu = xg[u];
      const int iu = (int)supi[u], ju = (int)supj[u];
      float av[RP], bv[TQ];
#pragma unroll
      for (int tp = 0; tp < RP; ++tp) {
        const int p = 16 * tp + r16;
        av[tp] = p < M1 ? xu * sD1T[iu + P1 * p] : 0.f;
      }
#pragma unroll
      for (int tq = 0; tq < TQ; ++tq) {
        const int q = 16 * tq + r16;
        bv[tq] = q < M2 ? sD2T[ju + P2 * q] : 0.f;
      }
#pragma unroll
      for (int tp = 0; tp < RP; ++tp)
#pragma unroll
        for (int tq = 0; tq < TQ; ++tq)
          dx[tp][tq] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[tp], bv[tq], dx[tp][tq], 0, 0, 0);
    }
    float rr = 0.f;
#pragma unroll
    for (int tp = 0; tp < RP; ++tp)
#pragma unroll
      for (int tq = 0; tq < TQ; ++tq)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int p = 16 * tp + 4 * k4 + v, q = 16 * tq + r16;
          if (p < M1 && q < M2) {
            const float r = ysT[q + YQ * p] - dx[tp][tq][v];
            rr += r * r;
          }
        }
    rr = wave_sum(rr);
    if (lane < S) {
      a.supp[k * S + lane] = lane < t ? my_i + N1 * my_j : -1;
      a.coef[k * S + lane] = lane < t ? my_x : 0.f;
    }
    if (lane == 0) {
      if (a.res2) a.res2[k] = rr;
      n_early += early ? 1u : 0u;
    }
    wave_sync();
  }
  // one atomic per workgroup: atomics on one address from every wave serialise
  __shared__ unsigned sEarly[C::WPB];
  if (lane == 0) sEarly[wv] = n_early;
  __syncthreads();
  if (tid == 0) {
    unsigned tot = 0;
    for (int w = 0; w < C::WPB; ++w) tot += sEarly[w];
    if (tot) atomicAdd(&a.counters[kCtrEarlyStop], (unsigned long long)tot);
  }
}

// One signal per wave up to kWaveMaxBlocks workgroups (a persistent grid measured slower:
// static striding leaves waves idle at the end).
template <typename T, class C>
hipError_t launch_wcfg(const OmpArgs<T>& a, hipStream_t st) {
  int64_t blocks = (a.N + C::WPB - 1) / C::WPB;
  if (blocks > kWaveMaxBlocks) blocks = kWaveMaxBlocks;
  if constexpr (sizeof(T) == 4 && C::MF)
    hipLaunchKernelGGL((omp_wave_mfma_kernel<C>), dim3((unsigned)blocks), dim3(kWave * C::WPB), 0, st, a);
  else
    hipLaunchKernelGGL((omp_wave_kernel<T, C>), dim3((unsigned)blocks), dim3(kWave * C::WPB), 0, st, a);
  return hipGetLastError();
}

struct WaveVariant {
  int m1, m2, n1, n2, s, lr, lc;
  hipError_t (*f32)(const OmpArgs<float>&, hipStream_t);
  hipError_t (*f64)(const OmpArgs<double>&, hipStream_t);
};

// Shapes with a one-wave-per-signal register kernel:
// (m1, m2, n1, n2, s, lane grid LR x LC, waves per workgroup, FP32 on the matrix cores)
// The s = 32 entries are the error-driven denoising shapes (8 x 8 patches, cap m1 m2 / 2).
#define SDL_WAVE_SHAPES(X)                                                                       \
  X(12, 12, 20, 20, 10, 4, 10, 4, true) X(12, 12, 24, 24, 12, 8, 8, 4, true)                    \
  X(16, 16, 32, 32, 16, 8, 8, 4, true) X(32, 24, 48, 36, 20, 16, 4, 4, true)                    \
  X(8, 8, 16, 16, 32, 8, 8, 4, true) X(8, 8, 8, 8, 32, 8, 8, 4, true)

const WaveVariant kWaveVariants[] = {
#define X(A_, B_, C_, D_, E_, F_, G_, H_, I_)                       \
  {A_, B_, C_, D_, E_, F_, G_, &launch_wcfg<float, WCfg<A_, B_, C_, D_, E_, F_, G_, H_, I_>>, \
   &launch_wcfg<double, WCfg<A_, B_, C_, D_, E_, F_, G_, H_, I_>>},
    SDL_WAVE_SHAPES(X)
#undef X
};

// FP32 one-wave shapes used only by the n-dimensional path, with every mode after the first
// collapsed into one Kronecker factor D_n (x) ... (x) D_2 (so m2 and n2 are products and may
// exceed the two-mode limits): (m1, m2, n1, n2, s, LR, LC, waves per workgroup).  Eight waves
// share the 34 KB of dictionary tables: 4 waves per SIMD (the register limit) instead of the
// 3 that LDS allows with four.
#define SDL_WAVE_COLLAPSED_SHAPES(X) X(8, 32, 12, 72, 8, 4, 8, 8)

const WaveVariant kWaveCollapsed[] = {
#define X(A_, B_, C_, D_, E_, F_, G_, H_) \
  {A_, B_, C_, D_, E_, F_, G_, &launch_wcfg<float, WCfg<A_, B_, C_, D_, E_, F_, G_, H_, true>>, nullptr},
    SDL_WAVE_COLLAPSED_SHAPES(X)
#undef X
};

const WaveVariant* find_wave(int m1, int m2, int n1, int n2, int s) {
  for (const WaveVariant& v : kWaveVariants)
    if (v.m1 == m1 && v.m2 == m2 && v.n1 == n1 && v.n2 == n2 && v.s == s) return &v;
  return nullptr;
}

}  // namespace

bool omp_wave_supported(int m1, int m2, int n1, int n2, int s) { return find_wave(m1, m2, n1, n2, s) != nullptr; }

bool omp_wave_grid(int m1, int m2, int n1, int n2, int s, int* lr, int* lc) {
  const WaveVariant* v = find_wave(m1, m2, n1, n2, s);
  if (!v) return false;
  *lr = v->lr;
  *lc = v->lc;
  return true;
}

bool omp_wave_collapsed_supported(int m1, int m2, int n1, int n2, int s) {
  for (const WaveVariant& v : kWaveCollapsed)
    if (v.m1 == m1 && v.m2 == m2 && v.n1 == n1 && v.n2 == n2 && v.s == s) return true;
  return false;
}

hipError_t launch_omp_wave_collapsed(const OmpArgs<float>& a, hipStream_t st) {
  for (const WaveVariant& v : kWaveCollapsed)
    if (v.m1 == a.m1 && v.m2 == a.m2 && v.n1 == a.n1 && v.n2 == a.n2 && v.s == a.s)
      return a.N == 0 ? hipSuccess : v.f32(a, st);
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_omp_wave(const OmpArgs<T>& a, hipStream_t st) {
  const WaveVariant* v = find_wave(a.m1, a.m2, a.n1, a.n2, a.s);
  if (!v || a.index || a.sums_side) return hipErrorInvalidValue;
  if (a.N == 0) return hipSuccess;
  if constexpr (sizeof(T) == 4) {
    // FP32 shapes with a quadrant kernel run four signals per wave (omp_quad.hip)
    if (omp_quad_supported(a.m1, a.m2, a.n1, a.n2, a.s)) return launch_omp_quad(a, st);
    return v->f32(a, st);
  } else {
    return v->f64(a, st);
  }
}

template hipError_t launch_omp_wave<float>(const OmpArgs<float>&, hipStream_t);
template hipError_t launch_omp_wave<double>(const OmpArgs<double>&, hipStream_t);

}  // namespace sdl
