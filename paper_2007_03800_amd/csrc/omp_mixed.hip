// SDL_MIXED_BF16 sparse coding: 2D-OMP (Sec. III step 1) in its direct form, where every
// greedy step recomputes the correlations of the current residual, D1^T R_k D2, here as two
// contractions on the BF16 matrix cores with FP32 accumulation.
//
// Mapping: a wave codes 16 signals, four lanes per signal: signal b of the wave is block b of
// the 4x4x4 16-block BF16 MFMA and of the 4x4x1 16-block FP32 MFMA, lane c (0..3) of the
// block is row c of an A operand, column c of a B operand and column c of a result tile.
//
//  * The residual is kept in FP32 registers as R^T (m2 x m1) in 4x4 tiles of the FP32 4x4x1
//    result layout: register v of tile (bq, bp) in lane c is R[4bp + c, 4bq + v].  Those four
//    registers, rounded to BF16, are exactly the A operand of V = R D2 for rows 4bp + c and
//    the K slice 4bq .. 4bq + 3; the residual update after each least-squares re-fit is a sum
//    of rank-one terms gamma_k d2_{j_k} d1_{i_k}^T, one FP32 4x4x1 MFMA per tile and term.
//  * V = R D2 (m1 x n2) comes out with register v of tile (bp, bj) in lane c equal to
//    V[4bp + v, 4bj + c]: four consecutive rows of one column, which rounded to BF16 is the B
//    operand of the second contraction D1^T V over the same rows.  The n1 x n2 correlations
//    are produced tile by tile and never stored: each tile's values feed packed keys
//    (|corr| with its low 8 bits replaced by the value's position in the lane) and each lane
//    keeps its two largest keys (max3 / med3).  Tile columns go in pairs: inside a pair the
//    positions are constants (6 bits), and the pair's code (2 bits) joins its two largest
//    keys before they meet the running ones, so a key costs one AND-OR.
//  * Near-ties: let M be the signal's largest BF16 |corr|.  Every kept key within tie_band of
//    M (at most two per lane, eight per signal) is re-scored exactly in FP32 as d1_i^T R d2_j
//    from the FP32 residual (the signal's four lanes each contribute their rows and add by
//    DPP), and the pick is the largest exact |corr| (ties: smaller atom).  A lane whose second
//    key is within the band may hold a third candidate that is not re-scored; such steps are
//    counted.  The winner's exact correlation drives the coefficient update, so the
//    coefficients do not see BF16 rounding.
//  * Cholesky factor, coefficient updates, small-pivot FP64 path, implicit masking and the
//    branch-free step (results committed with selects) as in omp_mfma.hip.
#include <limits.h>

#include <utility>

#include "sdl_internal.h"

namespace sdl {
namespace {

constexpr int kXWaves = 4;        // waves per workgroup
constexpr int kXMaxBlocks = 2048;
constexpr int kXLanes = 4;        // lanes per signal
constexpr int kXSigs = 16;        // signals per wave

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

template <int M1_, int M2_, int N1_, int N2_, int S_>
struct XCfg {
  static constexpr int M1 = M1_, M2 = M2_, N1 = N1_, N2 = N2_, S = S_;
  static constexpr int TP = M1 / 4, TQ = M2 / 4, TI = N1 / 4, TJ = N2 / 4;
  static constexpr int M = M1 * M2, NL = S * (S + 1) / 2;
  // odd LDS strides: the 16 signals of a wave fall into different banks
  // bfloat16 signals in LDS at a stride of M + 4 halves (8-byte aligned rows, and row starts spread
  // over the banks); odd strides for the dictionaries
  static constexpr int YH = M + 4, LD1 = M1 + 1, LD2 = M2 + 1, NLP = NL + 1;
  static_assert(M1 % 4 == 0 && M2 % 4 == 0 && N1 % 4 == 0 && N2 % 4 == 0, "4x4 tiles");
  static_assert(TI <= 8 && TJ <= 8, "key positions: 2 bits of tile-column pair, 6 bits inside the pair");
  static_assert(M % 4 == 0, "float4 staging");
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
__device__ inline float quad_sum(float v) {
  v += dppf<0xB1>(v);
  v += dppf<0x4E>(v);
  return v;
}

// two FP32 values rounded to BF16 (nearest even), the first in the low half
__device__ inline unsigned pack2(float a, float b) {
  const f32x2 v = {a, b};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
}
__device__ inline s16x4 pack4(const f32x4& v) {
  const u32x2 u = {pack2(v[0], v[1]), pack2(v[2], v[3])};
  return __builtin_bit_cast(s16x4, u);
}

constexpr int tri(int k, int l) { return k * (k + 1) / 2 + l; }

// middle of three (compiles to v_med3_u32)
__device__ inline unsigned umed3(unsigned a, unsigned b, unsigned c) { return max(min(a, b), min(max(a, b), c)); }

// atom of a packed key held by lane c of its signal.  Low 8 bits of a key: (3 - pair) << 6 |
// (63 - local), where the tile column bj = 2 pair + bl and local = (bl TI + bi) 4 + v, so larger
// low bits mean an earlier position (ties go to the smaller position).
template <class C>
__device__ inline int key_atom(unsigned key, int c) {
  const int pair = 3 - (int)((key >> 6) & 3u), local = 63 - (int)(key & 63u);
  const int bl = local / (4 * C::TI), rem = local % (4 * C::TI);
  const int v = rem & 3, bi = rem >> 2;
  const int bj = min(2 * pair + bl, C::TJ - 1);  // in range for any key
  return (4 * bi + v) + C::N1 * (4 * bj + c);
}

// (key, atom) of the quad's lanes merged: larger key, ties to the smaller atom
template <int CTRL>
__device__ inline void quad_argmax_stage(unsigned& key, int& atom) {
  const unsigned ok = (unsigned)dpp<CTRL>((int)key);
  const int oa = dpp<CTRL>(atom);
  const bool take = ok > key || (ok == key && oa < atom);
  key = take ? ok : key;
  atom = take ? oa : atom;
}

// Exact FP32 correlation of atom (i, j) with the signal's residual: this lane's rows
// p = 4bp + c of d1_i^T R d2_j, summed over the signal's four lanes.
template <class C>
__device__ inline float exact_corr(const f32x4 (&rt)[C::TQ][C::TP], const float* sD1, const f32x4* sD2c, int i, int j,
                                   int c) {
  f32x4 d2c[C::TQ];  // column j of D2, 16-byte loads
#pragma unroll
  for (int bq = 0; bq < C::TQ; ++bq) d2c[bq] = sD2c[j * C::TQ + bq];
  float part = 0.f;
#pragma unroll
  for (int bp = 0; bp < C::TP; ++bp) {
    float row = 0.f;
#pragma unroll
    for (int bq = 0; bq < C::TQ; ++bq)
#pragma unroll
      for (int v = 0; v < 4; ++v) row += rt[bq][bp][v] * d2c[bq][v];
    part += sD1[(4 * bp + c) + C::LD1 * i] * row;
  }
  return quad_sum(part);
}

// Everything one wave holds for its 16 signals while coding them (registers), plus the LDS
// rows of the Cholesky factor; lanes of a signal hold identical copies of the per-signal state.
template <class C>
struct Wave {
  f32x4 rt[C::TQ][C::TP];  // R^T tiles (see the file comment)
  float x[C::S];           // coefficients in selection order
  int at[C::S];            // atoms a = i + n1 j in selection order
  float* L;                // this signal's inverse Cholesky factor, rows with the diagonal (LDS)
  bool active;
  int nsel;
  float stop_thr;
  unsigned long long rescored, overflow;
};

// Greedy step T (compile-time, so the support state stays in registers).
template <class C, int T>
__device__ __forceinline__ void mixed_step(Wave<C>& w, const OmpArgs<float>& a, const float* sG1, const float* sG2,
                                           const float* sD1, const float* sD2, const f32x4* sD2c, const u32x2* sD1op,
                                           const u32x2* sD2op, int lane, int c, float keep, float dep_eps, float piv) {
  constexpr int N1 = C::N1, N2 = C::N2, S = C::S;
  constexpr int TP = C::TP, TQ = C::TQ, TI = C::TI, TJ = C::TJ;
  asm volatile("" ::: "memory");  // dictionary operands are read from LDS in each step, not held
  // ---- BF16 correlations D1^T (R D2), two largest packed keys per lane
  s16x4 rop[TP][TQ];
#pragma unroll
  for (int bp = 0; bp < TP; ++bp)
#pragma unroll
    for (int kq = 0; kq < TQ; ++kq) rop[bp][kq] = pack4(w.rt[kq][bp]);
  unsigned ka1 = 0u, ka2 = 0u, kb1 = 0u, kb2 = 0u;
  // tile columns in pairs: inside a pair the keys' positions are constants; each pair keeps its
  // own two largest keys per tracker and adds its pair code before they join the running ones
  for (int bj0 = 0; bj0 < TJ; bj0 += 2) {
    unsigned la1 = 0u, la2 = 0u, lb1 = 0u, lb2 = 0u;
#pragma unroll
    for (int bl = 0; bl < 2; ++bl) {
      const int bj = bj0 + bl;
      if (TJ % 2 == 0 || bj < TJ) {
        s16x4 vop[TP];
#pragma unroll
        for (int bp = 0; bp < TP; ++bp) {
          f32x4 vt = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kq = 0; kq < TQ; ++kq)
            vt = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(rop[bp][kq],
                                                        __builtin_bit_cast(s16x4, sD2op[(kq * TJ + bj) * 4 + c]), vt,
                                                        0, 0, 0);
          vop[bp] = pack4(vt);
        }
#pragma unroll
        for (int bi = 0; bi < TI; ++bi) {
          f32x4 al = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kp = 0; kp < TP; ++kp)
            al = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(__builtin_bit_cast(s16x4, sD1op[(kp * TI + bi) * 4 + c]),
                                                        vop[kp], al, 0, 0, 0);
          // keys: |corr| bits, low 6 bits = 63 - (position inside the pair)
          const unsigned e0 = (unsigned)((bl * TI + bi) * 4);
          const unsigned k0v = (__float_as_uint(al[0]) & 0x7FFFFF00u) | (63u - e0);
          const unsigned k1v = (__float_as_uint(al[1]) & 0x7FFFFF00u) | (62u - e0);
          const unsigned k2v = (__float_as_uint(al[2]) & 0x7FFFFF00u) | (61u - e0);
          const unsigned k3v = (__float_as_uint(al[3]) & 0x7FFFFF00u) | (60u - e0);
          // two largest of {la1, la2, k0v, k1v}: the second is max(la2, med3(la1, k0v, k1v))
          la2 = max(la2, umed3(la1, k0v, k1v));
          la1 = max(la1, max(k0v, k1v));
          lb2 = max(lb2, umed3(lb1, k2v, k3v));
          lb1 = max(lb1, max(k2v, k3v));
        }
      }
    }
    const unsigned code = (unsigned)(3 - bj0 / 2) << 6;
    la1 |= code;
    la2 |= code;
    lb1 |= code;
    lb2 |= code;
    // two largest of the running pair and the new pair (each sorted)
    ka2 = max(min(ka1, la1), max(ka2, la2));
    ka1 = max(ka1, la1);
    kb2 = max(min(kb1, lb1), max(kb2, lb2));
    kb1 = max(kb1, lb1);
  }
  const unsigned m1 = max(ka1, kb1), m2 = max(min(ka1, kb1), max(ka2, kb2));

  // ---- the signal's largest BF16 |corr| and the band of near-ties
  unsigned mkey = m1 & ~0xFFu;
  int matom = key_atom<C>(m1, c);
  quad_argmax_stage<0xB1>(mkey, matom);
  quad_argmax_stage<0x4E>(mkey, matom);
  const unsigned thr = __float_as_uint(__uint_as_float(mkey) * keep) & ~0xFFu;

  // ---- re-score the candidates within the band in FP32; the pick is the largest exact |corr|.
  // First the signal's BF16 maximum (its atom is known to the four lanes), then, while some
  // signal of the wave has candidates left, each signal's largest remaining one: the quad's
  // argmax over its lanes' remaining keys, whose owner lane then drops it.
  float best_cor = exact_corr<C>(w.rt, sD1, sD2c, matom % N1, matom / N1, c);
  float best_abs = fabsf(best_cor);
  int best_atom = matom, ncand = 1;
  best_abs = best_abs == best_abs ? best_abs : -1.f;  // NaN: no valid candidate
  unsigned c1 = ((m1 & ~0xFFu) >= thr && key_atom<C>(m1, c) != matom) ? m1 : 0u;
  unsigned c2 = (m2 & ~0xFFu) >= thr ? m2 : 0u;
  const bool overflow = c2 != 0u;  // a third candidate of this lane may exist
  while (__any((c1 | c2) != 0u)) {
    const unsigned ck = max(c1, c2);
    unsigned kq = ck;
    int aq = ck ? key_atom<C>(ck, c) : INT_MAX;
    quad_argmax_stage<0xB1>(kq, aq);
    quad_argmax_stage<0x4E>(kq, aq);
    if (ck && key_atom<C>(ck, c) == aq) {  // this lane owned it
      if (c1 == ck) c1 = 0u; else c2 = 0u;
    }
    const bool cand = kq != 0u;
    const int at = cand ? aq : matom;
    const float e = exact_corr<C>(w.rt, sD1, sD2c, at % N1, at / N1, c);
    const float ae = fabsf(e);
    const bool take = cand && (ae > best_abs || (ae == best_abs && at < best_atom));
    best_abs = take ? ae : best_abs;
    best_cor = take ? e : best_cor;
    best_atom = take ? at : best_atom;
    ncand += cand ? 1 : 0;
  }
  {
    // any lane of the signal whose second key lies in the band
    int ov = overflow ? 1 : 0;
    ov |= dpp<0xB1>(ov);
    ov |= dpp<0x4E>(ov);
    if (c == 0 && w.active) {
      w.rescored += ncand > 1 ? 1 : 0;
      w.overflow += ov ? 1 : 0;
    }
  }
  // a non-finite signal: best_abs < 0 stops it
  const int ba = best_atom;
  const int it = ba % N1, jt = ba / N1;
  const float cor = best_cor;
  bool stop = !(best_abs > w.stop_thr);
#pragma unroll
  for (int k = 0; k < T; ++k) stop = stop || (ba == w.at[k]);
  if (stop) w.active = false;

  // ---- least squares on the support with the inverse Cholesky factor Li = L^{-1} (rows in LDS, as
  // omp_quad.hip): with g = G_{S,a}, w = Li g and v = Li^T w are independent dot products,
  // delta^2 = G_aa - |w|^2, and the new row of Li is [-v^T, 1] / delta
  float* Li = w.L;
  float gv[S > 1 ? S - 1 : 1], wv[S > 1 ? S - 1 : 1];
#pragma unroll
  for (int k = 0; k < T; ++k) gv[k] = sG1[w.at[k] % N1 + N1 * it] * sG2[w.at[k] / N1 + N2 * jt];
  const float gaa = sG1[it + N1 * it] * sG2[jt + N2 * jt];
  float d2;
  {
    float ww = 0.f;
#pragma unroll
    for (int k = 0; k < T; ++k) {
      float b = 0.f;
#pragma unroll
      for (int l = 0; l <= k; ++l) b += Li[tri(k, l)] * gv[l];
      wv[k] = b;
      ww += b * b;
    }
    d2 = gaa - ww;
    if (w.active && d2 < piv * gaa) {
      // small pivot: w and |w|^2 again in FP64 (cancellation in G_aa - |w|^2)
      double accd = 0.0;
#pragma unroll
      for (int k = 0; k < T; ++k) {
        double b = 0.0;
#pragma unroll
        for (int l = 0; l <= k; ++l)
          b += (double)Li[tri(k, l)] *
               ((double)sG1[w.at[l] % N1 + N1 * it] * (double)sG2[w.at[l] / N1 + N2 * jt]);
        wv[k] = (float)b;
        accd += b * b;
      }
      d2 = (float)((double)gaa - accd);
      if (c == 0) atomicAdd(&a.counters[kCtrFp64Pivot], 1ull);
    }
    if (!(d2 > dep_eps * gaa)) w.active = false;
  }
  float vv[S > 1 ? S - 1 : 1];
#pragma unroll
  for (int l = 0; l < T; ++l) {
    float b = 0.f;
#pragma unroll
    for (int k = l; k < T; ++k) b += Li[tri(k, l)] * wv[k];
    vv[l] = b;
  }
  const float cst = cor / d2;
  const float dinv = rsqrtf(d2);
  // the signal's four lanes write the same row: no divergent store
#pragma unroll
  for (int k = 0; k < T; ++k) {
    Li[tri(T, k)] = -vv[k] * dinv;
    w.x[k] = w.active ? w.x[k] - cst * vv[k] : w.x[k];
  }
  Li[tri(T, T)] = dinv;
  w.x[T] = w.active ? cst : 0.f;
  w.at[T] = w.active ? ba : 0;
  w.nsel = w.active ? T + 1 : w.nsel;
  {
    // R -= sum_k dx_k d1_{i_k} d2_{j_k}^T with dx_T = cst, dx_k = -cst v_k, on R^T (FP32 4x4x1);
    // a stopped signal's residual stays as its committed coefficients left it
#pragma unroll
    for (int k = 0; k <= T; ++k) {
      const float gk = !w.active ? 0.f : k == T ? -cst : cst * vv[k < T ? k : 0];
      const int ak = k == T ? ba : w.at[k];
      const int ik = ak % N1, jk = ak / N1;
      float av[TQ], bv[TP];
#pragma unroll
      for (int bq = 0; bq < TQ; ++bq) av[bq] = gk * sD2[(4 * bq + c) + C::LD2 * jk];
#pragma unroll
      for (int bp = 0; bp < TP; ++bp) bv[bp] = sD1[(4 * bp + c) + C::LD1 * ik];
#pragma unroll
      for (int bq = 0; bq < TQ; ++bq)
#pragma unroll
        for (int bp = 0; bp < TP; ++bp)
          w.rt[bq][bp] = __builtin_amdgcn_mfma_f32_4x4x1f32(av[bq], bv[bp], w.rt[bq][bp], 0, 0, 0);
    }
  }
}

template <class C, int... T>
__device__ __forceinline__ void mixed_steps(std::integer_sequence<int, T...>, Wave<C>& w, const OmpArgs<float>& a,
                                            const float* sG1, const float* sG2, const float* sD1, const float* sD2,
                                            const f32x4* sD2c, const u32x2* sD1op, const u32x2* sD2op, int lane, int c,
                                            float keep, float dep_eps, float piv) {
  (mixed_step<C, T>(w, a, sG1, sG2, sD1, sD2, sD2c, sD1op, sD2op, lane, c, keep, dep_eps, piv), ...);
}

template <class C>
__global__ void __launch_bounds__(kWave* kXWaves) __attribute__((amdgpu_waves_per_eu(2, 2)))
    omp_mixed_kernel(OmpArgs<float> a) {
  constexpr int M1 = C::M1, N1 = C::N1, N2 = C::N2, S = C::S, M = C::M;
  constexpr int TP = C::TP, TQ = C::TQ, TI = C::TI, TJ = C::TJ;
  __shared__ float sG1[N1 * N1];
  __shared__ float sG2[N2 * N2];
  __shared__ float sD1[C::LD1 * N1];                  // D1[p, i] at p + LD1 i
  __shared__ float sD2[C::LD2 * C::N2];               // D2[q, j] at q + LD2 j
  __shared__ u32x2 sD1op[TP * TI * 4];                // [kp][bi][c] = D1[4kp + 0..3, 4bi + c] in BF16
  __shared__ u32x2 sD2op[TQ * TJ * 4];                // [kq][bj][c] = D2[4kq + 0..3, 4bj + c] in BF16
  __shared__ f32x4 sD2c[N2 * TQ];                     // D2 columns, 16-byte aligned: [j][bq] = D2[4bq + 0..3, j]
  __shared__ __align__(16) uint16_t sY[kXWaves][kXSigs * C::YH];  // the group's bfloat16 signals
  __shared__ float sL[kXWaves][kXSigs * C::NLP];

  const int tid = threadIdx.x, wv = tid / kWave, lane = tid % kWave;
  const int g = lane / kXLanes, c = lane % kXLanes;

  for (int e = tid; e < N1 * N1; e += blockDim.x) sG1[e] = a.G1[e];
  for (int e = tid; e < N2 * N2; e += blockDim.x) sG2[e] = a.G2[e];
  for (int e = tid; e < M1 * N1; e += blockDim.x) sD1[e % M1 + C::LD1 * (e / M1)] = a.D1[e];
  for (int e = tid; e < C::M2 * N2; e += blockDim.x) {
    sD2[e % C::M2 + C::LD2 * (e / C::M2)] = a.D2[e];
    reinterpret_cast<float*>(sD2c)[e] = a.D2[e];  // column-major m2 x n2, m2 a multiple of 4
  }
  for (int e = tid; e < TP * TI * 4; e += blockDim.x) {
    const int kp = e / (TI * 4), bi = (e / 4) % TI, cc = e % 4, col = 4 * bi + cc;
    const float* d = a.D1 + M1 * col + 4 * kp;
    sD1op[e] = u32x2{pack2(d[0], d[1]), pack2(d[2], d[3])};
  }
  for (int e = tid; e < TQ * TJ * 4; e += blockDim.x) {
    const int kq = e / (TJ * 4), bj = (e / 4) % TJ, cc = e % 4, col = 4 * bj + cc;
    const float* d = a.D2 + C::M2 * col + 4 * kq;
    sD2op[e] = u32x2{pack2(d[0], d[1]), pack2(d[2], d[3])};
  }
  __syncthreads();

  const float stop_rel = (float)a.stop_rel, dep_eps = (float)a.dep_eps, piv = (float)a.pivot_fp64;
  const float keep = 1.0f - (float)a.tie_band;
  const int64_t nsig = a.N;
  const int64_t ngroups = (nsig + kXSigs - 1) / kXSigs;
  uint16_t* ys = sY[wv];
  Wave<C> w;
  w.rescored = 0;
  w.overflow = 0;
  w.L = sL[wv] + g * C::NLP;

  unsigned n_early = 0;  // early-stopped signals seen by this lane, counted once at the end
  for (int64_t grp = (int64_t)blockIdx.x * kXWaves + wv; grp < ngroups; grp += (int64_t)gridDim.x * kXWaves) {
    const int64_t k0 = grp * kXSigs;
    const int nvalid = (int)((nsig - k0) < kXSigs ? (nsig - k0) : kXSigs);
    {
      // signal b of the group at ys + b * YH, four bfloat16 values (8 bytes) per load
      const int nchunk = nvalid * M / 4;
      for (int e = lane; e < kXSigs * M / 4; e += kWave) {
        const int b = e / (M / 4), off = e % (M / 4);
        const uint2 v = e < nchunk ? *reinterpret_cast<const uint2*>(a.Yh + (k0 + b) * M + 4 * off) : make_uint2(0u, 0u);
        *reinterpret_cast<uint2*>(ys + b * C::YH + 4 * off) = v;
      }
    }
    wave_sync();
    const uint16_t* y = ys + g * C::YH;
    const bool valid = g < nvalid;

    float yy = 0.f;
#pragma unroll
    for (int u = 0; u < M / kXLanes; ++u) {
      const float v = bf16_to_float(y[c * (M / kXLanes) + u]);
      yy += v * v;
    }
    const float ynorm = sqrtf(quad_sum(yy));

    // R^T = Y^T: register v of tile (bq, bp) is R[4bp + c, 4bq + v]
#pragma unroll
    for (int bq = 0; bq < TQ; ++bq)
#pragma unroll
      for (int bp = 0; bp < TP; ++bp)
#pragma unroll
        for (int v = 0; v < 4; ++v) w.rt[bq][bp][v] = bf16_to_float(y[(4 * bp + c) + M1 * (4 * bq + v)]);
#pragma unroll
    for (int k = 0; k < S; ++k) {
      w.x[k] = 0.f;
      w.at[k] = 0;
    }
    w.active = valid;
    w.nsel = 0;
    w.stop_thr = stop_rel * ynorm;
    mixed_steps<C>(std::make_integer_sequence<int, S>{}, w, a, sG1, sG2, sD1, sD2, sD2c, sD1op, sD2op, lane, c, keep,
                   dep_eps, piv);

    // ---- residual energy from the FP32 residual (updated after every committed step) and outputs
    float rr = 0.f;
#pragma unroll
    for (int bq = 0; bq < TQ; ++bq)
#pragma unroll
      for (int bp = 0; bp < TP; ++bp)
#pragma unroll
        for (int v = 0; v < 4; ++v) rr += w.rt[bq][bp][v] * w.rt[bq][bp][v];
    rr = quad_sum(rr);
    if (valid) {
      const int64_t k = k0 + g;
#pragma unroll
      for (int t = 0; t < S; ++t) {
        if (t % kXLanes == c) {
          a.supp[k * S + t] = t < w.nsel ? w.at[t] : -1;
          a.coef[k * S + t] = t < w.nsel ? w.x[t] : 0.f;
        }
      }
      if (c == 0) {
        if (a.res2) a.res2[k] = rr;
        n_early += w.nsel < S ? 1u : 0u;
      }
    }
    wave_sync();  // the next group's staging overwrites ys
  }
  if (n_early) atomicAdd(&a.counters[kCtrEarlyStop], (unsigned long long)n_early);
  // per-wave totals of the near-tie counters
  unsigned long long n_rescored = w.rescored, n_overflow = w.overflow;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    n_rescored += __shfl_xor(n_rescored, o, kWave);
    n_overflow += __shfl_xor(n_overflow, o, kWave);
  }
  if (lane == 0) {
    if (n_rescored) atomicAdd(&a.counters[kCtrRescored], n_rescored);
    if (n_overflow) atomicAdd(&a.counters[kCtrTieOverflow], n_overflow);
  }
}

template <class C>
hipError_t launch_xcfg(const OmpArgs<float>& a, hipStream_t st) {
  const int64_t ngroups = (a.N + kXSigs - 1) / kXSigs;
  int64_t blocks = (ngroups + kXWaves - 1) / kXWaves;
  if (blocks > kXMaxBlocks) blocks = kXMaxBlocks;
  hipLaunchKernelGGL(omp_mixed_kernel<C>, dim3((unsigned)blocks), dim3(kWave * kXWaves), 0, st, a);
  return hipGetLastError();
}

struct MixedVariant {
  int m1, m2, n1, n2, s;
  hipError_t (*f)(const OmpArgs<float>&, hipStream_t);
};

// Shapes with a mixed-precision kernel: (m1, m2, n1, n2, s)
#define SDL_MIXED_SHAPES(X) X(12, 12, 24, 24, 12) X(8, 8, 16, 16, 8) X(12, 12, 20, 20, 10)

const MixedVariant kMixedVariants[] = {
#define X(A_, B_, C_, D_, E_) {A_, B_, C_, D_, E_, &launch_xcfg<XCfg<A_, B_, C_, D_, E_>>},
    SDL_MIXED_SHAPES(X)
#undef X
};

const MixedVariant* find_mixed(int m1, int m2, int n1, int n2, int s) {
  for (const MixedVariant& v : kMixedVariants)
    if (v.m1 == m1 && v.m2 == m2 && v.n1 == n1 && v.n2 == n2 && v.s == s) return &v;
  return nullptr;
}

}  // namespace

bool omp_mixed_supported(int m1, int m2, int n1, int n2, int s) { return find_mixed(m1, m2, n1, n2, s) != nullptr; }

hipError_t launch_omp_mixed(const OmpArgs<float>& a, hipStream_t st) {
  const MixedVariant* v = find_mixed(a.m1, a.m2, a.n1, a.n2, a.s);
  if (!v || a.index || a.sums_side || !a.Yh) return hipErrorInvalidValue;
  if (a.N == 0) return hipSuccess;
  return v->f(a, st);
}

}  // namespace sdl
