// TMOD partial sums on the BF16 matrix cores (Algorithm 1 steps 1 and 3; the SDL_MIXED_BF16
// precision): the same sums as tmod_mfma.hip,
//
//   side 1 (Corollary 1):  T_k = X_k D2^T (n1 x m2),  A = sum T_k T_k^T,  B = sum Y_k T_k^T
//   side 2 (Result 1):     U_k = (D1 X_k)^T (n2 x m1), A = sum U_k U_k^T,  B = sum Y_k^T U_k^T
//
// with the batch factors Tcat = [T_1 .. T_bs] and Ycat = [Yt_1 .. Yt_bs] held in LDS as
// bfloat16, row-major by atom (resp. signal row) with the long inner index k contiguous, so one
// 8-byte read gives a lane its four consecutive k of a 16x16x16 BF16 MFMA operand (lane l: row
// l % 16, k = 4 (l / 16) + 0..3).  The signals are bfloat16 already (exact); each T_k entry is
// formed in FP32 (the codes of a row merged in selection order) and rounded once.  FP32
// accumulation on the matrix cores, then the same fixed-order FP64 reduction as the FP32 path
// (one partial row per workgroup), so the results are bitwise reproducible.
#include "sdl_internal.h"

namespace sdl {
namespace {

constexpr int kBWaves = 4;
constexpr int kBMaxBlocksPerCu = 8;
constexpr int kBMaxDynLds = 160 * 1024;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline uint16_t to_bf16(float v) {
  const f32x2 p = {v, 0.f};
  return (uint16_t)(__builtin_bit_cast(unsigned, __builtin_convertvector(p, bf16x2)) & 0xFFFFu);
}

// Batch layout of one wave in LDS (uint16 units): Tcat rows [16 TP][KP], Ycat rows [16 TR][KP],
// then the batch's codes (int32 atoms, float values).
struct BLayout {
  int K, KP, trows, yrows;
  size_t t_off, y_off, codes_bytes, wave_bytes;
};

__host__ __device__ inline BLayout blayout(int bs, int mc, int s, int tp, int tr) {
  BLayout L;
  L.K = bs * mc;
  // k padded to a multiple of 16 (the MFMA depth) plus 4 halves, so consecutive rows start in
  // different banks
  L.KP = ((L.K + 15) & ~15) + 4;
  L.trows = 16 * tp;
  L.yrows = 16 * tr;
  L.t_off = 0;
  L.y_off = (size_t)L.trows * L.KP;
  const size_t halves = (size_t)(L.trows + L.yrows) * L.KP;
  L.codes_bytes = (size_t)bs * s * 8;
  L.wave_bytes = ((halves * 2 + 15) & ~(size_t)15) + L.codes_bytes;
  return L;
}

template <int TP, int TR, int S>
__global__ void __launch_bounds__(kWave* kBWaves) tmod_sums_bf16_kernel(TmodArgs<float> a, double* part, int nblk,
                                                                         int bs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int side = a.side, n1 = a.n1;
  const int na = side == 1 ? a.n1 : a.n2;
  const int mr = side == 1 ? a.m1 : a.m2;
  const int mc = side == 1 ? a.m2 : a.m1;
  const int nbo = side == 1 ? a.n2 : a.n1;
  const int M = a.m1 * a.m2;
  const BLayout BL = blayout(bs, mc, S, TP, TR);
  const int KP = BL.KP, Kp16 = (BL.K + 15) & ~15;
  const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
  unsigned char* wbase = smem_raw + (size_t)w * BL.wave_bytes;
  uint16_t* Tb = reinterpret_cast<uint16_t*>(wbase) + BL.t_off;
  uint16_t* Yb = reinterpret_cast<uint16_t*>(wbase) + BL.y_off;
  int* cidx = reinterpret_cast<int*>(wbase + BL.wave_bytes - BL.codes_bytes);
  float* cval = reinterpret_cast<float*>(cidx + bs * S);
  float* Do = reinterpret_cast<float*>(smem_raw + (size_t)kBWaves * BL.wave_bytes);  // mc x nbo, FP32
  for (int e = tid; e < mc * nbo; e += blockDim.x) Do[e] = a.Dother[e];
  // padding rows of Ycat (mr .. 16 TR) stay zero for the whole kernel
  for (int e = lane; e < (BL.yrows - mr) * KP; e += kWave) Yb[mr * KP + e] = 0;
  __syncthreads();
  const int64_t k0 = (a.N * blockIdx.x) / nblk, k1 = (a.N * (blockIdx.x + 1)) / nblk;
  const int64_t nbatch = (k1 - k0 + bs - 1) / bs;

  f32x4 accP[TP][TP], accR[TR][TP];
#pragma unroll
  for (int i = 0; i < TP; ++i)
#pragma unroll
    for (int j = 0; j < TP; ++j) accP[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < TR; ++i)
#pragma unroll
    for (int j = 0; j < TP; ++j) accR[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int64_t bi = w; bi < nbatch; bi += kBWaves) {
    const int64_t kb = k0 + bi * bs;
    const int nb = (int)((k1 - kb) < bs ? (k1 - kb) : bs);
    // codes: atom a = i + n1 j split once per batch into this side's (row | other << 16), -1 unused
    for (int e = lane; e < nb * S; e += kWave) {
      const int at = a.supp[kb * S + e];
      const int i = at % n1, j = at / n1;
      cidx[e] = at < 0 ? -1 : (side == 1 ? (i | (j << 16)) : (j | (i << 16)));
      cval[e] = a.coef[kb * S + e];
    }
    // Tcat starts at zero (rows no code touches stay zero)
    for (int e = lane; e < BL.trows * KP / 4; e += kWave) reinterpret_cast<uint2*>(Tb)[e] = make_uint2(0u, 0u);
    wave_sync();
    // column k = b mc + c of Tcat and Ycat per lane: no cross-lane hazards
    for (int k = lane; k < Kp16; k += kWave) {
      const int b = k / mc, c = k % mc;
      if (b < nb) {
        float v[S];
        int ra[S];
#pragma unroll
        for (int t = 0; t < S; ++t) {
          const int pk = cidx[b * S + t];
          ra[t] = pk < 0 ? -1 : (pk & 0xFFFF);
          v[t] = pk < 0 ? 0.f : cval[b * S + t] * Do[c + mc * (pk < 0 ? 0 : (pk >> 16))];
        }
        // codes that share a row add up in selection order into the row's first code (later
        // ones of the row also collect partial sums, but only first occurrences are stored)
        unsigned long long seen = 0ull;
        bool first[S];
#pragma unroll
        for (int t = 0; t < S; ++t) {
          first[t] = ra[t] >= 0 && !((seen >> (ra[t] & 63)) & 1ull);
          seen |= ra[t] >= 0 ? (1ull << (ra[t] & 63)) : 0ull;
        }
#pragma unroll
        for (int t = 1; t < S; ++t)
#pragma unroll
          for (int u = 0; u < t; ++u) v[u] = ra[u] == ra[t] ? v[u] + v[t] : v[u];
#pragma unroll
        for (int t = 0; t < S; ++t)
          if (first[t]) Tb[ra[t] * KP + k] = to_bf16(v[t]);
        const int64_t yb = (kb + b) * M;
        for (int r = 0; r < mr; ++r)
          Yb[r * KP + k] = a.Yh[yb + (side == 1 ? r + a.m1 * c : c + a.m1 * r)];  // column / row c of Y_b
      } else {
        for (int r = 0; r < mr; ++r) Yb[r * KP + k] = 0;
      }
    }
    wave_sync();
    const int r16 = lane % 16, kq = lane / 16;
    for (int kk = 0; kk < Kp16; kk += 16) {
      s16x4 at[TP], ay[TR];
#pragma unroll
      for (int i = 0; i < TP; ++i) at[i] = *reinterpret_cast<const s16x4*>(Tb + (16 * i + r16) * KP + kk + 4 * kq);
#pragma unroll
      for (int i = 0; i < TR; ++i) ay[i] = *reinterpret_cast<const s16x4*>(Yb + (16 * i + r16) * KP + kk + 4 * kq);
      // A is symmetric: its diagonal and upper 16x16 tiles only (the write-out mirrors the rest)
#pragma unroll
      for (int i = 0; i < TP; ++i)
#pragma unroll
        for (int j = i; j < TP; ++j)
          accP[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(at[i], at[j], accP[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < TR; ++i)
#pragma unroll
        for (int j = 0; j < TP; ++j)
          accR[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ay[i], at[j], accR[i][j], 0, 0, 0);
    }
    wave_sync();
  }

  // fixed-order reduction of the four waves' tiles, then one FP64 partial per workgroup
  __syncthreads();
  const int nent = na * na + mr * na;
  float* red = reinterpret_cast<float*>(smem_raw);  // [kBWaves][nent]
  {
    const int col = lane % 16;
#pragma unroll
    for (int i = 0; i < TP; ++i)
#pragma unroll
      for (int j = i; j < TP; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * i + 4 * (lane / 16) + v, c = 16 * j + col;
          if (r < na && c < na) {
            red[w * nent + r + na * c] = accP[i][j][v];
            if (j > i) red[w * nent + c + na * r] = accP[i][j][v];
          }
        }
#pragma unroll
    for (int i = 0; i < TR; ++i)
#pragma unroll
      for (int j = 0; j < TP; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * i + 4 * (lane / 16) + v, c = 16 * j + col;
          if (r < mr && c < na) red[w * nent + na * na + r + mr * c] = accR[i][j][v];
        }
  }
  __syncthreads();
  for (int e = tid; e < nent; e += blockDim.x) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < kBWaves; ++q) v += (double)red[q * nent + e];
    part[(size_t)blockIdx.x * nent + e] = v;
  }
}

// batch size: about 48 columns of k per batch (a multiple of 16 where mc allows).  Each batch
// waits on its codes and signals before its products, so the kernel lives on the number of
// waves in flight: 48 columns leave room for 20 waves per CU (the register limit; 12 at 96
// columns, where LDS was the limit), 17-23% faster on 1M 12 x 12 signals.
int bf16_batch(int mc) {
  int bs = 48 / mc;
  if (bs < 1) bs = 1;
  return bs;
}

size_t bf16_lds(int na, int mr, int mc, int s, int nbo) {
  const int tp = (na + 15) / 16, tr = (mr + 15) / 16;
  const BLayout BL = blayout(bf16_batch(mc), mc, s, tp, tr);
  const size_t lds = (size_t)kBWaves * BL.wave_bytes + (size_t)mc * nbo * 4;
  const size_t red = (size_t)kBWaves * (na * na + mr * na) * 4;
  return red > lds ? red : lds;
}

typedef hipError_t (*BLaunch)(const TmodArgs<float>&, double*, int, int, size_t, hipStream_t);
typedef const void* (*BFunc)();

template <int TP, int TR, int S>
hipError_t launch_b(const TmodArgs<float>& a, double* part, int nblk, int bs, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL((tmod_sums_bf16_kernel<TP, TR, S>), dim3(nblk), dim3(kWave * kBWaves), lds, st, a, part, nblk,
                     bs);
  return hipGetLastError();
}
template <int TP, int TR, int S>
const void* func_b() {
  return reinterpret_cast<const void*>(&tmod_sums_bf16_kernel<TP, TR, S>);
}

struct BVariant {
  int tp, tr, s;
  BLaunch launch;
  BFunc func;
};

// (16-row tiles over the atoms, over the signal rows, s): the SDL_MIXED_BF16 shapes, both sides
#define SDL_BSUMS(X) X(2, 1, 12) X(1, 1, 8) X(2, 1, 10)
const BVariant kBVariants[] = {
#define X(P_, R_, S_) {P_, R_, S_, &launch_b<P_, R_, S_>, &func_b<P_, R_, S_>},
    SDL_BSUMS(X)
#undef X
};

const BVariant* find_b(int tp, int tr, int s) {
  for (const BVariant& v : kBVariants)
    if (v.tp == tp && v.tr == tr && v.s == s) return &v;
  return nullptr;
}

int g_bcus = 256;

}  // namespace

bool tmod_sums_bf16_supported(int m1, int m2, int n1, int n2, int s) {
  return find_b((n1 + 15) / 16, (m1 + 15) / 16, s) && find_b((n2 + 15) / 16, (m2 + 15) / 16, s);
}

int tmod_bf16_num_blocks(int64_t N, int na, int mr, int mc, int s, int nbo) {
  const BVariant* v = find_b((na + 15) / 16, (mr + 15) / 16, s);
  const int bs = bf16_batch(mc);
  int pc = 1;
  if (v && hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, v->func(), kWave * kBWaves, bf16_lds(na, mr, mc, s, nbo)) !=
               hipSuccess)
    pc = 1;
  if (pc < 1) pc = 1;
  if (pc > kBMaxBlocksPerCu) pc = kBMaxBlocksPerCu;
  int64_t b = (N + (int64_t)kBWaves * bs - 1) / ((int64_t)kBWaves * bs);
  if (b > (int64_t)g_bcus * pc) b = (int64_t)g_bcus * pc;
  if (b < 1) b = 1;
  return (int)b;
}

void tmod_bf16_set_cus(int n) {
  if (n > 0) g_bcus = n;
}

hipError_t launch_tmod_sums_bf16(const TmodArgs<float>& a, double* part, hipStream_t st) {
  const int na = a.side == 1 ? a.n1 : a.n2;
  const int mr = a.side == 1 ? a.m1 : a.m2;
  const int mc = a.side == 1 ? a.m2 : a.m1;
  const int nbo = a.side == 1 ? a.n2 : a.n1;
  const BVariant* v = find_b((na + 15) / 16, (mr + 15) / 16, a.s);
  if (!v || !a.Yh) return hipErrorInvalidValue;
  const int nblk = tmod_bf16_num_blocks(a.N, na, mr, mc, a.s, nbo);
  return v->launch(a, part, nblk, bf16_batch(mc), bf16_lds(na, mr, mc, a.s, nbo), st);
}

hipError_t tmod_sums_bf16_init_device() {
  for (const BVariant& v : kBVariants) {
    const hipError_t e = hipFuncSetAttribute(v.func(), hipFuncAttributeMaxDynamicSharedMemorySize, kBMaxDynLds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace sdl
