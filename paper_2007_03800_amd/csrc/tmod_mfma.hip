// TMOD partial sums on the matrix cores (Algorithm 1 steps 1 and 3).
//
// Side 1 (Corollary 1):  T_k = X_k D2^T (n1 x m2),  A = sum T_k T_k^T,  B = sum Y_k T_k^T
// Side 2 (Result 1): U_k = (D1 X_k)^T (n2 x m1), A = sum U_k U_k^T, B = sum Y_k^T U_k^T
//
// For a batch of bs signals the per-signal factors are laid side by side,
// Tcat = [T_1 ... T_bs] (na x K) and Ycat = [Yt_1 ... Yt_bs] (mr x K) with
// K = bs*mc, so the batch's contribution is two dense products with a long inner
// dimension: A += Tcat Tcat^T and B += Ycat Tcat^T.  Each wave builds Tcat in
// LDS from the sparse codes (one lane per column, so the scatter has no
// conflicts), stages Ycat with coalesced loads, and runs 16x16x4 MFMAs with FP32
// (or FP64) accumulation over K.  The four waves of a workgroup add their tiles in
// a fixed order and write one FP64 partial per workgroup; a separate fixed-order
// reduction and the FP64 solve follow (no floating-point atomics anywhere, so
// results are bitwise reproducible).
#include "sdl_internal.h"

namespace sdl {
namespace {

constexpr int kWaves = 4;
constexpr int kMaxBlocksPerCu = 4;  // grid cap: one round of at most 4 workgroups per CU
constexpr int kMaxDynLds = 160 * 1024;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// 16x16x4 MFMA: lane l supplies A[l%16][l/16] and B[l/16][l%16]; result element v of
// lane l is D[row(l, v)][l%16], where the row order differs between the FP32 and
// FP64 instructions (checked on the device).
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  using V = f32x4;
  static __device__ inline V step(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int lane, int v) { return 4 * (lane / 16) + v; }
};
template <>
struct Mfma<double> {
  using V = f64x4;
  static __device__ inline V step(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int lane, int v) { return lane / 16 + 4 * v; }
};

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// TP = 16-row tiles over the na atoms, TR = 16-row tiles over the mr signal rows.
template <typename T, int TP, int TR>
__global__ void __launch_bounds__(kWave* kWaves) tmod_sums_kernel(TmodArgs<T> a, double* part, int nblk, int bs) {
  using MF = Mfma<T>;
  using V = typename MF::V;
  constexpr int NP = 16 * TP + 1, MP = 16 * TR + 1;  // padded LDS row lengths (bank spread)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const int side = a.side, n1 = a.n1, s = a.s;
  const int na = side == 1 ? a.n1 : a.n2;
  const int mr = side == 1 ? a.m1 : a.m2;
  const int mc = side == 1 ? a.m2 : a.m1;
  const int M = a.m1 * a.m2;
  const int K = bs * mc, K4 = (K + 3) & ~3;
  const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
  const int nbo = side == 1 ? a.n2 : a.n1;                 // atoms of the fixed dictionary
  const size_t per_wave = (size_t)K4 * (NP + MP) + 2 * (size_t)bs * s;
  T* Do = smem + (size_t)kWaves * per_wave;                // fixed dictionary, mc x nbo
  T* Tb = smem + (size_t)w * per_wave;                     // [K4][NP]  Tcat, column-major by k
  T* Yt = Tb + (size_t)K4 * NP;                            // [K4][MP]  Ycat
  T* cval = Yt + (size_t)K4 * MP;                          // codes of the batch
  int* cidx = reinterpret_cast<int*>(cval + bs * s);
  for (int e = tid; e < mc * nbo; e += blockDim.x) Do[e] = a.Dother[e];
  __syncthreads();
  const int64_t k0 = (a.N * blockIdx.x) / nblk, k1 = (a.N * (blockIdx.x + 1)) / nblk;
  const int64_t nbatch = (k1 - k0 + bs - 1) / bs;

  V accP[TP][TP], accR[TR][TP];
#pragma unroll
  for (int i = 0; i < TP; ++i)
#pragma unroll
    for (int j = 0; j < TP; ++j) accP[i][j] = V{0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < TR; ++i)
#pragma unroll
    for (int j = 0; j < TP; ++j) accR[i][j] = V{0, 0, 0, 0};

  for (int64_t bi = w; bi < nbatch; bi += kWaves) {
    const int64_t kb = k0 + bi * bs;
    const int nb = (int)((k1 - kb) < bs ? (k1 - kb) : bs);
    // the batch's codes, staged with contiguous loads; atom a = i + n1 j split once here into
    // this side's (row | other << 16), -1 for unused slots
    for (int e = lane; e < nb * s; e += kWave) {
      const int at = a.supp[kb * s + e];
      const int i = at % n1, j = at / n1;
      cidx[e] = at < 0 ? -1 : (side == 1 ? (i | (j << 16)) : (j | (i << 16)));
      cval[e] = a.coef[kb * s + e];
    }
    wave_sync();
    // each lane owns whole columns k = b*mc + c of Tcat and Ycat: no cross-lane hazards
    for (int e = lane; e < K4; e += kWave) {
      const int b = e / mc, c = e % mc;
      T* tcol = Tb + (size_t)e * NP;
      T* ycol = Yt + (size_t)e * MP;
      for (int r = 0; r < NP; ++r) tcol[r] = T(0);
      if (b < nb) {
        for (int t = 0; t < s; ++t) {
          const int pk = cidx[b * s + t];
          if (pk < 0) continue;
          tcol[pk & 0xFFFF] += cval[b * s + t] * Do[c + mc * (pk >> 16)];
        }
        const int64_t yb = (kb + b) * M;
        for (int r = 0; r < mr; ++r) {
          const int64_t e = yb + (side == 1 ? r + a.m1 * c : c + a.m1 * r);  // column / row c of Y_b
          ycol[r] = a.Yh ? (T)bf16_to_float(a.Yh[e]) : a.Y[e];
        }
        for (int r = mr; r < MP; ++r) ycol[r] = T(0);
      } else {
        for (int r = 0; r < MP; ++r) ycol[r] = T(0);
      }
    }
    wave_sync();
    const int r16 = lane % 16, kq = lane / 16;
    for (int kk = 0; kk < K4; kk += 4) {
      const int k = kk + kq;
      T at[TP], ay[TR];
#pragma unroll
      for (int i = 0; i < TP; ++i) at[i] = Tb[k * NP + 16 * i + r16];
#pragma unroll
      for (int i = 0; i < TR; ++i) ay[i] = Yt[k * MP + 16 * i + r16];
      // P is symmetric: its diagonal and upper 16x16 tiles only (the write-out mirrors the rest)
#pragma unroll
      for (int i = 0; i < TP; ++i)
#pragma unroll
        for (int j = i; j < TP; ++j) accP[i][j] = MF::step(at[i], at[j], accP[i][j]);
#pragma unroll
      for (int i = 0; i < TR; ++i)
#pragma unroll
        for (int j = 0; j < TP; ++j) accR[i][j] = MF::step(ay[i], at[j], accR[i][j]);
    }
    wave_sync();
  }

  // fixed-order reduction of the four waves' tiles, then one FP64 partial per workgroup
  __syncthreads();
  const int nent = na * na + mr * na;
  T* red = smem;  // [kWaves][nent]
  {
    const int col = lane % 16;
#pragma unroll
    for (int i = 0; i < TP; ++i)
#pragma unroll
      for (int j = i; j < TP; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * i + MF::row(lane, v), c = 16 * j + col;
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
          const int r = 16 * i + MF::row(lane, v), c = 16 * j + col;
          if (r < mr && c < na) red[w * nent + na * na + r + mr * c] = accR[i][j][v];
        }
  }
  __syncthreads();
  for (int e = tid; e < nent; e += blockDim.x) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) v += (double)red[q * nent + e];
    part[(size_t)blockIdx.x * nent + e] = v;
  }
}

template <typename T, int TP, int TR>
hipError_t launch_tp_tr(const TmodArgs<T>& a, double* part, int nblk, int bs, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL((tmod_sums_kernel<T, TP, TR>), dim3(nblk), dim3(kWave * kWaves), lds, st, a, part, nblk, bs);
  return hipGetLastError();
}

template <typename T, int TP>
hipError_t launch_tp(int tr, const TmodArgs<T>& a, double* part, int nblk, int bs, size_t lds, hipStream_t st) {
  switch (tr) {
    case 1: return launch_tp_tr<T, TP, 1>(a, part, nblk, bs, lds, st);
    case 2: return launch_tp_tr<T, TP, 2>(a, part, nblk, bs, lds, st);
    case 3: return launch_tp_tr<T, TP, 3>(a, part, nblk, bs, lds, st);
    default: return launch_tp_tr<T, TP, 4>(a, part, nblk, bs, lds, st);
  }
}

// Workgroups of one instantiation that fit on a CU at once with `lds` bytes of LDS
// (registers and LDS, as the runtime computes it); 1 if the query fails.
template <typename T, int TP, int TR>
int per_cu_tp_tr(size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&tmod_sums_kernel<T, TP, TR>),
                                                   kWave * kWaves, lds) != hipSuccess || n < 1)
    n = 1;
  return n;
}

template <typename T, int TP>
int per_cu_tp(int tr, size_t lds) {
  switch (tr) {
    case 1: return per_cu_tp_tr<T, TP, 1>(lds);
    case 2: return per_cu_tp_tr<T, TP, 2>(lds);
    case 3: return per_cu_tp_tr<T, TP, 3>(lds);
    default: return per_cu_tp_tr<T, TP, 4>(lds);
  }
}

template <typename T>
int per_cu(int tp, int tr, size_t lds) {
  switch (tp) {
    case 1: return per_cu_tp<T, 1>(tr, lds);
    case 2: return per_cu_tp<T, 2>(tr, lds);
    case 3: return per_cu_tp<T, 3>(tr, lds);
    default: return per_cu_tp<T, 4>(tr, lds);
  }
}

int g_tcus = 256;

}  // namespace

// batch size so one wave's staging stays near 12 KiB (FP32) / 24 KiB (FP64)
static int sums_batch(int na, int mr, int mc) {
  const int tp = (na + 15) / 16, tr = (mr + 15) / 16;
  const int per = mc * (16 * tp + 1 + 16 * tr + 1);
  int bs = 3072 / per;
  if (bs < 1) bs = 1;
  if (bs > 32) bs = 32;
  return bs;
}

// dynamic LDS of one workgroup: four waves' staging plus the fixed dictionary (and at least
// the end-of-kernel reduction buffer)
static size_t sums_lds(int na, int mr, int mc, int s, int nbo, size_t elem) {
  const int bs = sums_batch(na, mr, mc);
  const int tp = (na + 15) / 16, tr = (mr + 15) / 16;
  const int K4 = (bs * mc + 3) & ~3;
  size_t lds = ((size_t)kWaves * ((size_t)K4 * (16 * tp + 1 + 16 * tr + 1) + 2 * (size_t)bs * s) + (size_t)mc * nbo) * elem;
  const size_t red = (size_t)kWaves * (na * na + mr * na) * elem;
  return red > lds ? red : lds;
}

void tmod_set_cus(int n) {
  if (n > 0) g_tcus = n;
}

// One round of resident workgroups (CUs x workgroups per CU, at most kMaxBlocksPerCu), or
// fewer when the signals run out; the same count sizes the partial buffer and the
// reduction.
int tmod_num_blocks_for(int64_t N, int na, int mr, int mc, int s, int nbo, size_t elem) {
  const int bs = sums_batch(na, mr, mc);
  const int tp = (na + 15) / 16, tr = (mr + 15) / 16;
  const size_t lds = sums_lds(na, mr, mc, s, nbo, elem);
  int pc = elem == 8 ? per_cu<double>(tp, tr, lds) : per_cu<float>(tp, tr, lds);
  if (pc > kMaxBlocksPerCu) pc = kMaxBlocksPerCu;
  int64_t b = (N + (int64_t)kWaves * bs - 1) / ((int64_t)kWaves * bs);
  if (b > (int64_t)g_tcus * pc) b = (int64_t)g_tcus * pc;
  if (b < 1) b = 1;
  return (int)b;
}

template <typename T>
hipError_t launch_tmod_sums(const TmodArgs<T>& a, double* part, hipStream_t st) {
  const int na = a.side == 1 ? a.n1 : a.n2;
  const int mr = a.side == 1 ? a.m1 : a.m2;
  const int mc = a.side == 1 ? a.m2 : a.m1;
  const int nbo = a.side == 1 ? a.n2 : a.n1;
  const int bs = sums_batch(na, mr, mc);
  const int nblk = tmod_num_blocks_for(a.N, na, mr, mc, a.s, nbo, sizeof(T));
  const int tp = (na + 15) / 16, tr = (mr + 15) / 16;
  const size_t lds = sums_lds(na, mr, mc, a.s, nbo, sizeof(T));
  switch (tp) {
    case 1: return launch_tp<T, 1>(tr, a, part, nblk, bs, lds, st);
    case 2: return launch_tp<T, 2>(tr, a, part, nblk, bs, lds, st);
    case 3: return launch_tp<T, 3>(tr, a, part, nblk, bs, lds, st);
    default: return launch_tp<T, 4>(tr, a, part, nblk, bs, lds, st);
  }
}

template <typename T, int TP, int TR>
hipError_t allow_lds() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&tmod_sums_kernel<T, TP, TR>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
}

template <typename T>
hipError_t allow_lds_all() {
  hipError_t e = hipSuccess;
#define A_(P, R) \
  if (e == hipSuccess) e = allow_lds<T, P, R>();
  A_(1, 1) A_(1, 2) A_(1, 3) A_(1, 4) A_(2, 1) A_(2, 2) A_(2, 3) A_(2, 4)
  A_(3, 1) A_(3, 2) A_(3, 3) A_(3, 4) A_(4, 1) A_(4, 2) A_(4, 3) A_(4, 4)
#undef A_
  return e;
}

hipError_t tmod_sums_init_device() {
  hipError_t e = allow_lds_all<float>();
  return e == hipSuccess ? allow_lds_all<double>() : e;
}

template hipError_t launch_tmod_sums<float>(const TmodArgs<float>&, double*, hipStream_t);
template hipError_t launch_tmod_sums<double>(const TmodArgs<double>&, double*, hipStream_t);

}  // namespace sdl
