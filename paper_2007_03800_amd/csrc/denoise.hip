// Patch-denoising driver of the experiments in Sec. IV: an H x W image is cut into all
// (H - m1 + 1)(W - m2 + 1) overlapping m1 x m2 patches (stride 1), the patches are coded (the
// error-driven 2D-OMP of sdl_sparse_code with err2), and the image is put back together from the
// coded patches D1 X_k D2^T, every pixel the plain average of the estimates of the patches that
// cover it.
//
// Image: row-major, pixel (y, x) at y W + x.  Patch k = r C + c (C = W - m2 + 1) holds pixel
// (r + i, c + j) at its (i, j), stored column-major like every signal of the library.
// The rebuild is one tiled pass (rebuild_kernel): each output pixel sums its covering patches'
// estimates in a fixed order, computed on the fly from codes gathered into LDS; nothing adds
// into the image atomically and the result is reproducible.
#include "sdl_internal.h"

namespace sdl {
namespace {

// A wave copies kPatchU patches at a time (wave-uniform patch indices, grid-stride): lane e of
// a chunk of kWave elements takes element e = i + m1 j of each, all loads issued before the
// stores (one load-store chain per wave leaves the copy latency-bound), and each patch's m1 m2
// values go out as one contiguous run.
constexpr int kPatchU = 8;

template <typename T>
__global__ void __launch_bounds__(256) image_to_patches_kernel(const T* __restrict__ img, int H, int W, int m1, int m2,
                                                               T* __restrict__ out, int64_t N) {
  const int C = W - m2 + 1, M = m1 * m2;
  const int lane = threadIdx.x % kWave;
  const int wpb = blockDim.x / kWave;
  const int64_t w0 = (int64_t)blockIdx.x * wpb + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t nwv = (int64_t)gridDim.x * wpb;
  for (int e0 = 0; e0 < M; e0 += kWave) {
    const int e = e0 + lane, i = e % m1, j = e / m1;
    for (int64_t k0 = w0 * kPatchU; k0 < N; k0 += nwv * kPatchU) {
      T v[kPatchU];
#pragma unroll
      for (int u = 0; u < kPatchU; ++u) {
        const int64_t k = k0 + u, r = k / C, c = k - r * C;
        v[u] = e < M && k < N ? img[(r + i) * W + (c + j)] : T(0);
      }
#pragma unroll
      for (int u = 0; u < kPatchU; ++u)
        if (e < M && k0 + u < N) out[(k0 + u) * M + e] = v[u];
    }
  }
}

// The rebuild in one pass, tiled over the output: a workgroup owns a kTile x kTile block of
// pixels, one thread each.  It first gathers the codes of the patches covering the block into
// LDS: one lane per support slot (a power-of-two group of lanes per patch, kStageU patches per
// group and pass with all their loads issued first), a ballot finds the used slots, one LDS
// atomic per patch reserves their room in a pool, and they are stored there in slot order as
// (m1 i, m2 j) offsets with their coefficients, beside the patch's count and pool start.  Each
// pixel then sums the estimates of its covering patches (r, c) in increasing r, then c, each
// estimate sum_t x_t D1[y-r, i_t] D2[x-c, j_t] over the patch's used slots in slot order, and
// divides by their count.  A patch whose slots no longer fit in the pool is read from global
// memory instead, with the same arithmetic in the same order, so the values do not depend on
// which patches got room (nor on the tiling), and there are no atomics on the image.
// Estimates never reach HBM: the codes are read about ((kTile + m - 1) / kTile)^2 times (the
// overlaps mostly from L2) and the image written once.
constexpr int kTile = 16;
constexpr int kStageU = 8;
constexpr size_t kRebuildLds = 40 * 1024;  // four workgroups per CU

template <typename T>
__global__ void __launch_bounds__(kTile* kTile) rebuild_kernel(const int32_t* __restrict__ supp,
                                                              const T* __restrict__ coef, const T* __restrict__ D1,
                                                              const T* __restrict__ D2, int H, int W, int m1, int m2,
                                                              int n1, int n2, int s, int pool, T* __restrict__ img) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int R = H - m1 + 1, C = W - m2 + 1;
  const int PC = kTile + m2 - 1, PT = (kTile + m1 - 1) * PC;  // covering patches of a tile, at most
  T* sD1 = reinterpret_cast<T*>(smem_raw);                     // m1 x n1
  T* sD2 = sD1 + m1 * n1;                                      // m2 x n2
  T* tcf = sD2 + m2 * n2;                                      // pool coefficients
  unsigned* tof = reinterpret_cast<unsigned*>(tcf + pool);     // pool offsets m1 i | (m2 j) << 16
  // per patch: its used slots and pool start (-1: not in the pool), 8-byte aligned
  int2* nb = reinterpret_cast<int2*>(((uintptr_t)(tof + pool) + 7) & ~(uintptr_t)7);
  int* top = reinterpret_cast<int*>(nb + PT);  // pool entries reserved
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave, nw = blockDim.x / kWave;
  const int y0 = blockIdx.y * kTile, x0 = blockIdx.x * kTile;
  // the block's covering patches: rows rb..re and columns cb..ce of the patch grid
  const int rb = max(0, y0 - m1 + 1), re = min(R - 1, y0 + kTile - 1);
  const int cb = max(0, x0 - m2 + 1), ce = min(C - 1, x0 + kTile - 1);
  const int npc = ce - cb + 1, np = (re - rb + 1) * npc;
  for (int e = tid; e < m1 * n1; e += blockDim.x) sD1[e] = D1[e];
  for (int e = tid; e < m2 * n2; e += blockDim.x) sD2[e] = D2[e];
  if (tid == 0) *top = 0;
  __syncthreads();
  int sw = 1;  // lanes per patch: the power of two >= s
  while (sw < s) sw <<= 1;
  const int gpw = kWave / sw, g = lane / sw, sl = lane % sw;
  const unsigned long long gm = (sw == kWave ? ~0ull : (1ull << sw) - 1ull) << (g * sw);
  const int pstep = nw * gpw;  // patches per pass of the workgroup
  for (int p0 = wv * gpw; p0 < np; p0 += kStageU * pstep) {  // wave-uniform trip count
    int a[kStageU];
    T cf[kStageU];
#pragma unroll
    for (int u = 0; u < kStageU; ++u) {
      const int p = p0 + u * pstep + g;
      a[u] = -1;
      cf[u] = 0;
      if (p < np && sl < s) {
        const int64_t k = (int64_t)(rb + p / npc) * C + (cb + p % npc);
        a[u] = supp[k * s + sl];
        cf[u] = coef[k * s + sl];
      }
    }
#pragma unroll
    for (int u = 0; u < kStageU; ++u) {
      const int p = p0 + u * pstep + g;
      const unsigned long long mine = __ballot(a[u] >= 0) & gm;
      const int cnt = __popcll(mine);
      const int pos = __popcll(mine & ((1ull << lane) - 1ull));  // rank among the patch's used slots
      int base = 0;
      if (p < np && sl == 0 && cnt > 0) base = atomicAdd(top, cnt);
      base = __shfl(base, g * sw);
      const bool fits = base + cnt <= pool;
      if (p < np) {
        const int lp = (p / npc) * PC + p % npc;
        if (sl == 0) nb[lp] = make_int2(cnt, fits ? base : -1);
        if (a[u] >= 0 && fits) {
          tof[base + pos] = (unsigned)(m1 * (a[u] % n1)) | ((unsigned)(m2 * (a[u] / n1)) << 16);
          tcf[base + pos] = cf[u];
        }
      }
    }
  }
  __syncthreads();
  const int y = y0 + tid / kTile, x = x0 + tid % kTile;
  if (y >= H || x >= W) return;
  const int r0 = y - m1 + 1 > 0 ? y - m1 + 1 : 0, r1 = y < R - 1 ? y : R - 1;
  const int c0 = x - m2 + 1 > 0 ? x - m2 + 1 : 0, c1 = x < C - 1 ? x : C - 1;
  T acc = 0;
  for (int r = r0; r <= r1; ++r)
    for (int c = c0; c <= c1; ++c) {
      const int i = y - r, j = x - c;
      const int2 cb2 = nb[(r - rb) * PC + (c - cb)];
      const int n = cb2.x, b = cb2.y;
      T v = 0;
      if (b >= 0) {
        for (int q = b; q < b + n; ++q) {
          const unsigned o = tof[q];
          v += tcf[q] * sD1[i + (int)(o & 0xFFFFu)] * sD2[j + (int)(o >> 16)];
        }
      } else {
        const int64_t k = (int64_t)r * C + c;
        for (int t = 0; t < s; ++t) {
          const int at = supp[k * s + t];
          if (at < 0) continue;
          v += coef[k * s + t] * sD1[i + m1 * (at % n1)] * sD2[j + m2 * (at / n1)];
        }
      }
      acc += v;
    }
  img[(int64_t)y * W + x] = acc / (T)((r1 - r0 + 1) * (c1 - c0 + 1));
}

// LDS of rebuild_kernel with a pool of `pool` slots
template <typename T>
size_t rebuild_lds_bytes(int m1, int m2, int n1, int n2, int pool) {
  const size_t pt = (size_t)(kTile + m1 - 1) * (kTile + m2 - 1);
  return sizeof(T) * ((size_t)m1 * n1 + (size_t)m2 * n2) + (sizeof(T) + sizeof(unsigned)) * (size_t)pool +
         8 + sizeof(int2) * pt + sizeof(int);  // 8: alignment of the int2 table
}

}  // namespace

template <typename T>
hipError_t launch_image_to_patches(const T* img, int H, int W, int m1, int m2, T* out, hipStream_t st) {
  const int64_t N = (int64_t)(H - m1 + 1) * (W - m2 + 1);
  if (N <= 0) return hipSuccess;
  int64_t blocks = (N + 4 * kPatchU - 1) / (4 * kPatchU);  // four waves per workgroup
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(image_to_patches_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, st, img, H, W, m1, m2, out, N);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_patches_to_image(const int32_t* supp, const T* coef, const T* D1, const T* D2, int H, int W, int m1,
                                   int m2, int n1, int n2, int s, T* img, hipStream_t st) {
  if ((int64_t)H * W <= 0) return hipSuccess;
  // the pool takes what kRebuildLds leaves, and never more than every slot of every patch
  const int64_t pt = (int64_t)(kTile + m1 - 1) * (kTile + m2 - 1);
  const size_t fixed = rebuild_lds_bytes<T>(m1, m2, n1, n2, 0);
  int64_t pool = fixed < kRebuildLds ? (int64_t)((kRebuildLds - fixed) / (sizeof(T) + sizeof(unsigned))) : 0;
  if (pool > pt * s) pool = pt * s;
  const size_t lds = rebuild_lds_bytes<T>(m1, m2, n1, n2, (int)pool);
  const dim3 grid((unsigned)((W + kTile - 1) / kTile), (unsigned)((H + kTile - 1) / kTile));
  hipLaunchKernelGGL(rebuild_kernel<T>, grid, dim3(kTile * kTile), lds, st, supp, coef, D1, D2, H, W, m1, m2, n1, n2,
                     s, (int)pool, img);
  return hipGetLastError();
}

hipError_t denoise_init_device() {
  // the dictionaries and per-patch tables of the largest shapes (64 x 64 patches, FP64) need
  // up to ~90 KiB (then with no pool)
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&rebuild_kernel<float>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&rebuild_kernel<double>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

template hipError_t launch_image_to_patches<float>(const float*, int, int, int, int, float*, hipStream_t);
template hipError_t launch_image_to_patches<double>(const double*, int, int, int, int, double*, hipStream_t);
template hipError_t launch_patches_to_image<float>(const int32_t*, const float*, const float*, const float*, int, int,
                                                   int, int, int, int, int, float*, hipStream_t);
template hipError_t launch_patches_to_image<double>(const int32_t*, const double*, const double*, const double*, int,
                                                    int, int, int, int, int, int, double*, hipStream_t);

}  // namespace sdl
