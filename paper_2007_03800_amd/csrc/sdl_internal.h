// Internal declarations shared by the HIP translation units of libsdl.
// Device code targets gfx950 (CDNA4, wave64) only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sdl.h"

namespace sdl {

constexpr int kWave = 64;

// Device-side status bits, OR-ed into a per-call word and read back at sync.
enum : int { kStatusSingular = 1, kStatusNonfinite = 2 };

// Device counters (one int64-sized slot each) accumulated with integer atomics.
enum : int {
  kCtrEarlyStop = 0,
  kCtrFp64Pivot = 1,
  kCtrUnusedAtoms = 2,
  kCtrSingular = 3,
  kCtrRescored = 4,     // SDL_MIXED_BF16: signal steps with more than one candidate re-scored in FP32
  kCtrTieOverflow = 5,  // SDL_MIXED_BF16: signal steps where a lane's second key was within the band
  kCtrProposed = 6,     // learned path: signals given a proposal
  kCtrFallback = 7,     // learned path: signals whose proposal failed the test (coded by 2D-OMP)
  kNumCounters = 8
};

// Arguments of one sparse-coding launch over one problem.
template <typename T>
struct OmpArgs {
  int m1, m2, n1, n2, s;
  int64_t N;
  const T* Y;
  const uint16_t* Yh;  // non-null: the signals are bfloat16 (Y unused), widened to FP32 on load
  const T* D1;  // m1 x n1 column-major, in the compute type
  const T* D2;  // m2 x n2
  const T* G1;  // n1 x n1 = D1^T D1
  const T* G2;  // n2 x n2 = D2^T D2
  int32_t* supp;
  T* coef;
  T* res2;  // may be null
  double stop_rel, dep_eps, pivot_fp64;
  double err2;  // > 0: error-driven stop (generic kernel only), residual energy target
  double tie_band;  // SDL_MIXED_BF16: relative band of BF16 near-ties re-scored in FP32
  unsigned long long* counters;  // kNumCounters entries
  // Register-resident kernel only: also accumulate the TMOD sums of the new codes for
  // side sums_side (1: D1 update, 2: D2 update; 0: none) plus the sum of res2, one
  // row of (nent + 1) doubles per wave into sums_part (see omp_fast_partial_rows).
  int sums_side;
  double* sums_part;
  // Register-resident kernel only: code only the signals index[0 .. *count-1] (device
  // pointers; outputs go to those positions).  Null: all N signals in order.
  const int32_t* index;
  const int32_t* count;
};

// Buffers describing one TMOD half-step for one problem.
template <typename T>
struct TmodArgs {
  int side;  // 1: update D1 (Corollary 1), 2: update D2 (Result 1)
  int m1, m2, n1, n2, s;
  int64_t N;
  const T* Y;
  const uint16_t* Yh;  // non-null: the signals are bfloat16 (Y unused), widened to FP32 on load
  const T* Dother;  // compute-type copy of the dictionary that stays fixed
  const int32_t* supp;
  const T* coef;
};

// bfloat16 bit pattern -> FP32 (exact: the pattern is the upper half of the FP32 encoding)
__device__ inline float bf16_to_float(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Four consecutive signal values starting at element off (a multiple of 4) as FP32:
// one 16-byte load of FP32 signals, or one 8-byte load of bfloat16 signals.
__device__ inline float4 load_signal4(const OmpArgs<float>& a, int64_t off) {
  if (a.Yh) {
    const uint2 h = *reinterpret_cast<const uint2*>(a.Yh + off);
    return make_float4(bf16_to_float((uint16_t)(h.x & 0xFFFFu)), bf16_to_float((uint16_t)(h.x >> 16)),
                       bf16_to_float((uint16_t)(h.y & 0xFFFFu)), bf16_to_float((uint16_t)(h.y >> 16)));
  }
  return *reinterpret_cast<const float4*>(a.Y + off);
}

// ---- launchers (defined in the .hip files) ----
template <typename T>
hipError_t launch_omp_generic(const OmpArgs<T>& a, hipStream_t st);
template <typename T>
bool omp_fast_supported(int m1, int m2, int n1, int n2, int s);
template <typename T>
hipError_t launch_omp_fast(const OmpArgs<T>& a, hipStream_t st);
// One wave per signal with the correlations in registers (omp_wave.hip), for the large
// shapes it is compiled for; FP32 and FP64; no index mode, no sums epilogue.
bool omp_wave_supported(int m1, int m2, int n1, int n2, int s);
bool omp_wave_grid(int m1, int m2, int n1, int n2, int s, int* lanes_row, int* lanes_col);
// Per-shape choice between the fused multi-signal path and the one-wave-per-signal
// path (sparse coding + standalone sums), made by the autotuner or forced (autotune.hip).
bool wave_chosen(int m1, int m2, int n1, int n2, int s);
void set_wave_choice(int m1, int m2, int n1, int n2, int s, bool on, double ms);
double wave_choice_ms(int m1, int m2, int n1, int n2, int s);
template <typename T>
hipError_t launch_omp_wave(const OmpArgs<T>& a, hipStream_t st);
// FP32 on matrix-core quadrants, 16 lanes and 4 signals per wave (omp_quad.hip): the FP32
// form of the standalone-sums path for the shapes it is compiled for (launch_omp_wave
// dispatches to it); no index mode, no sums epilogue.
bool omp_quad_supported(int m1, int m2, int n1, int n2, int s);
// Orthonormal variant (ortho.hip): hard-thresholded codes and the Procrustes update (one wave,
// FP64 Jacobi SVD of the B block of the reduced sums, then D, its compute copy and Gram).
bool ortho_supported(int m1, int m2, int n1, int n2, int s);
template <typename T>
hipError_t launch_ortho_code(const OmpArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_procrustes(const double* src, int nrow, int ld, int n, double* D, T* Dc, double* G64, T* Gc,
                             int* status, unsigned long long* counters, hipStream_t st);
hipError_t ortho_init_device();
// SDL_MIXED_BF16 sparse coding (omp_mixed.hip): correlations D1^T R D2 on the BF16 matrix
// cores every step, near-ties re-scored in FP32; shapes it is compiled for.
bool omp_mixed_supported(int m1, int m2, int n1, int n2, int s);
hipError_t launch_omp_mixed(const OmpArgs<float>& a, hipStream_t st);
hipError_t launch_omp_quad(const OmpArgs<float>& a, hipStream_t st);
// Matrix-core variants (omp_mfma.hip): four lanes per signal, refresh on 4x4x1 MFMA.
struct MfmaVariant {
  int m1, m2, n1, n2, s, wpe;
  hipError_t (*launch)(const OmpArgs<float>&, hipStream_t);
};
extern MfmaVariant mfma_variants_table[];
extern const int mfma_variants_count;
int64_t mfma_partial_rows(int64_t N, int wpe);
void mfma_set_cus(int n);

// Register-resident variants for a shape (VALU layouts and matrix-core layouts): writes
// up to cap variant ids, returns the count.  Info: lane split over atom rows/columns,
// register budget in waves per SIMD, and whether the refresh runs on the matrix cores.
int omp_fast_variants(int m1, int m2, int n1, int n2, int s, int* ids, int cap);
void omp_fast_variant_info(int id, int* lr, int* lc, int* wpe, int* mfma);
hipError_t launch_omp_fast_variant(int id, const OmpArgs<float>& a, hipStream_t st);
// Variant used for a shape: the autotuned one if tuned in this process, else the first listed.
int omp_fast_choice(int m1, int m2, int n1, int n2, int s);
// Partial rows (workgroups) of a register-resident launch over N signals with the
// variant currently chosen for the shape, and the maximum over all variants.
int omp_fast_partial_rows(int64_t N, int m1, int m2, int n1, int n2, int s);
int omp_fast_max_partial_rows();
hipError_t omp_fast_init_device();
void omp_fast_set_choice(int m1, int m2, int n1, int n2, int s, int id);
hipError_t autotune_problem(const OmpArgs<float>& a, hipStream_t st, int reps, int* chosen, double* best_ms);
bool tuned_config(int m1, int m2, int n1, int n2, int s, int* lr, int* lc, int* wpe, int* mfma, double* ms);
// Counter bumped whenever a kernel choice (autotuned or forced) changes.
long tuning_epoch();
size_t omp_generic_lds_bytes(int m1, int m2, int n1, int n2, int s, size_t elem);
hipError_t omp_generic_init_device();

// Workgroup partials of the standalone sums kernel (a fixed function of N and the shape).
// workgroups (= partial rows) of the standalone sums kernel: na atoms being solved, mr
// signal rows on that side, mc the other side's signal extent, s the sparsity, nbo the
// other dictionary's atoms, elem the element size of the arithmetic
int tmod_num_blocks_for(int64_t N, int na, int mr, int mc, int s, int nbo, size_t elem);
void tmod_set_cus(int n);
hipError_t tmod_sums_init_device();
template <typename T>
hipError_t launch_tmod_sums(const TmodArgs<T>& a, double* part, hipStream_t st);
// The same sums on the BF16 matrix cores (SDL_MIXED_BF16; bfloat16 signals), for the shapes
// compiled in tmod_bf16.hip; partial rows: tmod_bf16_num_blocks.
bool tmod_sums_bf16_supported(int m1, int m2, int n1, int n2, int s);
int tmod_bf16_num_blocks(int64_t N, int na, int mr, int mc, int s, int nbo);
void tmod_bf16_set_cus(int n);
hipError_t launch_tmod_sums_bf16(const TmodArgs<float>& a, double* part, hipStream_t st);
hipError_t tmod_sums_bf16_init_device();
// First stage of the fixed-order reduction of P partial rows (row stride ld): when P is
// large, consecutive chunks of rows are summed in row order into stage (which holds
// reduce_stage_rows(P) rows); returns the number of rows the solve kernel still has to
// sum and points *src at them (part itself when P is small, then nothing is launched).
int launch_reduce_stage1(const double* part, int P, int ld, double* stage, const double** src, hipStream_t st,
                         hipError_t* err);
int reduce_stage_rows(int P);
// The last stage alone: out[e] = row-order sum of the nrow rows at src (stride ld), e < n.
hipError_t launch_reduce_final(const double* src, int nrow, int ld, int n, double* out, hipStream_t st);
// *out = sum of res2[0 .. N-1] in a fixed order (nblk = rmse_num_blocks(N) partials in part).
template <typename T>
hipError_t launch_sum_res2(const T* res2, int64_t N, double* part, int nblk, double* out, hipStream_t st);
hipError_t launch_fill_double(double* p, int n, double v, hipStream_t st);
// Optional RMSE output of the solve kernel: trace[*counter + offset] = sqrt(sums[idx] / denom), then ++*counter.
struct RmseOut {
  double* trace;  // null: no RMSE
  int* counter;
  int offset;
  int idx;
  double denom;
};
// Last reduction stage + solve + normalise (one workgroup): sums (ld doubles) = the
// row-order sum of the nrow rows at src; D: the dictionary being updated (mr x na
// FP64, in/out).  tmod_solve_init_device raises the kernel's LDS limit (call once per
// device).
template <typename T>
hipError_t launch_tmod_solve(const double* src, int nrow, int ld, double* sums, int mr, int na, double* D, T* Dc,
                             double* G64, T* Gc, double* w, int* status, unsigned long long* counters,
                             const RmseOut& r, hipStream_t st);
hipError_t tmod_solve_init_device();
// Measurement aids (probe.hip): best copy rate (read + write, GB/s) and arithmetic peaks
// (kind 0 FP32 FMA, 1 FP32 MFMA 16x16x4, 2 FP32 MFMA 4x4x1, 3 FP64 FMA; TFLOP/s).
hipError_t probe_hbm_copy(void* dst, const void* src, size_t bytes, int reps, hipStream_t st, double* gbs);
hipError_t probe_peak(int kind, float* sink, int reps, hipStream_t st, double* tflops);
template <typename T>
hipError_t launch_dict_prep(const double* D, int mr, int na, T* Dc, double* G64, T* Gc, hipStream_t st);
template <typename T>
hipError_t launch_rescale(int side, int n1, int s, int64_t N, const int32_t* supp, T* coef, const double* w,
                          hipStream_t st);
int rmse_num_blocks(int64_t N);
template <typename T>
hipError_t launch_rmse(const T* res2, int64_t N, double denom, double* part, int nblk, double* trace,
                       int stride, int offset, int* counter, hipStream_t st);
template <typename T>
hipError_t launch_check_finite(const T* x, int64_t n, int* status, hipStream_t st);
hipError_t launch_check_finite_bf16(const uint16_t* x, int64_t n, int* status, hipStream_t st);
hipError_t launch_fill_int(int* p, int n, int v, hipStream_t st);
// n-dimensional signals (Remark 3, tensor.hip): m[d] x n[d] dictionaries per mode, atom
// a = i_0 + n_0 (i_1 + n_1 (...)); entries of m and n beyond nmodes are 1.
constexpr int kTensorMaxModes = 4;
template <typename T>
struct TensorArgs {
  int nmodes, s;
  int m[kTensorMaxModes], n[kTensorMaxModes];
  int64_t N;
  const T* Y;
  const T* D[kTensorMaxModes];  // compute-type copies, column-major
  const T* G[kTensorMaxModes];  // their Gram matrices
  int32_t* supp;
  T* coef;
  T* res2;  // may be null
  double stop_rel, dep_eps, pivot_fp64, err2;
  unsigned long long* counters;
};
size_t tensor_omp_lds_bytes(int nmodes, const int* m, const int* n, int s, size_t elem);
size_t tensor_sums_lds(int nmodes, const int* m, const int* n, int mode, size_t elem);
int tensor_sums_rows(int64_t N);  // partial rows written by launch_tensor_sums
template <typename T>
hipError_t launch_tensor_omp(const TensorArgs<T>& a, hipStream_t st);
// sums of the update of mode `mode` (0-based): one row of n^2 + m n doubles per partial row
template <typename T>
hipError_t launch_tensor_sums(const TensorArgs<T>& a, int mode, double* part, hipStream_t st);
template <typename T>
hipError_t launch_tensor_rescale(const TensorArgs<T>& a, int mode, const double* w, hipStream_t st);
hipError_t tensor_init_device();
// Remark 1's codes on the matrix-core multi-signal layout of omp_mfma.hip (FP32), with the update
// sums of a.sums_side in the epilogue (one partial row per workgroup, ortho_mfma_partial_rows)
bool ortho_mfma_supported(int m1, int m2, int n1, int n2, int s);
int64_t ortho_mfma_partial_rows(int64_t N, int m1, int m2, int s);
hipError_t launch_ortho_mfma(const OmpArgs<float>& a, hipStream_t st);
// n-dimensional sparse coding on the two-mode one-wave kernel: the modes after the first
// collapsed into one Kronecker factor (FP32 shapes compiled in omp_wave.hip)
bool omp_wave_collapsed_supported(int m1, int m2, int n1, int n2, int s);
hipError_t launch_omp_wave_collapsed(const OmpArgs<float>& a, hipStream_t st);
// Dk = D_nm-1 (x) ... (x) D_1 (mode 0 excluded): prod_{d>=1} m[d] x prod_{d>=1} n[d], FP64
hipError_t launch_kron_tail(const TensorArgs<double>& d, double* Dk, hipStream_t st);
// Denoising driver (denoise.hip): overlapping patches of a row-major image as column-major
// signals, and the image rebuilt as the average of the coded patches covering each pixel.
template <typename T>
hipError_t launch_image_to_patches(const T* img, int H, int W, int m1, int m2, T* out, hipStream_t st);
// (one pass, no scratch); denoise_init_device raises the rebuild kernel's LDS limit (call once
// per device)
template <typename T>
hipError_t launch_patches_to_image(const int32_t* supp, const T* coef, const T* D1, const T* D2, int H, int W, int m1,
                                   int m2, int n1, int n2, int s, T* img, hipStream_t st);
hipError_t denoise_init_device();

}  // namespace sdl
