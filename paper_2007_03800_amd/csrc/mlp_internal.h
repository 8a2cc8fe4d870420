// Internal declarations of the learned-proposal kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sdl_internal.h"

namespace sdl {

enum : int { kEpiStoreF32 = 0, kEpiBiasGelu = 1, kEpiGeluGrad = 2 };

// C (M x N, ldc) = op(A) (M x K) * op(B) (K x N) with a fused epilogue.
// M % 64 == 0, N % 64 == 0, K % 32 == 0.
struct GemmArgs {
  const void* A;
  const void* B;
  void* C;
  int M, N, K, lda, ldb, ldc;
  int epi;
  const float* bias;  // kEpiStoreF32 (optional), kEpiBiasGelu
  float* Z;           // kEpiBiasGelu: pre-activation out (optional); kEpiGeluGrad: pre-activation in
};

template <typename T>
hipError_t launch_gemm(const GemmArgs& g, int opA, int opB, hipStream_t st);
template <typename T>
hipError_t launch_prep_input(const float* Y, const int32_t* idx, int64_t B, int M, T* X, float* ynorm2, hipStream_t st);
template <typename T>
hipError_t launch_bce_grad(const float* Z, const int32_t* supp, const int32_t* idx, int64_t B, int A, int s, T* dZ,
                           double* loss_part, double* loss, hipStream_t st);
template <typename T>
hipError_t launch_bias_grad(const T* dZ, int64_t B, int N, float* db, hipStream_t st);
template <typename T>
hipError_t launch_adam(float* p, float* m, float* v, const float* g, T* pc, int64_t n, float lr, int step,
                       hipStream_t st);
template <typename T>
hipError_t launch_copy_params(const float* p, T* pc, int64_t n, hipStream_t st);

// Proposal: top-s atoms of the logits (ties: smallest index), least squares on them,
// explicit residual; accept[k] = res2 <= tau * ||Y_k||^2.
struct ProposeArgs {
  int m1, m2, n1, n2, s;
  int64_t N;
  const float* logits;  // N x (n1*n2)
  const float* Y;
  const float* D1;
  const float* D2;
  const float* G1;
  const float* G2;
  int32_t* supp;
  float* coef;
  float* res2;
  int32_t* accept;
  double tau;
};
bool propose_supported(int n1, int n2, int s);
hipError_t launch_propose(const ProposeArgs& a, hipStream_t st);

// Ascending list of the k with accept[k] == 0; *count = its length.  blkcount holds
// compact_blocks(N) ints.
int compact_blocks(int64_t N);
hipError_t launch_compact_rejected(const int32_t* accept, int64_t N, int32_t* blkcount, int32_t* list, int32_t* count,
                                   hipStream_t st);

}  // namespace sdl
