// Device routine of the TMOD dictionary update: the FP64 solve on the used atoms with
// normalisation (Corollary 1 / Result 1), which also rewrites the compute-type
// dictionary copy and the Gram matrix.
#pragma once

#include "sdl_internal.h"

namespace sdl {

constexpr double kSpdRelTol = 1e-12;  // Cholesky pivot <= tol * diagonal entry -> not positive definite

// LDS bytes the block solve needs for na atoms and mr rows: the augmented system
// (na rows of na + mr entries, padded), the new dictionary, the pivots' reference
// diagonal and the used-atom list.
__host__ __device__ inline size_t solve_lds_bytes(int na, int mr) {
  return sizeof(double) * ((size_t)na * (na + mr + 1) + (size_t)(mr + 1) * na + na) + sizeof(int) * (na + 1) + 16;
}

// LDS bytes of ld reduced sums kept in front of the solve's workspace (16-byte multiple).
__host__ __device__ inline size_t solve_sums_lds_bytes(int ld) { return ((size_t)ld * sizeof(double) + 15) & ~(size_t)15; }

// Whole workgroup (tid = 0..nt-1).  sums = [A (na x na) | B (mr x na)], column-major,
// A = the update's Gram sum, B = its right-hand side (global memory or LDS, written by the
// caller before a block barrier).  Atoms with A_ii = 0 are used by no code: the
// system decouples exactly and they keep their old value.  On the used set U the
// symmetric positive definite system A_UU D*^T = B_U^T is solved by Gauss-Jordan
// elimination without pivoting on the augmented matrix [A_UU | B_U^T]: step k
// removes column k from every other row using row k as it stands, so each entry is
// written by one thread per step and one barrier per step suffices.  The pivot of
// step k is the k-th Schur complement diagonal, the same quantity a Cholesky
// factorisation takes the root of; a pivot below kSpdRelTol times its diagonal entry
// marks the sum as not positive definite: D is left unchanged and the singular
// status bit is set.  Each solved column is then normalised (w_i = its norm; a zero
// column keeps the old atom), and D, its compute-type copy and the Gram matrix D^T D
// are rewritten.  smem: solve_lds_bytes(na, mr) bytes; nt a multiple of 32.
template <typename T>
__device__ void solve_update_block(const double* sums, int mr, int na, double* D, T* Dc, double* G64, T* Gc,
                                   double* w, int* status, unsigned long long* counters, unsigned char* smem,
                                   int tid, int nt) {
  const int ldm = na + mr + 1;
  double* M = reinterpret_cast<double*>(smem);  // M[k * ldm + c], c < nu: A_UU, c >= nu: B_U^T
  const int ldd = mr + 1;                        // odd column stride: Gram reads spread over banks
  double* Dn = M + (size_t)na * ldm;             // new dictionary, mr x na column-major, stride ldd
  double* diag0 = Dn + (size_t)ldd * na;
  int* U = reinterpret_cast<int*>(diag0 + na);
  int* nu_s = U + na;
  const double* A = sums;
  const double* B = sums + na * na;
  if (tid < kWave) {
    const bool used = tid < na && A[tid + na * tid] > 0.0;
    const unsigned long long mask = __ballot(used);
    const int nu = __popcll(mask);
    if (used) U[__popcll(mask & ((1ull << tid) - 1ull))] = tid;
    if (tid == 0) {
      *nu_s = nu;
      if (nu < na) atomicAdd(&counters[kCtrUnusedAtoms], (unsigned long long)(na - nu));
    }
  }
  for (int e = tid; e < mr * na; e += nt) Dn[e % mr + ldd * (e / mr)] = D[e];
  for (int i = tid; i < na; i += nt) w[i] = 1.0;
  __syncthreads();
  const int nu = *nu_s, ncol = nu + mr;
  for (int e = tid; e < nu * ncol; e += nt) {
    const int k = e / ncol, c = e % ncol;
    M[k * ldm + c] = c < nu ? A[U[k] + na * U[c]] : B[(c - nu) + mr * U[k]];
    if (c == k) diag0[k] = A[U[k] + na * U[k]];
  }
  __syncthreads();
  bool bad = false;
  // thread tid updates rows i = tid / kGJCols (+ multiples of nt / kGJCols) at columns
  // c = tid % kGJCols (+ multiples of kGJCols): no index division inside the steps
  constexpr int kGJCols = 32;
  const int ci = tid % kGJCols, ri = tid / kGJCols, rstep = nt / kGJCols;
  for (int k = 0; k < nu; ++k) {
    const double piv = M[k * ldm + k];
    if (!(piv > kSpdRelTol * diag0[k])) {  // same value in every thread: uniform exit
      bad = true;
      break;
    }
    const double inv = 1.0 / piv;
    for (int i = ri; i < nu; i += rstep) {
      if (i == k) continue;
      const double f = M[i * ldm + k] * inv;
      for (int c = k + 1 + ci; c < ncol; c += kGJCols) M[i * ldm + c] -= f * M[k * ldm + c];
    }
    __syncthreads();
  }
  if (!bad) {
    // row k now reads [pivot_k e_k | pivot_k * (D*^T)_k]: normalise each solved atom, one
    // thread per entry (k, p), each forming the atom's norm itself
    for (int e = tid; e < nu * mr; e += nt) {
      const int k = e / mr, p = e % mr;
      const double inv = 1.0 / M[k * ldm + k];
      double nrm = 0.0;
      for (int q = 0; q < mr; ++q) {
        const double v = M[k * ldm + nu + q] * inv;
        nrm += v * v;
      }
      nrm = sqrt(nrm);
      if (nrm > 0.0) {
        const int i = U[k];
        if (p == 0) w[i] = nrm;
        Dn[p + ldd * i] = (M[k * ldm + nu + p] * inv) / nrm;
      }
    }
  } else if (tid == 0) {
    atomicOr(status, kStatusSingular);
    atomicAdd(&counters[kCtrSingular], 1ull);
  }
  __syncthreads();
  for (int e = tid; e < mr * na; e += nt) {
    const double v = Dn[e % mr + ldd * (e / mr)];
    D[e] = v;
    Dc[e] = (T)v;
  }
  for (int e = tid; e < na * na; e += nt) {
    const int i = e % na, j = e / na;
    double v = 0.0;
    for (int p = 0; p < mr; ++p) v += Dn[p + ldd * i] * Dn[p + ldd * j];
    G64[e] = v;
    Gc[e] = (T)v;
  }
}

}  // namespace sdl
