// Device routines of the TMOD dictionary update shared by several kernels:
// the FP64 solve on the used atoms with normalisation (Corollary 1 / Proposition 1)
// and the refresh of the compute-type dictionary copy and Gram matrix.
#pragma once

#include "sdl_internal.h"

namespace sdl {

constexpr double kSpdRelTol = 1e-12;  // Cholesky pivot <= tol * diagonal entry -> not positive definite

__device__ inline void wave_fence_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// D (mr x na FP64) -> compute-type copy, FP64 and compute-type Gram D^T D; threads t0..t0+nt-1.
template <typename T>
__device__ void write_copies(const double* D, int mr, int na, T* Dc, double* G64, T* Gc, int t, int nt) {
  for (int e = t; e < mr * na; e += nt) Dc[e] = (T)D[e];
  for (int e = t; e < na * na; e += nt) {
    const int i = e % na, j = e / na;
    double v = 0.0;
    for (int p = 0; p < mr; ++p) v += D[p + mr * i] * D[p + mr * j];
    G64[e] = v;
    Gc[e] = (T)v;
  }
}

// LDS bytes the solve needs for na atoms and mr rows.
__host__ __device__ inline size_t solve_lds_bytes(int na, int mr) {
  return sizeof(double) * (2 * (size_t)na * (na + 1) + 2 * (size_t)na * (mr + 1) + na + (size_t)mr * na) +
         sizeof(int) * na + 16;
}

// One wavefront (lane = 0..63).  sums = [A (na x na) | B (mr x na)], column-major,
// A = the update's Gram sum, B = its right-hand side.  Atoms with A_ii = 0 are used by
// no code: the system decouples exactly and they keep their old value.  On the used
// set, D* A_UU = B_U is solved by FP64 Cholesky; each solved column is normalised
// (w_i = its norm; a zero column keeps the old atom).  A pivot below kSpdRelTol times
// its diagonal entry marks the sum as not positive definite: D is left unchanged and
// the singular status bit is set.  smem: solve_lds_bytes(na, mr) bytes.
template <typename T>
__device__ void solve_update(const double* sums, int mr, int na, double* D, T* Dc, double* G64, T* Gc, double* w,
                             int* status, unsigned long long* counters, unsigned char* smem, int lane) {
  const int ldc = na + 1, ldx = mr + 1;
  double* C = reinterpret_cast<double*>(smem);  // Schur complement being reduced
  double* Lf = C + (size_t)na * ldc;              // Cholesky factor, written once per column
  double* X = Lf + (size_t)na * ldc;              // X[k*ldx + p]: right-hand sides, atom k, row p
  double* Z = X + (size_t)na * ldx;               // finished rows of the triangular solves
  double* diag0 = Z + (size_t)na * ldx;
  double* Dn = diag0 + na;  // the new dictionary, mr x na column-major
  int* U = reinterpret_cast<int*>(Dn + (size_t)mr * na);
  const double* A = sums;
  const double* B = sums + na * na;
  const bool used = lane < na && A[lane + na * lane] > 0.0;
  const unsigned long long mask = __ballot(used);
  const int nu = __popcll(mask);
  if (used) U[__popcll(mask & ((1ull << lane) - 1ull))] = lane;
  if (lane == 0 && nu < na) atomicAdd(&counters[kCtrUnusedAtoms], (unsigned long long)(na - nu));
  wave_fence_sync();
  for (int e = lane; e < nu * nu; e += kWave) {
    const int k = e % nu, l = e / nu;
    C[k * ldc + l] = A[U[k] + na * U[l]];
    if (k == l) diag0[k] = C[k * ldc + k];
  }
  for (int e = lane; e < nu * mr; e += kWave) {
    const int k = e % nu, p = e / nu;
    X[k * ldx + p] = B[p + mr * U[k]];
  }
  wave_fence_sync();
  // Each elimination step reads only values finished in earlier steps and writes
  // different locations, so one wave synchronisation per step suffices.
  bool bad = false;
  for (int k = 0; k < nu; ++k) {
    const double d = C[k * ldc + k];
    if (!(d > kSpdRelTol * diag0[k])) {
      bad = true;
      break;
    }
    const double inv = 1.0 / sqrt(d);
    if (lane == 0) Lf[k * ldc + k] = sqrt(d);
    for (int i = k + 1 + lane; i < nu; i += kWave) Lf[i * ldc + k] = C[i * ldc + k] * inv;
    const int rem = nu - k - 1;
    const double inv2 = inv * inv;
    for (int e = lane; e < rem * rem; e += kWave) {
      const int i = k + 1 + e % rem, j = k + 1 + e / rem;
      if (j <= i) C[i * ldc + j] -= C[i * ldc + k] * C[j * ldc + k] * inv2;
    }
    wave_fence_sync();
  }
  if (!bad) {
    // L Z = X: row k of Z is X[k] / L_kk once rows < k have been eliminated from X[k]
    for (int k = 0; k < nu; ++k) {
      const double inv = 1.0 / Lf[k * ldc + k];
      for (int p = lane; p < mr; p += kWave) Z[k * ldx + p] = X[k * ldx + p] * inv;
      for (int e = lane; e < (nu - k - 1) * mr; e += kWave) {
        const int i = k + 1 + e / mr, p = e % mr;
        X[i * ldx + p] -= Lf[i * ldc + k] * (X[k * ldx + p] * inv);
      }
      wave_fence_sync();
    }
    // L^T X = Z, from the last row up; the solution goes to X
    for (int k = nu - 1; k >= 0; --k) {
      const double inv = 1.0 / Lf[k * ldc + k];
      for (int p = lane; p < mr; p += kWave) X[k * ldx + p] = Z[k * ldx + p] * inv;
      for (int e = lane; e < k * mr; e += kWave) {
        const int i = e / mr, p = e % mr;
        Z[i * ldx + p] -= Lf[k * ldc + i] * (Z[k * ldx + p] * inv);
      }
      wave_fence_sync();
    }
  }
  // new dictionary in LDS: solved atoms normalised (W), every other atom unchanged
  for (int e = lane; e < mr * na; e += kWave) Dn[e] = D[e];
  for (int i = lane; i < na; i += kWave) w[i] = 1.0;
  wave_fence_sync();
  if (!bad) {
    for (int k = lane; k < nu; k += kWave) {
      const int i = U[k];
      double nrm = 0.0;
      for (int p = 0; p < mr; ++p) nrm += X[k * ldx + p] * X[k * ldx + p];
      nrm = sqrt(nrm);
      if (nrm > 0.0) {
        w[i] = nrm;
        for (int p = 0; p < mr; ++p) Dn[p + mr * i] = X[k * ldx + p] / nrm;
      }
    }
  } else if (lane == 0) {
    atomicOr(status, kStatusSingular);
    atomicAdd(&counters[kCtrSingular], 1ull);
  }
  wave_fence_sync();
  // write back D, its compute-type copy and the Gram matrix D^T D (from LDS)
  for (int e = lane; e < mr * na; e += kWave) {
    D[e] = Dn[e];
    Dc[e] = (T)Dn[e];
  }
  for (int e = lane; e < na * na; e += kWave) {
    const int i = e % na, j = e / na;
    double v = 0.0;
    for (int p = 0; p < mr; ++p) v += Dn[p + mr * i] * Dn[p + mr * j];
    G64[e] = v;
    Gc[e] = (T)v;
  }
}

}  // namespace sdl
