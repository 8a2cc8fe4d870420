// Host side of the learned support proposal (C ABI in include/sdl.h).
//
// Network: x = vec(Y)/||Y||_F (m1*m2) -> GELU(W1 x + b1) (hidden) -> GELU(W2 . + b2)
// (hidden) -> W3 . + b3 (one logit per atom, n1*n2).  Trained with mean sigmoid
// cross-entropy against the multi-hot support that 2D-OMP chose, Adam on FP32 master
// weights, BF16 (or FP32 in the check mode) copies used by the matrix-core GEMMs.
// Inference: logits -> top-s atoms -> least squares -> accept if the residual passes
// the calibrated test, otherwise the signal goes to the 2D-OMP kernel.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include <hip/hip_bf16.h>

#include "mlp_internal.h"

using namespace sdl;

namespace sdl {
int abi_fail(int st, const char* msg);  // sets the thread's last error (sdl_abi.hip)
}

struct sdl_proposer {
  int m1, m2, n1, n2, H, M, A;
  int fp32;  // 1: FP32 check mode, 0: BF16 compute copies
  int64_t np;
  size_t elem;
  int64_t off[6];  // W1t, b1, W2t, b2, W3t, b3
  float* p = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* g = nullptr;
  void* pc = nullptr;
  int step = 0;
  int64_t cap = 0;  // batch capacity of the activation buffers
  void* X = nullptr;
  float* Z1 = nullptr;
  void* H1 = nullptr;
  float* Z2 = nullptr;
  void* H2 = nullptr;
  float* Z3 = nullptr;
  void* dZ3 = nullptr;
  void* dZ2 = nullptr;
  void* dZ1 = nullptr;
  double* loss_part = nullptr;
  double* loss = nullptr;
  int32_t* idx = nullptr;
  int64_t idx_cap = 0;
  // learned sparse coding workspace
  int64_t ncap = 0;
  int32_t* accept = nullptr;
  int32_t* list = nullptr;
  int32_t* blk = nullptr;
  int32_t* count = nullptr;
  float* Dc1 = nullptr;
  float* Dc2 = nullptr;
  float* G1c = nullptr;
  float* G2c = nullptr;
  double* G64 = nullptr;
  unsigned long long* ctr = nullptr;
};

namespace {

#define HT(expr)                                                                         \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return abi_fail(SDL_E_DEVICE, (std::string(#expr) + ": " + hipGetErrorString(e_)).c_str()); \
  } while (0)
#define ST(expr)                 \
  do {                           \
    int s_ = (expr);             \
    if (s_ != SDL_OK) return s_; \
  } while (0)

uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double unif(uint64_t key, uint64_t i) { return ((double)(splitmix64(key + i) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

template <typename F>
int dalloc(F** ptr, size_t n) {
  if (*ptr) {
    (void)hipFree(*ptr);
    *ptr = nullptr;
  }
  if (n == 0) n = 1;
  if (hipMalloc((void**)ptr, n * sizeof(F)) != hipSuccess) {
    *ptr = nullptr;
    return abi_fail(SDL_E_NOMEM, "device allocation failed");
  }
  return SDL_OK;
}

int ensure_batch(sdl_proposer* P, int64_t B) {
  if (B <= P->cap) return SDL_OK;
  const int64_t c = B;
  ST(dalloc((char**)&P->X, (size_t)c * P->M * P->elem));
  ST(dalloc(&P->Z1, (size_t)c * P->H));
  ST(dalloc((char**)&P->H1, (size_t)c * P->H * P->elem));
  ST(dalloc(&P->Z2, (size_t)c * P->H));
  ST(dalloc((char**)&P->H2, (size_t)c * P->H * P->elem));
  ST(dalloc(&P->Z3, (size_t)c * P->A));
  ST(dalloc((char**)&P->dZ3, (size_t)c * P->A * P->elem));
  ST(dalloc((char**)&P->dZ2, (size_t)c * P->H * P->elem));
  ST(dalloc((char**)&P->dZ1, (size_t)c * P->H * P->elem));
  ST(dalloc(&P->loss_part, (size_t)c));
  ST(dalloc(&P->loss, 1));
  P->cap = c;
  return SDL_OK;
}

template <typename T>
int gemm(const void* A, int opA, const void* B, int opB, void* C, int M, int N, int K, int lda, int ldb, int ldc, int epi,
         const float* bias, float* Z, hipStream_t st) {
  GemmArgs g{A, B, C, M, N, K, lda, ldb, ldc, epi, bias, Z};
  HT(launch_gemm<T>(g, opA, opB, st));
  return SDL_OK;
}

// logits of B signals (B % 64 == 0) whose normalised inputs are already in P->X
template <typename T>
int forward(sdl_proposer* P, int64_t B, bool keep, hipStream_t st) {
  const T* pc = (const T*)P->pc;
  const float* p = P->p;
  const int H = P->H, M = P->M, A = P->A;
  ST(gemm<T>(P->X, 0, pc + P->off[0], 1, P->H1, (int)B, H, M, M, M, H, kEpiBiasGelu, p + P->off[1], keep ? P->Z1 : nullptr, st));
  ST(gemm<T>(P->H1, 0, pc + P->off[2], 1, P->H2, (int)B, H, H, H, H, H, kEpiBiasGelu, p + P->off[3], keep ? P->Z2 : nullptr, st));
  ST(gemm<T>(P->H2, 0, pc + P->off[4], 1, P->Z3, (int)B, A, H, H, H, A, kEpiStoreF32, p + P->off[5], nullptr, st));
  return SDL_OK;
}

// gradient of the mean BCE into P->g for the batch rows idx (or 0..B-1), loss into P->loss
template <typename T>
int backward(sdl_proposer* P, const int32_t* supp, const int32_t* idx, int s, int64_t B, hipStream_t st) {
  const T* pc = (const T*)P->pc;
  const int H = P->H, M = P->M, A = P->A;
  float* g = P->g;
  HT(launch_bce_grad<T>(P->Z3, supp, idx, B, A, s, (T*)P->dZ3, P->loss_part, P->loss, st));
  // layer 3
  ST(gemm<T>(P->dZ3, 1, P->H2, 0, g + P->off[4], A, H, (int)B, A, H, H, kEpiStoreF32, nullptr, nullptr, st));
  HT(launch_bias_grad<T>((const T*)P->dZ3, B, A, g + P->off[5], st));
  ST(gemm<T>(P->dZ3, 0, pc + P->off[4], 0, P->dZ2, (int)B, H, A, A, H, H, kEpiGeluGrad, nullptr, P->Z2, st));
  // layer 2
  ST(gemm<T>(P->dZ2, 1, P->H1, 0, g + P->off[2], H, H, (int)B, H, H, H, kEpiStoreF32, nullptr, nullptr, st));
  HT(launch_bias_grad<T>((const T*)P->dZ2, B, H, g + P->off[3], st));
  ST(gemm<T>(P->dZ2, 0, pc + P->off[2], 0, P->dZ1, (int)B, H, H, H, H, H, kEpiGeluGrad, nullptr, P->Z1, st));
  // layer 1
  ST(gemm<T>(P->dZ1, 1, P->X, 0, g + P->off[0], H, M, (int)B, H, M, M, kEpiStoreF32, nullptr, nullptr, st));
  HT(launch_bias_grad<T>((const T*)P->dZ1, B, H, g + P->off[1], st));
  return SDL_OK;
}

template <typename T>
int train_step(sdl_proposer* P, const float* Y, const int32_t* supp, const int32_t* idx, int s, int64_t B, float lr,
               hipStream_t st) {
  HT(launch_prep_input<T>(Y, idx, B, P->M, (T*)P->X, nullptr, st));
  ST(forward<T>(P, B, true, st));
  ST(backward<T>(P, supp, idx, s, B, st));
  P->step += 1;
  HT(launch_adam<T>(P->p, P->m, P->v, P->g, (T*)P->pc, P->np, lr, P->step, st));
  return SDL_OK;
}

int copy_params(sdl_proposer* P, hipStream_t st) {
  if (P->fp32)
    HT(launch_copy_params<float>(P->p, (float*)P->pc, P->np, st));
  else
    HT(launch_copy_params<__bf16>(P->p, (__bf16*)P->pc, P->np, st));
  return SDL_OK;
}

int check_shape(const sdl_proposer* P, int32_t s) {
  if (s < 1 || s > 16) return abi_fail(SDL_E_SHAPE, "proposal supports 1 <= s <= 16");
  (void)P;
  return SDL_OK;
}

}  // namespace

extern "C" {

int sdl_proposer_create(int32_t m1, int32_t m2, int32_t n1, int32_t n2, int32_t hidden, int32_t fp32_check,
                        uint64_t seed, sdl_proposer** out) {
  if (!out) return abi_fail(SDL_E_INVAL, "out is NULL");
  *out = nullptr;
  if (m1 <= 0 || m2 <= 0 || n1 <= 0 || n2 <= 0 || hidden <= 0)
    return abi_fail(SDL_E_SHAPE, "sizes must be positive");
  const int M = m1 * m2, A = n1 * n2;
  if (M % 64 || A % 64 || hidden % 64 || M > 64)
    return abi_fail(SDL_E_UNSUPPORTED, "the proposal network needs m1*m2 = 64, n1*n2 and hidden multiples of 64");
  if (!propose_supported(n1, n2, 1)) return abi_fail(SDL_E_UNSUPPORTED, "no proposal kernel for this atom count");
  sdl_proposer* P = new sdl_proposer();
  P->m1 = m1; P->m2 = m2; P->n1 = n1; P->n2 = n2; P->H = hidden; P->M = M; P->A = A;
  P->fp32 = fp32_check ? 1 : 0;
  P->elem = P->fp32 ? 4 : 2;
  const int64_t H = hidden;
  P->off[0] = 0;
  P->off[1] = P->off[0] + H * M;
  P->off[2] = P->off[1] + H;
  P->off[3] = P->off[2] + H * H;
  P->off[4] = P->off[3] + H;
  P->off[5] = P->off[4] + (int64_t)A * H;
  P->np = P->off[5] + A;
  int st = SDL_OK;
  if (st == SDL_OK) st = dalloc(&P->p, P->np);
  if (st == SDL_OK) st = dalloc(&P->m, P->np);
  if (st == SDL_OK) st = dalloc(&P->v, P->np);
  if (st == SDL_OK) st = dalloc(&P->g, P->np);
  if (st == SDL_OK) st = dalloc((char**)&P->pc, (size_t)P->np * P->elem);
  if (st != SDL_OK) {
    sdl_proposer_destroy(P);
    return st;
  }
  // seeded Kaiming-normal weights (fan-in), zero biases; counter-based (stream 7)
  std::vector<float> h(P->np, 0.f);
  const uint64_t key = splitmix64(seed * 256 + 7);
  const int64_t fan[3] = {M, H, H}, rows[3] = {H, H, A};
  for (int l = 0; l < 3; ++l) {
    const double sd = std::sqrt(2.0 / (double)fan[l]);
    const int64_t o = P->off[2 * l], n = rows[l] * fan[l];
    for (int64_t i = 0; i < n; ++i) {
      const uint64_t c = (uint64_t)(o + i);
      const double u1 = unif(key, 2 * c), u2 = unif(key, 2 * c + 1);
      h[o + i] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
    }
  }
  st = sdl_proposer_set_params(P, h.data());
  if (st != SDL_OK) {
    sdl_proposer_destroy(P);
    return st;
  }
  *out = P;
  return SDL_OK;
}

void sdl_proposer_destroy(sdl_proposer* P) {
  if (!P) return;
  void* bufs[] = {P->p, P->m, P->v, P->g, P->pc, P->X, P->Z1, P->H1, P->Z2, P->H2, P->Z3, P->dZ3, P->dZ2, P->dZ1,
                  P->loss_part, P->loss, P->idx, P->accept, P->list, P->blk, P->count, P->Dc1, P->Dc2, P->G1c,
                  P->G2c, P->G64, P->ctr};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  delete P;
}

int64_t sdl_proposer_num_params(const sdl_proposer* P) { return P ? P->np : -1; }

int sdl_proposer_get_params(const sdl_proposer* P, float* host) {
  if (!P || !host) return abi_fail(SDL_E_INVAL, "NULL argument");
  HT(hipDeviceSynchronize());
  HT(hipMemcpy(host, P->p, sizeof(float) * P->np, hipMemcpyDeviceToHost));
  return SDL_OK;
}

int sdl_proposer_set_params(sdl_proposer* P, const float* host) {
  if (!P || !host) return abi_fail(SDL_E_INVAL, "NULL argument");
  HT(hipDeviceSynchronize());
  HT(hipMemcpy(P->p, host, sizeof(float) * P->np, hipMemcpyHostToDevice));
  HT(hipMemset(P->m, 0, sizeof(float) * P->np));
  HT(hipMemset(P->v, 0, sizeof(float) * P->np));
  P->step = 0;
  ST(copy_params(P, nullptr));
  HT(hipDeviceSynchronize());
  return SDL_OK;
}

int sdl_proposer_gradient(sdl_proposer* P, const float* Y, const int32_t* supp, int32_t s, int64_t B, float* grad_host,
                          double* loss_host, void* stream) {
  if (!P || !Y || !supp) return abi_fail(SDL_E_INVAL, "NULL argument");
  ST(check_shape(P, s));
  if (B <= 0 || B % 64) return abi_fail(SDL_E_SHAPE, "batch must be a positive multiple of 64");
  hipStream_t st = (hipStream_t)stream;
  ST(ensure_batch(P, B));
  if (P->fp32) {
    HT(launch_prep_input<float>(Y, nullptr, B, P->M, (float*)P->X, nullptr, st));
    ST(forward<float>(P, B, true, st));
    ST(backward<float>(P, supp, nullptr, s, B, st));
  } else {
    HT(launch_prep_input<__bf16>(Y, nullptr, B, P->M, (__bf16*)P->X, nullptr, st));
    ST(forward<__bf16>(P, B, true, st));
    ST(backward<__bf16>(P, supp, nullptr, s, B, st));
  }
  HT(hipStreamSynchronize(st));
  if (grad_host) HT(hipMemcpy(grad_host, P->g, sizeof(float) * P->np, hipMemcpyDeviceToHost));
  if (loss_host) HT(hipMemcpy(loss_host, P->loss, sizeof(double), hipMemcpyDeviceToHost));
  return SDL_OK;
}

int sdl_proposer_train(sdl_proposer* P, const float* Y, const int32_t* supp, int32_t s, int64_t N, int32_t epochs,
                       int32_t batch, float lr, uint64_t seed, double* loss_trace, void* stream) {
  if (!P || !Y || !supp) return abi_fail(SDL_E_INVAL, "NULL argument");
  ST(check_shape(P, s));
  if (batch <= 0 || batch % 64 || N < batch || epochs < 0) return abi_fail(SDL_E_SHAPE, "need N >= batch, batch % 64 == 0");
  if (N > INT32_MAX) return abi_fail(SDL_E_SHAPE, "N > 2^31 - 1 (batch indices are 32-bit)");
  hipStream_t st = (hipStream_t)stream;
  ST(ensure_batch(P, batch));
  if (P->idx_cap < N) {
    ST(dalloc(&P->idx, (size_t)N));
    P->idx_cap = N;
  }
  std::vector<int32_t> perm(N);
  const int64_t nb = N / batch;  // full batches per epoch
  std::vector<double> ep_loss;
  double* dloss = nullptr;
  ST(dalloc(&dloss, (size_t)(nb > 0 ? nb : 1)));
  struct FreeOnExit {  // per-batch losses, released on every return path
    double* p;
    ~FreeOnExit() { (void)hipFree(p); }
  } dloss_guard{dloss};
  for (int ep = 0; ep < epochs; ++ep) {
    // batch order: Fisher-Yates with a counter-based generator (stream 8)
    for (int64_t i = 0; i < N; ++i) perm[i] = (int32_t)i;
    const uint64_t key = splitmix64(seed * 256 + 8) + (uint64_t)ep * 0x100000000ull;
    for (int64_t i = N - 1; i > 0; --i) {
      const int64_t j = (int64_t)(unif(key, (uint64_t)i) * (double)(i + 1));
      std::swap(perm[i], perm[j < i ? j : i]);
    }
    HT(hipMemcpyAsync(P->idx, perm.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, st));
    for (int64_t b = 0; b < nb; ++b) {
      const int32_t* bidx = P->idx + b * batch;
      if (P->fp32)
        ST(train_step<float>(P, Y, supp, bidx, s, batch, lr, st));
      else
        ST(train_step<__bf16>(P, Y, supp, bidx, s, batch, lr, st));
      HT(hipMemcpyAsync(dloss + b, P->loss, sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    HT(hipStreamSynchronize(st));
    if (loss_trace) {
      std::vector<double> h(nb);
      HT(hipMemcpy(h.data(), dloss, sizeof(double) * nb, hipMemcpyDeviceToHost));
      double acc = 0.0;
      for (double x : h) acc += x;
      loss_trace[ep] = nb > 0 ? acc / nb : 0.0;
    }
  }
  return SDL_OK;
}

// File layout: 8-byte magic, six int32 (m1, m2, n1, n2, hidden, fp32_check), int64 parameter
// count, then the FP32 master weights (host byte order; little-endian on the hosts this runs on).
static const char kPropMagic[8] = {'S', 'D', 'L', 'P', 'R', 'O', 'P', '1'};

int sdl_proposer_save(const sdl_proposer* P, const char* path) {
  if (!P || !path) return abi_fail(SDL_E_INVAL, "NULL argument");
  std::vector<float> h((size_t)P->np);
  ST(sdl_proposer_get_params(P, h.data()));
  FILE* f = fopen(path, "wb");
  if (!f) return abi_fail(SDL_E_INVAL, "cannot open the file for writing");
  const int32_t dims[6] = {P->m1, P->m2, P->n1, P->n2, P->H, P->fp32};
  const int64_t np = P->np;
  bool ok = fwrite(kPropMagic, 1, 8, f) == 8 && fwrite(dims, sizeof(int32_t), 6, f) == 6 &&
            fwrite(&np, sizeof(int64_t), 1, f) == 1 && fwrite(h.data(), sizeof(float), h.size(), f) == h.size();
  ok = (fclose(f) == 0) && ok;
  return ok ? SDL_OK : abi_fail(SDL_E_INVAL, "writing the file failed");
}

int sdl_proposer_load(const char* path, sdl_proposer** out) {
  if (!path || !out) return abi_fail(SDL_E_INVAL, "NULL argument");
  *out = nullptr;
  FILE* f = fopen(path, "rb");
  if (!f) return abi_fail(SDL_E_INVAL, "cannot open the file for reading");
  char magic[8];
  int32_t dims[6];
  int64_t np = 0;
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kPropMagic, 8) == 0 &&
            fread(dims, sizeof(int32_t), 6, f) == 6 && fread(&np, sizeof(int64_t), 1, f) == 1;
  sdl_proposer* P = nullptr;
  if (ok && sdl_proposer_create(dims[0], dims[1], dims[2], dims[3], dims[4], dims[5], 0, &P) != SDL_OK) {
    fclose(f);
    return SDL_E_INVAL;  // message set by sdl_proposer_create
  }
  ok = ok && P->np == np;
  std::vector<float> h(ok ? (size_t)np : 0);
  ok = ok && fread(h.data(), sizeof(float), h.size(), f) == h.size();
  char extra;
  ok = ok && fread(&extra, 1, 1, f) == 0;  // nothing after the weights
  fclose(f);
  if (!ok) {
    if (P) sdl_proposer_destroy(P);
    return abi_fail(SDL_E_INVAL, "not a proposer file written by sdl_proposer_save");
  }
  const int st = sdl_proposer_set_params(P, h.data());
  if (st != SDL_OK) {
    sdl_proposer_destroy(P);
    return st;
  }
  *out = P;
  return SDL_OK;
}

int sdl_proposer_logits(sdl_proposer* P, const float* Y, int64_t N, float* logits, void* stream) {
  if (!P || !Y || !logits) return abi_fail(SDL_E_INVAL, "NULL argument");
  if (N < 0) return abi_fail(SDL_E_INVAL, "N < 0");
  hipStream_t st = (hipStream_t)stream;
  const int64_t chunk = 65536;
  ST(ensure_batch(P, chunk));
  for (int64_t k0 = 0; k0 < N; k0 += chunk) {
    const int64_t n = std::min(chunk, N - k0);
    const int64_t B = (n + 63) / 64 * 64;
    if (P->fp32) {
      HT(launch_prep_input<float>(Y + k0 * P->M, nullptr, n, P->M, (float*)P->X, nullptr, st));
      ST(forward<float>(P, B, false, st));
    } else {
      HT(launch_prep_input<__bf16>(Y + k0 * P->M, nullptr, n, P->M, (__bf16*)P->X, nullptr, st));
      ST(forward<__bf16>(P, B, false, st));
    }
    HT(hipMemcpyAsync(logits + k0 * P->A, P->Z3, sizeof(float) * n * P->A, hipMemcpyDeviceToDevice, st));
  }
  return SDL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- learned sparse coding

namespace sdl {

int learned_prepare(sdl_proposer* P, int64_t N) {
  if (N > P->ncap) {
    ST(dalloc(&P->accept, (size_t)N));
    ST(dalloc(&P->list, (size_t)N));
    ST(dalloc(&P->blk, (size_t)compact_blocks(N) + 1));
    ST(dalloc(&P->count, 1));
    P->ncap = N;
  }
  return ensure_batch(P, 65536);
}

// Proposal + least squares for all signals, then the register-resident 2D-OMP on the
// rejected ones (gathered by index).  Needs the FP32 copies of D and the Grams: they are
// computed here from the FP64 dictionaries.  Writes accept[] (1 = proposal kept).
// counters[kCtrProposed] += n, counters[kCtrFallback] += *count (one thread; graph-capturable)
__global__ void count_fallbacks_kernel(const int32_t* count, int64_t n, unsigned long long* counters) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    counters[kCtrProposed] += (unsigned long long)n;
    counters[kCtrFallback] += (unsigned long long)*count;
  }
}

int learned_code(sdl_proposer* P, const sdl_problem& r, double tau, int32_t* accept_out, const OmpArgs<float>& omp,
                 hipStream_t st, int64_t* nfallback_host) {
  ST(learned_prepare(P, r.N));
  int32_t* accept = accept_out ? accept_out : P->accept;
  const int64_t chunk = 65536;
  ST(ensure_batch(P, chunk));
  const float* Y = (const float*)r.Y;
  for (int64_t k0 = 0; k0 < r.N; k0 += chunk) {
    const int64_t n = std::min(chunk, r.N - k0);
    const int64_t B = (n + 63) / 64 * 64;
    if (P->fp32) {
      HT(launch_prep_input<float>(Y + k0 * P->M, nullptr, n, P->M, (float*)P->X, nullptr, st));
      ST(forward<float>(P, B, false, st));
    } else {
      HT(launch_prep_input<__bf16>(Y + k0 * P->M, nullptr, n, P->M, (__bf16*)P->X, nullptr, st));
      ST(forward<__bf16>(P, B, false, st));
    }
    ProposeArgs pa;
    pa.m1 = r.m1; pa.m2 = r.m2; pa.n1 = r.n1; pa.n2 = r.n2; pa.s = r.s; pa.N = n;
    pa.logits = P->Z3;
    pa.Y = Y + k0 * P->M;
    pa.D1 = omp.D1; pa.D2 = omp.D2; pa.G1 = omp.G1; pa.G2 = omp.G2;
    pa.supp = r.supp + k0 * r.s;
    pa.coef = (float*)r.coef + k0 * r.s;
    pa.res2 = r.res2 ? (float*)r.res2 + k0 : nullptr;
    pa.accept = accept + k0;
    pa.tau = tau;
    HT(launch_propose(pa, st));
  }
  HT(launch_compact_rejected(accept, r.N, P->blk, P->list, P->count, st));
  OmpArgs<float> a = omp;
  a.index = P->list;
  a.count = P->count;
  HT(launch_omp_fast<float>(a, st));
  if (omp.counters) {
    hipLaunchKernelGGL(count_fallbacks_kernel, dim3(1), dim3(64), 0, st, (const int32_t*)P->count, r.N, omp.counters);
    HT(hipGetLastError());
  }
  if (nfallback_host) {
    int32_t c = 0;
    HT(hipMemcpyAsync(&c, P->count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HT(hipStreamSynchronize(st));
    *nfallback_host = c;
  }
  return SDL_OK;
}

bool proposer_matches(const sdl_proposer* P, const sdl_problem& r) {
  return P && P->m1 == r.m1 && P->m2 == r.m2 && P->n1 == r.n1 && P->n2 == r.n2;
}

}  // namespace sdl
