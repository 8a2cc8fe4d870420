// Host side of the C ABI declared in include/sdl.h: argument validation,
// workspace, launch sequencing (Algorithm 1), HIP graph replay and timing.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "mlp_internal.h"
#include "sdl_internal.h"

using namespace sdl;

namespace sdl {
int learned_code(sdl_proposer* P, const sdl_problem& r, double tau, int32_t* accept_out, const OmpArgs<float>& omp,
                 hipStream_t st, int64_t* nfallback_host);
bool proposer_matches(const sdl_proposer* P, const sdl_problem& r);
int learned_prepare(sdl_proposer* P, int64_t N);
}  // namespace sdl

namespace {

thread_local std::string g_err;

int fail(int st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(SDL_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------------ per-stream context

struct Ctx {
  int device = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t side = nullptr;  // internal stream for graph replay (default priority)
  std::vector<hipEvent_t> ev;  // timing events
  hipEvent_t join_a = nullptr, join_b = nullptr;
  // graph branches for the problems of one call (default priority, created on first use)
  std::vector<hipStream_t> branch;
  std::vector<hipEvent_t> branch_join;
  hipEvent_t fork = nullptr;
  // the last instantiated learning graph and what it was captured for (see graph_key)
  std::vector<unsigned char> gkey;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
};

// Problems of one sdl_learn call run as parallel branches of the captured graph (at
// most this many streams; problems beyond it share branches round-robin).
constexpr int kMaxBranches = 8;
// Algorithm 1 iterations captured per graph (replayed K / this times; the remainder
// is launched directly).
constexpr int kItersPerGraph = 4;

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Ctx*> g_ctx;

int get_ctx(hipStream_t st, Ctx** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(dev, st);
  auto it = g_ctx.find(key);
  if (it == g_ctx.end()) {
    Ctx* c = new Ctx();
    c->device = dev;
    hipError_t e = omp_generic_init_device();
    if (e == hipSuccess) e = tmod_sums_init_device();
    if (e == hipSuccess) e = tmod_solve_init_device();
    if (e == hipSuccess) e = omp_fast_init_device();
    if (e == hipSuccess) e = tmod_sums_bf16_init_device();
    if (e == hipSuccess) e = ortho_init_device();
    if (e == hipSuccess) e = tensor_init_device();
    if (e == hipSuccess) e = denoise_init_device();
    if (e != hipSuccess) {
      delete c;
      return fail(SDL_E_DEVICE, "kernel attribute setup: %s", hipGetErrorString(e));
    }
    it = g_ctx.emplace(key, c).first;
  }
  *out = it->second;
  return SDL_OK;
}

int ensure_ws(Ctx* c, size_t bytes, hipStream_t st) {
  if (c->ws_bytes >= bytes) return SDL_OK;
  if (c->ws) {
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipFree(c->ws));
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  size_t n = bytes + bytes / 4 + 4096;
  if (hipMalloc(&c->ws, n) != hipSuccess) {
    c->ws = nullptr;
    return fail(SDL_E_NOMEM, "workspace allocation of %zu bytes failed", n);
  }
  c->ws_bytes = n;
  return SDL_OK;
}

// bump allocator over the workspace
struct Bump {
  char* base;
  size_t off = 0;
  explicit Bump(void* b) : base((char*)b) {}
  template <typename T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? (T*)(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

#define SDL_TRY_WS(expr)         \
  do {                           \
    int s_ = (expr);             \
    if (s_ != SDL_OK) return s_; \
  } while (0)

// ------------------------------------------------------------------ options / validation

struct Opt {
  int prec, schedule, use_graph, check_finite, timing, kernel;
  double stop_rel, dep_eps, pivot_fp64;
  sdl_stats* stats;
  sdl_proposer* proposer;
  double tau;
  double err2;
  double tie_band, fallback_margin;
  int deterministic, reserved0;
  void* workspace;
  size_t workspace_bytes;
  int method, reserved1;
};

Opt resolve(const sdl_options* o) {
  sdl_options d;
  sdl_default_options(&d);
  if (!o) o = &d;
  Opt r;
  r.prec = o->prec;
  r.schedule = o->schedule;
  r.use_graph = o->use_graph;
  r.check_finite = o->check_finite;
  r.timing = o->timing;
  r.kernel = o->kernel;
  r.stop_rel = o->stop_rel >= 0 ? o->stop_rel : (o->prec == SDL_FP64 ? 1e-14 : 1e-6);
  r.dep_eps = o->dep_eps >= 0 ? o->dep_eps : 1e-10;
  r.pivot_fp64 = o->pivot_fp64 >= 0 ? o->pivot_fp64 : 1e-3;
  r.stats = o->stats;
  r.proposer = o->proposer;
  r.tau = o->tau;
  r.err2 = o->err2;
  r.tie_band = o->tie_band;
  r.fallback_margin = o->fallback_margin;
  r.deterministic = o->deterministic;
  r.reserved0 = o->reserved0;
  r.workspace = o->workspace;
  r.workspace_bytes = o->workspace_bytes;
  r.method = o->method;
  r.reserved1 = o->reserved1;
  return r;
}

// Workspace of one call: the caller's (sdl_options.workspace) or the context's own, grown on demand.
int acquire_ws(Ctx* c, const Opt& o, size_t bytes, hipStream_t st, void** base) {
  if (o.workspace) {
    if ((uintptr_t)o.workspace % 256 != 0) return fail(SDL_E_INVAL, "workspace must be 256-byte aligned");
    if (o.workspace_bytes < bytes)
      return fail(SDL_E_NOMEM, "workspace of %zu bytes given, %zu needed", o.workspace_bytes, bytes);
    *base = o.workspace;
    return SDL_OK;
  }
  SDL_TRY_WS(ensure_ws(c, bytes, st));
  *base = c->ws;
  return SDL_OK;
}

int validate(const sdl_problem* p, int32_t nprob, const Opt& o, bool need_codes_in) {
  if (nprob < 0) return fail(SDL_E_INVAL, "nprob = %d < 0", nprob);
  if (nprob > 0 && !p) return fail(SDL_E_INVAL, "problem array is NULL");
  if (o.prec != SDL_FP64 && o.prec != SDL_FP32 && o.prec != SDL_BF16 && o.prec != SDL_MIXED_BF16)
    return fail(SDL_E_INVAL, "prec = %d is not an sdl_prec", o.prec);
  if (o.schedule != 0 && o.schedule != 1) return fail(SDL_E_INVAL, "schedule = %d (0 or 1)", o.schedule);
  if (o.kernel < 0 || o.kernel > 3) return fail(SDL_E_INVAL, "kernel = %d (0..3)", o.kernel);
  if (!(o.err2 >= 0.0)) return fail(SDL_E_INVAL, "err2 must be >= 0 (0: off)");
  if (!(o.tie_band >= 0.0 && o.tie_band < 0.5)) return fail(SDL_E_INVAL, "tie_band must be in [0, 0.5)");
  if (!(o.fallback_margin >= 1.0)) return fail(SDL_E_INVAL, "fallback_margin must be >= 1");
  if (o.deterministic != 0 && o.deterministic != 1) return fail(SDL_E_INVAL, "deterministic must be 0 or 1");
  if (o.reserved0 != 0) return fail(SDL_E_INVAL, "reserved0 must be 0");
  if (o.workspace && o.workspace_bytes == 0) return fail(SDL_E_INVAL, "workspace given with workspace_bytes = 0");
  if (o.method != 0 && o.method != 1) return fail(SDL_E_INVAL, "method = %d (0 or 1)", o.method);
  if (o.reserved1 != 0) return fail(SDL_E_INVAL, "reserved1 must be 0");
  if (o.method == 1) {
    if (o.prec != SDL_FP64 && o.prec != SDL_FP32)
      return fail(SDL_E_UNSUPPORTED, "the orthonormal variant runs in SDL_FP64 or SDL_FP32");
    if (o.err2 > 0.0 || o.proposer || o.schedule != 0)
      return fail(SDL_E_UNSUPPORTED, "the orthonormal variant has no error-driven stop, proposer or other schedule");
  }
  if (o.err2 > 0.0 && o.kernel == 2)
    return fail(SDL_E_UNSUPPORTED, "the error-driven stop does not run on the multi-signal kernels (kernel 2)");
  const size_t elem = o.prec == SDL_FP64 ? 8 : 4;
  for (int q = 0; q < nprob; ++q) {
    const sdl_problem& r = p[q];
    if (r.m1 <= 0 || r.m2 <= 0 || r.n1 <= 0 || r.n2 <= 0 || r.s <= 0)
      return fail(SDL_E_SHAPE, "problem %d: sizes must be positive (m1=%d m2=%d n1=%d n2=%d s=%d)", q, r.m1, r.m2,
                  r.n1, r.n2, r.s);
    if (r.N < 0) return fail(SDL_E_INVAL, "problem %d: N = %lld < 0", q, (long long)r.N);
    if (r.reserved != 0) return fail(SDL_E_INVAL, "problem %d: reserved field must be 0", q);
    if ((int64_t)r.s > (int64_t)r.n1 * r.n2 || (int64_t)r.s > (int64_t)r.m1 * r.m2)
      return fail(SDL_E_SHAPE, "problem %d: s = %d exceeds n1*n2 = %d or m1*m2 = %d", q, r.s, r.n1 * r.n2,
                  r.m1 * r.m2);
    if (r.m1 > SDL_MAX_M || r.m2 > SDL_MAX_M || r.n1 > SDL_MAX_N || r.n2 > SDL_MAX_N || r.s > SDL_MAX_S)
      return fail(SDL_E_SHAPE, "problem %d: sizes exceed the limits m <= %d, n <= %d, s <= %d", q, SDL_MAX_M,
                  SDL_MAX_N, SDL_MAX_S);
    if (!r.D1 || !r.D2) return fail(SDL_E_INVAL, "problem %d: D1/D2 is NULL", q);
    if (r.N > 0 && (!r.Y || !r.supp || !r.coef)) return fail(SDL_E_INVAL, "problem %d: Y/supp/coef is NULL", q);
    (void)need_codes_in;
    if (o.method == 1 && !ortho_supported(r.m1, r.m2, r.n1, r.n2, r.s))
      return fail(SDL_E_SHAPE, "problem %d: the orthonormal variant needs n1 = m1, n2 = m2, m1, m2 <= %d, m1*m2 <= 256",
                  q, SDL_ORTHO_MAX_N);
    if (o.prec == SDL_MIXED_BF16 && !omp_mixed_supported(r.m1, r.m2, r.n1, r.n2, r.s))
      return fail(SDL_E_UNSUPPORTED, "problem %d: no SDL_MIXED_BF16 kernel for m=%dx%d n=%dx%d s=%d", q, r.m1, r.m2,
                  r.n1, r.n2, r.s);
    if (o.err2 > 0.0 && o.kernel == 3 &&
        (!omp_wave_supported(r.m1, r.m2, r.n1, r.n2, r.s) ||
         (o.prec != SDL_FP64 && omp_quad_supported(r.m1, r.m2, r.n1, r.n2, r.s))))
      return fail(SDL_E_UNSUPPORTED, "problem %d: no one-wave-per-signal kernel with the error-driven stop for this shape",
                  q);
    if (o.prec == SDL_MIXED_BF16 && (o.err2 > 0.0 || o.proposer))
      return fail(SDL_E_UNSUPPORTED, "SDL_MIXED_BF16 runs plain 2D-OMP (no error-driven stop, no proposer)");
    if (omp_generic_lds_bytes(r.m1, r.m2, r.n1, r.n2, r.s, elem) > 160 * 1024)
      return fail(SDL_E_UNSUPPORTED, "problem %d: working set of one signal exceeds the 160 KiB LDS", q);
  }
  return SDL_OK;
}

// ------------------------------------------------------------------ per-problem buffers

struct PBuf {
  void* Dc1;  // compute-type copies
  void* Dc2;
  double* G1_64;
  double* G2_64;
  void* G1c;
  void* G2c;
  double* part;   // workgroup / wave partial rows of the TMOD sums
  double* stage;  // first-stage reduction rows
  double* sums;   // reduced [A | B | sum res2]
  double* w;
  double* rpart;
  int nblk, rblk, nent;
};

struct Plan {
  std::vector<PBuf> pb;
  int* status;
  unsigned long long* counters;
  int* iter;     // per-problem RMSE counters
  bool ybf16 = false;  // signals are bfloat16 (SDL_BF16, SDL_MIXED_BF16)
  double* trace; // device trace
  size_t bytes;
};

// Lay out the workspace; with base == nullptr only measures.  codes_only: only what sparse
// coding alone uses (no partial-sum, reduction or RMSE buffers).
void layout(const sdl_problem* p, int nprob, size_t elem, int K, void* base, Plan* pl, bool codes_only = false) {
  Bump b(base);
  pl->pb.resize(nprob);
  pl->status = b.take<int>(4);
  pl->counters = b.take<unsigned long long>(kNumCounters);
  pl->iter = b.take<int>(nprob > 0 ? nprob : 1);
  pl->trace = b.take<double>((size_t)(nprob > 0 ? nprob : 1) * (K + 1));
  for (int q = 0; q < nprob; ++q) {
    const sdl_problem& r = p[q];
    PBuf& x = pl->pb[q];
    x.Dc1 = b.take<char>(elem * r.m1 * r.n1);
    x.Dc2 = b.take<char>(elem * r.m2 * r.n2);
    x.G1_64 = b.take<double>((size_t)r.n1 * r.n1);
    x.G2_64 = b.take<double>((size_t)r.n2 * r.n2);
    x.G1c = b.take<char>(elem * r.n1 * r.n1);
    x.G2c = b.take<char>(elem * r.n2 * r.n2);
    if (codes_only) {
      x.part = x.stage = x.sums = x.w = x.rpart = nullptr;
      x.nblk = x.rblk = x.nent = 0;
      continue;
    }
    const int na = r.n1 > r.n2 ? r.n1 : r.n2, mr = r.m1 > r.m2 ? r.m1 : r.m2;
    x.nent = na * na + mr * na;
    const size_t ae = elem == 8 ? 8 : 4;  // arithmetic element size (BF16 signals compute in FP32)
    int nb1 = tmod_num_blocks_for(r.N, r.n1, r.m1, r.m2, r.s, r.n2, ae);
    int nb2 = tmod_num_blocks_for(r.N, r.n2, r.m2, r.m1, r.s, r.n1, ae);
    if (elem == 4 && tmod_sums_bf16_supported(r.m1, r.m2, r.n1, r.n2, r.s)) {
      const int b1 = tmod_bf16_num_blocks(r.N, r.n1, r.m1, r.m2, r.s, r.n2);
      const int b2 = tmod_bf16_num_blocks(r.N, r.n2, r.m2, r.m1, r.s, r.n1);
      nb1 = nb1 > b1 ? nb1 : b1;
      nb2 = nb2 > b2 ? nb2 : b2;
    }
    x.nblk = nb1 > nb2 ? nb1 : nb2;
    const int rows = x.nblk > omp_fast_max_partial_rows() ? x.nblk : omp_fast_max_partial_rows();
    x.rblk = rmse_num_blocks(r.N);
    x.part = b.take<double>((size_t)rows * (x.nent + 1));
    x.stage = b.take<double>((size_t)reduce_stage_rows(rows) * (x.nent + 1));
    x.sums = b.take<double>((size_t)x.nent + 1);
    x.w = b.take<double>((size_t)na);
    x.rpart = b.take<double>((size_t)x.rblk);
  }
  pl->bytes = b.off + 256;
}

// A caller-supplied workspace is checked against the call's layout before any device work.
int check_workspace(const sdl_problem* p, int nprob, int K, const Opt& o) {
  if (!o.workspace) return SDL_OK;
  Plan pl;
  layout(p, nprob, o.prec == SDL_FP64 ? 8 : 4, K, nullptr, &pl);
  if ((uintptr_t)o.workspace % 256 != 0) return fail(SDL_E_INVAL, "workspace must be 256-byte aligned");
  if (o.workspace_bytes < pl.bytes)
    return fail(SDL_E_NOMEM, "workspace of %zu bytes given, %zu needed", o.workspace_bytes, pl.bytes);
  return SDL_OK;
}

// ------------------------------------------------------------------ launch helpers

struct Launcher {
  hipStream_t st;
  bool timing;
  Ctx* ctx;
  std::vector<std::pair<int, int>>* marks;  // (class, event index of start)
  int next_ev = 0;

  int begin(int cls) {
    if (!timing) return SDL_OK;
    if ((size_t)next_ev + 2 > ctx->ev.size()) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        ctx->ev.push_back(e);
      }
    }
    HIP_TRY(hipEventRecord(ctx->ev[next_ev], st));
    marks->push_back({cls, next_ev});
    next_ev += 2;
    return SDL_OK;
  }
  int end() {
    if (!timing) return SDL_OK;
    HIP_TRY(hipEventRecord(ctx->ev[marks->back().second + 1], st));
    return SDL_OK;
  }
};

#define SDL_TRY(expr)            \
  do {                           \
    int s_ = (expr);             \
    if (s_ != SDL_OK) return s_; \
  } while (0)

template <typename T>
OmpArgs<T> omp_args(const sdl_problem& r, const PBuf& b, const Opt& o, const Plan& pl) {
  OmpArgs<T> a;
  a.m1 = r.m1; a.m2 = r.m2; a.n1 = r.n1; a.n2 = r.n2; a.s = r.s; a.N = r.N;
  a.Y = (const T*)r.Y;
  a.Yh = nullptr;
  if (pl.ybf16) {
    a.Yh = (const uint16_t*)r.Y;
    a.Y = nullptr;
  }
  a.D1 = (const T*)b.Dc1;
  a.D2 = (const T*)b.Dc2;
  a.G1 = (const T*)b.G1c;
  a.G2 = (const T*)b.G2c;
  a.supp = r.supp;
  a.coef = (T*)r.coef;
  a.res2 = (T*)r.res2;
  a.stop_rel = o.stop_rel;
  a.dep_eps = o.dep_eps;
  a.pivot_fp64 = o.pivot_fp64;
  a.err2 = o.err2;
  a.tie_band = o.tie_band;
  a.counters = pl.counters;
  a.sums_side = 0;
  a.sums_part = nullptr;
  a.index = nullptr;
  a.count = nullptr;
  return a;
}

template <typename T>
bool use_fast(const sdl_problem& r, const Opt& o) {
  if (o.prec == SDL_MIXED_BF16 || o.method == 1) return false;
  if (!omp_fast_supported<T>(r.m1, r.m2, r.n1, r.n2, r.s) || o.err2 > 0.0) return false;
  return o.kernel == 2 || (o.kernel == 0 && !wave_chosen(r.m1, r.m2, r.n1, r.n2, r.s));
}

// sums_side != 0 (register-resident path only): the sweep also writes the partial
// rows of that side's TMOD sums and of sum(res2) into b.part.
template <typename T>
int run_omp(const sdl_problem& r, const PBuf& b, const Opt& o, const Plan& pl, int sums_side, Launcher& L) {
  OmpArgs<T> a = omp_args<T>(r, b, o, pl);
  a.sums_side = sums_side;
  a.sums_part = b.part;
  if (o.method == 1) {
    if constexpr (sizeof(T) == 4) {
      if (ortho_mfma_supported(r.m1, r.m2, r.n1, r.n2, r.s)) {
        SDL_TRY(L.begin(0));
        HIP_TRY(launch_ortho_mfma(a, L.st));
        return L.end();
      }
    }
    if (sums_side != 0) return fail(SDL_E_UNSUPPORTED, "no fused sums for the orthonormal variant at this shape");
    SDL_TRY(L.begin(0));
    HIP_TRY(launch_ortho_code<T>(a, L.st));
    return L.end();
  }
  if constexpr (sizeof(T) == 4) {
    if (o.prec == SDL_MIXED_BF16) {
      if (sums_side != 0) return fail(SDL_E_UNSUPPORTED, "SDL_MIXED_BF16 has no fused sums");
      SDL_TRY(L.begin(0));
      HIP_TRY(launch_omp_mixed(a, L.st));
      return L.end();
    }
  }
  const bool fast = use_fast<T>(r, o);
  if (o.kernel == 2 && !fast)
    return fail(SDL_E_UNSUPPORTED, "no register-resident kernel for m=%dx%d n=%dx%d s=%d in this precision", r.m1,
                r.m2, r.n1, r.n2, r.s);
  // the error-driven stop runs on the one-wave-per-signal kernels (not on the quadrant kernel
  // that serves some FP32 shapes) and on the generic kernel
  bool wave = !fast && sums_side == 0 && (o.kernel == 0 || o.kernel == 3) &&
              omp_wave_supported(r.m1, r.m2, r.n1, r.n2, r.s);
  if (o.err2 > 0.0 && sizeof(T) == 4 && omp_quad_supported(r.m1, r.m2, r.n1, r.n2, r.s)) wave = false;
  if (o.kernel == 3 && !wave)
    return fail(SDL_E_UNSUPPORTED, "no one-wave-per-signal kernel for m=%dx%d n=%dx%d s=%d", r.m1, r.m2, r.n1, r.n2,
                r.s);
  SDL_TRY(L.begin(0));
  HIP_TRY(fast ? launch_omp_fast<T>(a, L.st) : wave ? launch_omp_wave<T>(a, L.st) : launch_omp_generic<T>(a, L.st));
  return L.end();
}

template <typename T>
int run_prep(const sdl_problem& r, const PBuf& b, Launcher& L) {
  SDL_TRY(L.begin(4));
  HIP_TRY(launch_dict_prep<T>(r.D1, r.m1, r.n1, (T*)b.Dc1, b.G1_64, (T*)b.G1c, L.st));
  HIP_TRY(launch_dict_prep<T>(r.D2, r.m2, r.n2, (T*)b.Dc2, b.G2_64, (T*)b.G2c, L.st));
  return L.end();
}

// reduce the partial rows of one side's sums (plus the res2 entry when fused) and solve;
// rmse_q >= 0: also record the RMSE of the sweep that produced the codes for problem rmse_q
template <typename T>
int run_reduce_solve(int side, const sdl_problem& r, const PBuf& b, const Plan& pl, int rows, bool with_res2,
                     int rmse_q, int K, Launcher& L, int method = 0) {
  const int na = side == 1 ? r.n1 : r.n2, mr = side == 1 ? r.m1 : r.m2;
  const int nent = na * na + mr * na;
  const int ld = nent + (with_res2 ? 1 : 0);
  const double* src = nullptr;
  int nrow = rows;
  if (rows > 0) {
    SDL_TRY(L.begin(2));
    hipError_t e;
    nrow = launch_reduce_stage1(b.part, rows, ld, b.stage, &src, L.st, &e);
    HIP_TRY(e);
    SDL_TRY(L.end());
  }
  if (method == 1) {
    // Remark 1: the orthogonal Procrustes update from the B block of the reduced sums
    SDL_TRY(L.begin(3));
    if (side == 1)
      HIP_TRY(launch_procrustes<T>(src, nrow, ld, r.n1, r.D1, (T*)b.Dc1, b.G1_64, (T*)b.G1c, pl.status, pl.counters,
                                   L.st));
    else
      HIP_TRY(launch_procrustes<T>(src, nrow, ld, r.n2, r.D2, (T*)b.Dc2, b.G2_64, (T*)b.G2c, pl.status, pl.counters,
                                   L.st));
    return L.end();
  }
  RmseOut ro{nullptr, nullptr, 0, 0, 0.0};
  if (rmse_q >= 0) ro = RmseOut{pl.trace, pl.iter + rmse_q, rmse_q * (K + 1), nent, (double)r.N * r.m1 * r.m2};
  SDL_TRY(L.begin(3));
  if (side == 1)
    HIP_TRY(launch_tmod_solve<T>(src, nrow, ld, b.sums, r.m1, r.n1, r.D1, (T*)b.Dc1, b.G1_64, (T*)b.G1c, b.w,
                                 pl.status, pl.counters, ro, L.st));
  else
    HIP_TRY(launch_tmod_solve<T>(src, nrow, ld, b.sums, r.m2, r.n2, r.D2, (T*)b.Dc2, b.G2_64, (T*)b.G2c, b.w,
                                 pl.status, pl.counters, ro, L.st));
  return L.end();
}

template <typename T>
TmodArgs<T> tmod_args(int side, const sdl_problem& r, const PBuf& b, const Plan& pl) {
  TmodArgs<T> a;
  a.side = side;
  a.m1 = r.m1; a.m2 = r.m2; a.n1 = r.n1; a.n2 = r.n2; a.s = r.s; a.N = r.N;
  a.Y = pl.ybf16 ? nullptr : (const T*)r.Y;
  a.Yh = pl.ybf16 ? (const uint16_t*)r.Y : nullptr;
  a.Dother = (const T*)(side == 1 ? b.Dc2 : b.Dc1);
  a.supp = r.supp;
  a.coef = (const T*)r.coef;
  return a;
}

// one TMOD half-step from the codes in supp/coef: standalone sums -> reduce -> solve (+ rescale)
// Standalone sums of one side into b.part; returns the number of partial rows.  SDL_MIXED_BF16
// runs them on the BF16 matrix cores where that kernel is compiled for the shape.
template <typename T>
int run_sums(int side, const sdl_problem& r, const PBuf& b, const Plan& pl, const Opt& o, Launcher& L, int* rows) {
  const TmodArgs<T> a = tmod_args<T>(side, r, b, pl);
  bool bf16 = false;
  if constexpr (sizeof(T) == 4) bf16 = o.prec == SDL_MIXED_BF16 && tmod_sums_bf16_supported(r.m1, r.m2, r.n1, r.n2, r.s);
  if (bf16) {
    *rows = side == 1 ? tmod_bf16_num_blocks(r.N, r.n1, r.m1, r.m2, r.s, r.n2)
                      : tmod_bf16_num_blocks(r.N, r.n2, r.m2, r.m1, r.s, r.n1);
  } else {
    *rows = side == 1 ? tmod_num_blocks_for(r.N, r.n1, r.m1, r.m2, r.s, r.n2, sizeof(T))
                      : tmod_num_blocks_for(r.N, r.n2, r.m2, r.m1, r.s, r.n1, sizeof(T));
  }
  SDL_TRY(L.begin(1));
  if constexpr (sizeof(T) == 4) {
    if (bf16) {
      HIP_TRY(launch_tmod_sums_bf16(a, b.part, L.st));
      return L.end();
    }
  }
  HIP_TRY(launch_tmod_sums<T>(a, b.part, L.st));
  return L.end();
}

template <typename T>
int run_update(int side, const sdl_problem& r, const PBuf& b, const Plan& pl, const Opt& o, bool rescale, Launcher& L) {
  int nblk = 0;
  SDL_TRY(run_sums<T>(side, r, b, pl, o, L, &nblk));
  SDL_TRY(run_reduce_solve<T>(side, r, b, pl, nblk, false, -1, 0, L, o.method));
  if (rescale && o.method == 0) {
    SDL_TRY(L.begin(6));
    HIP_TRY(launch_rescale<T>(side, r.n1, r.s, r.N, r.supp, (T*)r.coef, b.w, L.st));
    SDL_TRY(L.end());
  }
  return SDL_OK;
}

template <typename T>
int run_rmse(const sdl_problem& r, const PBuf& b, const Plan& pl, int q, int K, Launcher& L) {
  SDL_TRY(L.begin(5));
  HIP_TRY(launch_rmse<T>((const T*)r.res2, r.N, (double)r.N * r.m1 * r.m2, b.rpart, b.rblk, pl.trace, 1,
                         q * (K + 1), pl.iter + q, L.st));
  return L.end();
}

int begin_call(hipStream_t st, Ctx* ctx, const Plan& pl, int nprob) {
  (void)ctx;
  HIP_TRY(launch_fill_int(pl.status, 4, 0, st));
  HIP_TRY(launch_fill_int((int*)pl.counters, 2 * kNumCounters, 0, st));
  HIP_TRY(launch_fill_int(pl.iter, nprob > 0 ? nprob : 1, 0, st));
  return SDL_OK;
}

template <typename T>
int run_check_finite(const sdl_problem* p, int nprob, const Plan& pl, hipStream_t st) {
  for (int q = 0; q < nprob; ++q) {
    if (pl.ybf16)
      HIP_TRY(launch_check_finite_bf16((const uint16_t*)p[q].Y, p[q].N * p[q].m1 * p[q].m2, pl.status, st));
    else
      HIP_TRY(launch_check_finite<T>((const T*)p[q].Y, p[q].N * p[q].m1 * p[q].m2, pl.status, st));
    HIP_TRY(launch_check_finite<double>(p[q].D1, (int64_t)p[q].m1 * p[q].n1, pl.status, st));
    HIP_TRY(launch_check_finite<double>(p[q].D2, (int64_t)p[q].m2 * p[q].n2, pl.status, st));
  }
  return SDL_OK;
}

// Sync, read back status / counters / timings.
int finish_call(hipStream_t st, Ctx* ctx, const Plan& pl, const Opt& o, std::vector<std::pair<int, int>>& marks,
                bool sync) {
  if (!sync && !o.stats) return SDL_OK;
  HIP_TRY(hipStreamSynchronize(st));
  int status = 0;
  unsigned long long ctr[kNumCounters];
  HIP_TRY(hipMemcpy(&status, pl.status, sizeof(int), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(ctr, pl.counters, sizeof(ctr), hipMemcpyDeviceToHost));
  if (o.stats) {
    o.stats->early_stops += (int64_t)ctr[kCtrEarlyStop];
    o.stats->fp64_pivots += (int64_t)ctr[kCtrFp64Pivot];
    o.stats->unused_atoms += (int64_t)ctr[kCtrUnusedAtoms];
    o.stats->singular_updates += (int64_t)ctr[kCtrSingular];
    o.stats->near_tie_rescores += (int64_t)ctr[kCtrRescored];
    o.stats->near_tie_overflows += (int64_t)ctr[kCtrTieOverflow];
    o.stats->proposals_accepted += (int64_t)(ctr[kCtrProposed] - ctr[kCtrFallback]);
    o.stats->fallbacks += (int64_t)ctr[kCtrFallback];
    for (auto& m : marks) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[m.second], ctx->ev[m.second + 1]));
      o.stats->kernel_ms[m.first] += ms;
      o.stats->kernel_launches[m.first] += 1;
    }
  }
  if (status & kStatusNonfinite) return fail(SDL_E_NONFINITE, "non-finite value in Y or a dictionary");
  if (status & kStatusSingular)
    return fail(SDL_E_SINGULAR, "a dictionary update's Gram sum was not positive definite; dictionary kept");
  return SDL_OK;
}

template <typename T>
int sparse_code_impl(const sdl_problem* p, int nprob, const Opt& o, hipStream_t st) {
  Ctx* ctx;
  SDL_TRY(get_ctx(st, &ctx));
  Plan pl;
  layout(p, nprob, sizeof(T), 0, nullptr, &pl);
  void* wsb = nullptr;
  SDL_TRY(acquire_ws(ctx, o, pl.bytes, st, &wsb));
  layout(p, nprob, sizeof(T), 0, wsb, &pl);
  pl.ybf16 = o.prec == SDL_BF16 || o.prec == SDL_MIXED_BF16;
  std::vector<std::pair<int, int>> marks;
  Launcher L{st, o.timing != 0 && o.stats != nullptr, ctx, &marks};
  SDL_TRY(begin_call(st, ctx, pl, nprob));
  if (o.check_finite) {
    SDL_TRY(run_check_finite<T>(p, nprob, pl, st));
    SDL_TRY(finish_call(st, ctx, pl, o, marks, true));
  }
  for (int q = 0; q < nprob; ++q) {
    if (p[q].N == 0) continue;
    SDL_TRY(run_prep<T>(p[q], pl.pb[q], L));
    SDL_TRY(run_omp<T>(p[q], pl.pb[q], o, pl, 0, L));
  }
  return finish_call(st, ctx, pl, o, marks, false);
}

// ------------------------------------------------------------------ allocation-free sparse coding
//
// sdl_sparse_code_noalloc keeps its workspace (status word, counters, compute-type dictionary
// copies and Gram matrices) in this file-scope device array instead of allocated memory.  Each
// device holds its own copy; host code reaches it only through the address that
// hipGetSymbolAddress returns for that device (kept in g_scratch_ptr), never through the
// array's name.

constexpr size_t kScratchBytes = SDL_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Once per device, with that device current: the array's device address and the kernel
// attributes the sparse-coding kernels need (no allocation).
int scratch_for_device(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(SDL_E_DEVICE, "device index %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(SDL_E_DEVICE, "hipGetSymbolAddress returned a null address for the scratch array");
    HIP_TRY(omp_generic_init_device());
    HIP_TRY(tmod_sums_init_device());
    HIP_TRY(tmod_solve_init_device());
    HIP_TRY(omp_fast_init_device());
    HIP_TRY(tmod_sums_bf16_init_device());
    HIP_TRY(ortho_init_device());
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SDL_OK;
}

template <typename T>
int sparse_code_noalloc_impl(const sdl_problem* p, int nprob, const Opt& o, hipStream_t st) {
  Plan pl;
  layout(p, nprob, sizeof(T), 0, nullptr, &pl, true);
  if (pl.bytes > kScratchBytes)
    return fail(SDL_E_NOMEM, "these problems need %zu bytes of workspace; the allocation-free call has %zu",
                pl.bytes, kScratchBytes);
  void* base = nullptr;
  SDL_TRY(scratch_for_device(&base));
  layout(p, nprob, sizeof(T), 0, base, &pl, true);
  pl.ybf16 = o.prec == SDL_BF16 || o.prec == SDL_MIXED_BF16;
  std::vector<std::pair<int, int>> marks;
  Launcher L{st, false, nullptr, &marks};
  SDL_TRY(begin_call(st, nullptr, pl, nprob));
  if (o.check_finite) {
    SDL_TRY(run_check_finite<T>(p, nprob, pl, st));
    SDL_TRY(finish_call(st, nullptr, pl, o, marks, true));
  }
  for (int q = 0; q < nprob; ++q) {
    if (p[q].N == 0) continue;
    SDL_TRY(run_prep<T>(p[q], pl.pb[q], L));
    SDL_TRY(run_omp<T>(p[q], pl.pb[q], o, pl, 0, L));
  }
  return finish_call(st, nullptr, pl, o, marks, false);
}

template <typename T>
int tmod_update_impl(sdl_problem* p, int nprob, uint32_t sides, const Opt& o, hipStream_t st) {
  Ctx* ctx;
  SDL_TRY(get_ctx(st, &ctx));
  Plan pl;
  layout(p, nprob, sizeof(T), 0, nullptr, &pl);
  void* wsb = nullptr;
  SDL_TRY(acquire_ws(ctx, o, pl.bytes, st, &wsb));
  layout(p, nprob, sizeof(T), 0, wsb, &pl);
  pl.ybf16 = o.prec == SDL_BF16 || o.prec == SDL_MIXED_BF16;
  std::vector<std::pair<int, int>> marks;
  Launcher L{st, o.timing != 0 && o.stats != nullptr, ctx, &marks};
  SDL_TRY(begin_call(st, ctx, pl, nprob));
  if (o.check_finite) {
    SDL_TRY(run_check_finite<T>(p, nprob, pl, st));
    SDL_TRY(finish_call(st, ctx, pl, o, marks, true));
  }
  for (int q = 0; q < nprob; ++q) {
    SDL_TRY(run_prep<T>(p[q], pl.pb[q], L));
    if (sides & 1u) SDL_TRY(run_update<T>(1, p[q], pl.pb[q], pl, o, true, L));
    if (sides & 2u) SDL_TRY(run_update<T>(2, p[q], pl.pb[q], pl, o, true, L));
  }
  return finish_call(st, ctx, pl, o, marks, true);
}

// One node's work in Algorithm 1 step 1 (side 1) or step 3 (side 2): the sparse coding and the
// reduced sums [A | B | sum res2] of its new codes, written to `sums`.
template <typename T>
int sparse_code_sums_impl(const sdl_problem* p, int side, double* sums, const Opt& o, hipStream_t st) {
  Ctx* ctx;
  SDL_TRY(get_ctx(st, &ctx));
  Plan pl;
  layout(p, 1, sizeof(T), 0, nullptr, &pl);
  void* wsb = nullptr;
  SDL_TRY(acquire_ws(ctx, o, pl.bytes, st, &wsb));
  layout(p, 1, sizeof(T), 0, wsb, &pl);
  pl.ybf16 = o.prec == SDL_BF16 || o.prec == SDL_MIXED_BF16;
  std::vector<std::pair<int, int>> marks;
  Launcher L{st, o.timing != 0 && o.stats != nullptr, ctx, &marks};
  SDL_TRY(begin_call(st, ctx, pl, 1));
  if (o.check_finite) {
    SDL_TRY(run_check_finite<T>(p, 1, pl, st));
    SDL_TRY(finish_call(st, ctx, pl, o, marks, true));
  }
  const sdl_problem& r = p[0];
  const PBuf& b = pl.pb[0];
  const int na = side == 1 ? r.n1 : r.n2, mr = side == 1 ? r.m1 : r.m2;
  const int nent = na * na + mr * na;
  if (r.N == 0) {
    HIP_TRY(launch_fill_double(sums, nent + 1, 0.0, st));
    return finish_call(st, ctx, pl, o, marks, false);
  }
  SDL_TRY(run_prep<T>(r, b, L));
  hipError_t e;
  const double* src = nullptr;
  if (o.prec != SDL_MIXED_BF16 && use_fast<T>(r, o)) {
    // sums accumulated in the sparse-coding launch (one row of nent + 1 per workgroup)
    const int rows = omp_fast_partial_rows(r.N, r.m1, r.m2, r.n1, r.n2, r.s);
    SDL_TRY(run_omp<T>(r, b, o, pl, side, L));
    SDL_TRY(L.begin(2));
    const int nrow = launch_reduce_stage1(b.part, rows, nent + 1, b.stage, &src, st, &e);
    HIP_TRY(e);
    HIP_TRY(launch_reduce_final(src, nrow, nent + 1, nent + 1, sums, st));
    SDL_TRY(L.end());
  } else {
    SDL_TRY(run_omp<T>(r, b, o, pl, 0, L));
    int nblk = 0;
    SDL_TRY(run_sums<T>(side, r, b, pl, o, L, &nblk));
    SDL_TRY(L.begin(2));
    const int nrow = launch_reduce_stage1(b.part, nblk, nent, b.stage, &src, st, &e);
    HIP_TRY(e);
    HIP_TRY(launch_reduce_final(src, nrow, nent, nent, sums, st));
    HIP_TRY(launch_sum_res2<T>((const T*)r.res2, r.N, b.rpart, b.rblk, sums + nent, st));
    SDL_TRY(L.end());
  }
  return finish_call(st, ctx, pl, o, marks, false);
}

int validate_learned(const sdl_problem* p, int nprob, const Opt& o) {
  if (!o.proposer) return SDL_OK;
  if (o.err2 > 0.0) return fail(SDL_E_UNSUPPORTED, "the error-driven stop does not apply to the learned proposal");
  if (o.prec != SDL_FP32) return fail(SDL_E_UNSUPPORTED, "the learned proposal runs on FP32 problems");
  for (int q = 0; q < nprob; ++q) {
    if (!proposer_matches(o.proposer, p[q]))
      return fail(SDL_E_SHAPE, "problem %d: shape differs from the proposer's", q);
    if (!omp_fast_supported<float>(p[q].m1, p[q].m2, p[q].n1, p[q].n2, p[q].s) || !propose_supported(p[q].n1, p[q].n2, p[q].s))
      return fail(SDL_E_UNSUPPORTED, "problem %d: no register-resident fallback kernel for this shape", q);
    if (p[q].N > 0 && !p[q].res2) return fail(SDL_E_INVAL, "problem %d: the learned path needs res2", q);
    SDL_TRY(learned_prepare(o.proposer, p[q].N));
  }
  return SDL_OK;
}

// sparse coding of one problem: learned proposal + fallback when a proposer is given
template <typename T>
int run_code(const sdl_problem& r, const PBuf& b, const Opt& o, const Plan& pl, Launcher& L) {
  if constexpr (sizeof(T) == 4) {
    if (o.proposer) {
      SDL_TRY(L.begin(0));
      SDL_TRY(learned_code(o.proposer, r, o.tau, nullptr, omp_args<float>(r, b, o, pl), L.st, nullptr));
      return L.end();
    }
  }
  return run_omp<T>(r, b, o, pl, 0, L);
}

template <typename T>
int iterate_problem(sdl_problem* p, int q, int K, const Opt& o, const Plan& pl, Launcher& L) {
  {
    const sdl_problem& r = p[q];
    if (r.N == 0) return SDL_OK;
    const PBuf& b = pl.pb[q];
    if (o.proposer) {
      SDL_TRY(run_code<T>(r, b, o, pl, L));
      SDL_TRY(run_rmse<T>(r, b, pl, q, K, L));
      SDL_TRY(run_update<T>(1, r, b, pl, o, false, L));
      SDL_TRY(run_code<T>(r, b, o, pl, L));
      SDL_TRY(run_update<T>(2, r, b, pl, o, false, L));
    } else if (o.schedule == 0 && use_fast<T>(r, o)) {
      // Algorithm 1 with the sums (and the RMSE) computed in the sparse-coding epilogue
      const int rows = omp_fast_partial_rows(r.N, r.m1, r.m2, r.n1, r.n2, r.s);
      SDL_TRY(run_omp<T>(r, b, o, pl, 1, L));
      SDL_TRY(run_reduce_solve<T>(1, r, b, pl, rows, true, q, K, L));
      SDL_TRY(run_omp<T>(r, b, o, pl, 2, L));
      SDL_TRY(run_reduce_solve<T>(2, r, b, pl, rows, true, -1, K, L));
    } else if (o.method == 1 && o.schedule == 0 && sizeof(T) == 4 &&
               ortho_mfma_supported(r.m1, r.m2, r.n1, r.n2, r.s)) {
      // Remark 1's variant with the B sums of each Procrustes update in the coding epilogue
      const int rows = (int)ortho_mfma_partial_rows(r.N, r.m1, r.m2, r.s);
      SDL_TRY(run_omp<T>(r, b, o, pl, 1, L));
      SDL_TRY(run_rmse<T>(r, b, pl, q, K, L));
      SDL_TRY(run_reduce_solve<T>(1, r, b, pl, rows, true, -1, K, L, 1));
      SDL_TRY(run_omp<T>(r, b, o, pl, 2, L));
      SDL_TRY(run_reduce_solve<T>(2, r, b, pl, rows, true, -1, K, L, 1));
    } else {
      SDL_TRY(run_omp<T>(r, b, o, pl, 0, L));
      SDL_TRY(run_rmse<T>(r, b, pl, q, K, L));
      if (o.schedule == 0) {
        SDL_TRY(run_update<T>(1, r, b, pl, o, false, L));
        SDL_TRY(run_omp<T>(r, b, o, pl, 0, L));
        SDL_TRY(run_update<T>(2, r, b, pl, o, false, L));
      } else {
        SDL_TRY(run_update<T>(2, r, b, pl, o, true, L));
        SDL_TRY(run_update<T>(1, r, b, pl, o, false, L));
      }
    }
  }
  return SDL_OK;
}

// One Algorithm 1 iteration of every problem, in order on L's stream.
template <typename T>
int one_iteration(sdl_problem* p, int nprob, int K, const Opt& o, const Plan& pl, Launcher& L) {
  for (int q = 0; q < nprob; ++q) SDL_TRY(iterate_problem<T>(p, q, K, o, pl, L));
  return SDL_OK;
}

// The same while L's stream is being captured: the problems are independent (own
// buffers; shared counters are updated atomically), so each gets a branch of the
// graph, forked from and joined back into L's stream.
template <typename T>
int one_iteration_branched(sdl_problem* p, int nprob, int K, const Opt& o, const Plan& pl, Launcher& L, Ctx* ctx) {
  int nact = 0;
  for (int q = 0; q < nprob; ++q) nact += p[q].N > 0;
  // a proposer's scratch buffers are shared by all problems: those run in order
  if (nact <= 1 || o.proposer) return one_iteration<T>(p, nprob, K, o, pl, L);
  const int nb = nact < kMaxBranches ? nact : kMaxBranches;
  while ((int)ctx->branch.size() < nb) {
    hipStream_t s;
    hipEvent_t e;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ctx->branch.push_back(s);
    ctx->branch_join.push_back(e);
  }
  if (!ctx->fork) HIP_TRY(hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(ctx->fork, L.st));
  for (int i = 0; i < nb; ++i) HIP_TRY(hipStreamWaitEvent(ctx->branch[i], ctx->fork, 0));
  int slot = 0;
  for (int q = 0; q < nprob; ++q) {
    if (p[q].N == 0) continue;
    Launcher B{ctx->branch[slot % nb], false, ctx, L.marks};
    SDL_TRY(iterate_problem<T>(p, q, K, o, pl, B));
    ++slot;
  }
  for (int i = 0; i < nb; ++i) {
    HIP_TRY(hipEventRecord(ctx->branch_join[i], ctx->branch[i]));
    HIP_TRY(hipStreamWaitEvent(L.st, ctx->branch_join[i], 0));
  }
  return SDL_OK;
}

// Everything a captured learning graph bakes in: the problems (pointers and shapes), the
// iterations per graph and K (the RMSE trace offsets), the options that select kernels or
// enter kernel arguments, the workspace base and the kernel choices in force.  A later call
// with an equal key replays the instantiated graph instead of capturing it again.
std::vector<unsigned char> graph_key(const sdl_problem* p, int nprob, int K, int per, const Opt& o, const void* ws) {
  std::vector<unsigned char> k;
  auto put = [&k](const void* v, size_t n) {
    const unsigned char* b = (const unsigned char*)v;
    k.insert(k.end(), b, b + n);
  };
  put(p, sizeof(sdl_problem) * (size_t)nprob);
  const long epoch = tuning_epoch();
  const int ints[] = {nprob, K, per, o.prec, o.schedule, o.kernel, o.method};
  const double dbl[] = {o.stop_rel, o.dep_eps, o.pivot_fp64, o.tau, o.err2, o.tie_band};
  put(ints, sizeof(ints));
  put(dbl, sizeof(dbl));
  put(&o.proposer, sizeof(o.proposer));
  put(&ws, sizeof(ws));
  put(&epoch, sizeof(epoch));
  return k;
}

template <typename T>
int learn_impl(sdl_problem* p, int nprob, int K, double* trace, const Opt& o, hipStream_t st) {
  Ctx* ctx;
  SDL_TRY(get_ctx(st, &ctx));
  // res2 is needed for the RMSE trace; require it
  for (int q = 0; q < nprob; ++q)
    if (p[q].N > 0 && !p[q].res2) return fail(SDL_E_INVAL, "problem %d: sdl_learn needs res2", q);
  Plan pl;
  layout(p, nprob, sizeof(T), K, nullptr, &pl);
  void* wsb = nullptr;
  SDL_TRY(acquire_ws(ctx, o, pl.bytes, st, &wsb));
  layout(p, nprob, sizeof(T), K, wsb, &pl);
  pl.ybf16 = o.prec == SDL_BF16 || o.prec == SDL_MIXED_BF16;
  std::vector<std::pair<int, int>> marks;
  const bool timing = o.timing != 0 && o.stats != nullptr;
  Launcher L{st, timing, ctx, &marks};
  SDL_TRY(begin_call(st, ctx, pl, nprob));
  if (o.check_finite) {
    SDL_TRY(run_check_finite<T>(p, nprob, pl, st));
    SDL_TRY(finish_call(st, ctx, pl, o, marks, true));
  }
  for (int q = 0; q < nprob; ++q) SDL_TRY(run_prep<T>(p[q], pl.pb[q], L));
  const bool graph = o.use_graph && !timing && K > 1;
  if (graph) {
    if (!ctx->side) {
      HIP_TRY(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
      HIP_TRY(hipEventCreateWithFlags(&ctx->join_a, hipEventDisableTiming));
      HIP_TRY(hipEventCreateWithFlags(&ctx->join_b, hipEventDisableTiming));
    }
    HIP_TRY(hipEventRecord(ctx->join_a, st));
    HIP_TRY(hipStreamWaitEvent(ctx->side, ctx->join_a, 0));
    Launcher G{ctx->side, false, ctx, &marks};
    const int per = K < kItersPerGraph ? K : kItersPerGraph;
    std::vector<unsigned char> key = graph_key(p, nprob, K, per, o, wsb);
    if (!ctx->gexec || key != ctx->gkey) {
      if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
      if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
      ctx->gexec = nullptr;
      ctx->graph = nullptr;
      ctx->gkey.clear();
      hipGraph_t g = nullptr;
      HIP_TRY(hipStreamBeginCapture(ctx->side, hipStreamCaptureModeRelaxed));
      int rc = SDL_OK;
      for (int it = 0; it < per && rc == SDL_OK; ++it) rc = one_iteration_branched<T>(p, nprob, K, o, pl, G, ctx);
      hipError_t ce = hipStreamEndCapture(ctx->side, &g);
      if (rc != SDL_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      HIP_TRY(ce);
      hipGraphExec_t ge = nullptr;
      hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      if (ie != hipSuccess) {
        (void)hipGraphDestroy(g);
        HIP_TRY(ie);
      }
      ctx->graph = g;
      ctx->gexec = ge;
      ctx->gkey.swap(key);
    }
    for (int it = 0; it + per <= K; it += per) HIP_TRY(hipGraphLaunch(ctx->gexec, ctx->side));
    for (int it = 0; it < K % per; ++it) SDL_TRY(one_iteration<T>(p, nprob, K, o, pl, G));
    HIP_TRY(hipEventRecord(ctx->join_b, ctx->side));
    HIP_TRY(hipStreamWaitEvent(st, ctx->join_b, 0));
  } else {
    for (int it = 0; it < K; ++it) SDL_TRY(one_iteration<T>(p, nprob, K, o, pl, L));
  }
  for (int q = 0; q < nprob; ++q) {
    if (p[q].N == 0) continue;
    SDL_TRY(run_code<T>(p[q], pl.pb[q], o, pl, L));
    SDL_TRY(run_rmse<T>(p[q], pl.pb[q], pl, q, K, L));
  }
  int rc = finish_call(st, ctx, pl, o, marks, true);
  if (trace && (rc == SDL_OK || rc == SDL_E_SINGULAR)) {
    std::vector<double> h((size_t)(nprob > 0 ? nprob : 1) * (K + 1), 0.0);
    HIP_TRY(hipMemcpy(h.data(), pl.trace, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
    memcpy(trace, h.data(), sizeof(double) * (size_t)nprob * (K + 1));
  }
  return rc;
}

}  // namespace

namespace sdl {
int abi_fail(int st, const char* msg) { return fail(st, "%s", msg); }
}  // namespace sdl

namespace {

// Median over reps of the device time of f() (one warm-up call first), with events on st.
template <class F>
int time_median(hipStream_t st, int reps, double* out, F f) {
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(f());
  std::vector<float> t;
  for (int r = 0; r < reps; ++r) {
    HIP_TRY(hipEventRecord(e0, st));
    HIP_TRY(f());
    HIP_TRY(hipEventRecord(e1, st));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    t.push_back(ms);
  }
  HIP_TRY(hipEventDestroy(e0));
  HIP_TRY(hipEventDestroy(e1));
  std::sort(t.begin(), t.end());
  *out = t[t.size() / 2];
  return SDL_OK;
}

// ------------------------------------------------------------------ n-dimensional signals (Remark 3)

struct TPlan {
  Plan pl;  // status, counters, iteration counter, RMSE trace
  void* Dc[kTensorMaxModes];
  double* G64[kTensorMaxModes];
  void* Gc[kTensorMaxModes];
  double *part, *stage, *sums, *w, *rpart;
  int rows, rblk, nent;
  // FP32 shapes coded by the two-mode one-wave kernel: modes 2.. collapsed into one Kronecker
  // factor Dk (mk x nk, FP64 master, compute-type copy and Grams)
  bool collapsed;
  int mk, nk;
  double *Dk64, *Gk64;
  void *Dkc, *Gkc;
  size_t bytes;
};

bool tensor_collapsed(const sdl_tensor_problem* p, size_t elem) {
  if (elem != 4) return false;
  int64_t mk = 1, nk = 1;
  for (int d = 1; d < p->nmodes; ++d) {
    mk *= p->m[d];
    nk *= p->n[d];
  }
  // the dictionary preparation stages the factor in LDS at (mk + 1) x nk doubles
  if ((mk + 1) * nk > (int64_t)(SDL_MAX_M + 1) * SDL_MAX_N) return false;
  return omp_wave_collapsed_supported(p->m[0], (int)mk, p->n[0], (int)nk, p->s);
}

void tensor_ws_layout(const sdl_tensor_problem* p, size_t elem, int K, void* base, TPlan* tp) {
  Bump b(base);
  tp->pl.status = b.take<int>(4);
  tp->pl.counters = b.take<unsigned long long>(kNumCounters);
  tp->pl.iter = b.take<int>(1);
  tp->pl.trace = b.take<double>((size_t)K + 1);
  int nmax = 1, nent = 1;
  for (int d = 0; d < p->nmodes; ++d) {
    tp->Dc[d] = b.take<char>(elem * p->m[d] * p->n[d]);
    tp->G64[d] = b.take<double>((size_t)p->n[d] * p->n[d]);
    tp->Gc[d] = b.take<char>(elem * p->n[d] * p->n[d]);
    nmax = p->n[d] > nmax ? p->n[d] : nmax;
    const int e = p->n[d] * p->n[d] + p->m[d] * p->n[d];
    nent = e > nent ? e : nent;
  }
  tp->collapsed = tensor_collapsed(p, elem);
  tp->mk = tp->nk = 1;
  for (int d = 1; d < p->nmodes; ++d) {
    tp->mk *= p->m[d];
    tp->nk *= p->n[d];
  }
  if (tp->collapsed) {
    tp->Dk64 = b.take<double>((size_t)tp->mk * tp->nk);
    tp->Gk64 = b.take<double>((size_t)tp->nk * tp->nk);
    tp->Dkc = b.take<char>(elem * tp->mk * tp->nk);
    tp->Gkc = b.take<char>(elem * tp->nk * tp->nk);
  } else {
    tp->Dk64 = tp->Gk64 = nullptr;
    tp->Dkc = tp->Gkc = nullptr;
  }
  tp->rows = tensor_sums_rows(p->N);
  tp->nent = nent;
  tp->part = b.take<double>((size_t)tp->rows * nent);
  tp->stage = b.take<double>((size_t)reduce_stage_rows(tp->rows) * nent);
  tp->sums = b.take<double>((size_t)nent);
  tp->w = b.take<double>((size_t)nmax);
  tp->rblk = rmse_num_blocks(p->N);
  tp->rpart = b.take<double>((size_t)tp->rblk);
  tp->bytes = b.off + 256;
  tp->pl.bytes = tp->bytes;
}

int64_t tensor_elems(const int32_t* v, int nm) {
  int64_t e = 1;
  for (int d = 0; d < nm; ++d) e *= v[d];
  return e;
}

int validate_tensor(const sdl_tensor_problem* p, const Opt& o, bool update) {
  SDL_TRY(validate(nullptr, 0, o, false));  // the options alone
  if (!p) return fail(SDL_E_INVAL, "problem is NULL");
  if (o.prec != SDL_FP64 && o.prec != SDL_FP32)
    return fail(SDL_E_UNSUPPORTED, "n-dimensional signals run in SDL_FP64 or SDL_FP32");
  if (o.kernel != 0 || o.method != 0 || o.schedule != 0 || o.proposer)
    return fail(SDL_E_UNSUPPORTED, "n-dimensional signals have one kernel, Algorithm 1's schedule and no proposer");
  if (o.workspace) return fail(SDL_E_UNSUPPORTED, "n-dimensional calls use the library's own workspace");
  if (p->nmodes < 2 || p->nmodes > SDL_TENSOR_MAX_MODES)
    return fail(SDL_E_SHAPE, "nmodes = %d (2..%d)", p->nmodes, SDL_TENSOR_MAX_MODES);
  const int nm = p->nmodes;
  for (int d = 0; d < nm; ++d) {
    if (p->m[d] <= 0 || p->n[d] <= 0 || p->m[d] > SDL_MAX_M || p->n[d] > SDL_MAX_N)
      return fail(SDL_E_SHAPE, "mode %d: m = %d, n = %d (1..%d, 1..%d)", d + 1, p->m[d], p->n[d], SDL_MAX_M,
                  SDL_MAX_N);
    if (!p->D[d]) return fail(SDL_E_INVAL, "mode %d: dictionary is NULL", d + 1);
  }
  const int64_t M = tensor_elems(p->m, nm), A = tensor_elems(p->n, nm);
  if (M > SDL_TENSOR_MAX_ELEMS || A > SDL_TENSOR_MAX_ELEMS)
    return fail(SDL_E_SHAPE, "prod m = %lld, prod n = %lld (at most %d each)", (long long)M, (long long)A,
                SDL_TENSOR_MAX_ELEMS);
  if (p->s <= 0 || p->s > SDL_MAX_S || p->s > M || p->s > A)
    return fail(SDL_E_SHAPE, "s = %d (1..%d, at most prod m and prod n)", p->s, SDL_MAX_S);
  if (p->N < 0) return fail(SDL_E_INVAL, "N = %lld < 0", (long long)p->N);
  if (p->N > 0 && (!p->Y || !p->supp || !p->coef)) return fail(SDL_E_INVAL, "Y/supp/coef is NULL");
  const size_t elem = o.prec == SDL_FP64 ? 8 : 4;
  int m[kTensorMaxModes], n[kTensorMaxModes];
  for (int d = 0; d < kTensorMaxModes; ++d) {
    m[d] = d < nm ? p->m[d] : 1;
    n[d] = d < nm ? p->n[d] : 1;
  }
  if (tensor_omp_lds_bytes(nm, m, n, p->s, elem) > 160 * 1024)
    return fail(SDL_E_UNSUPPORTED, "the working set of one signal exceeds the 160 KiB LDS");
  if (update)
    for (int d = 0; d < nm; ++d)
      if (tensor_sums_lds(nm, m, n, d, elem) > 160 * 1024)
        return fail(SDL_E_UNSUPPORTED, "mode %d: the update's working set exceeds the 160 KiB LDS", d + 1);
  return SDL_OK;
}

template <typename T>
TensorArgs<T> tensor_args(const sdl_tensor_problem* p, const TPlan& tp, const Opt& o) {
  TensorArgs<T> a;
  a.nmodes = p->nmodes;
  a.s = p->s;
  for (int d = 0; d < kTensorMaxModes; ++d) {
    const bool on = d < p->nmodes;
    a.m[d] = on ? p->m[d] : 1;
    a.n[d] = on ? p->n[d] : 1;
    a.D[d] = on ? (const T*)tp.Dc[d] : nullptr;
    a.G[d] = on ? (const T*)tp.Gc[d] : nullptr;
  }
  a.N = p->N;
  a.Y = (const T*)p->Y;
  a.supp = p->supp;
  a.coef = (T*)p->coef;
  a.res2 = (T*)p->res2;
  a.stop_rel = o.stop_rel;
  a.dep_eps = o.dep_eps;
  a.pivot_fp64 = o.pivot_fp64;
  a.err2 = o.err2;
  a.counters = tp.pl.counters;
  return a;
}

template <typename T>
int tensor_prep(const sdl_tensor_problem* p, const TPlan& tp, hipStream_t st) {
  for (int d = 0; d < p->nmodes; ++d)
    HIP_TRY(launch_dict_prep<T>(p->D[d], p->m[d], p->n[d], (T*)tp.Dc[d], tp.G64[d], (T*)tp.Gc[d], st));
  return SDL_OK;
}

// mode d (0-based) update from the codes: sums, fixed-order reduction, FP64 solve with
// normalisation, then (rescale) the codes' rescaling by the column norms
template <typename T>
int tensor_update_mode(const sdl_tensor_problem* p, const TPlan& tp, const Opt& o, int d, bool rescale,
                       hipStream_t st) {
  const TensorArgs<T> a = tensor_args<T>(p, tp, o);
  const int na = p->n[d], mr = p->m[d], nent = na * na + mr * na;
  HIP_TRY(launch_tensor_sums<T>(a, d, tp.part, st));
  const double* src = nullptr;
  hipError_t e;
  const int nrow = launch_reduce_stage1(tp.part, tp.rows, nent, tp.stage, &src, st, &e);
  HIP_TRY(e);
  const RmseOut none{nullptr, nullptr, 0, 0, 0.0};
  HIP_TRY(launch_tmod_solve<T>(src, nrow, nent, tp.sums, mr, na, p->D[d], (T*)tp.Dc[d], tp.G64[d], (T*)tp.Gc[d],
                               tp.w, tp.pl.status, tp.pl.counters, none, st));
  if (rescale) HIP_TRY(launch_tensor_rescale<T>(a, d, tp.w, st));
  return SDL_OK;
}

// sparse coding of every signal: the two-mode one-wave kernel on (D_1, D_n (x) ... (x) D_2) for the
// collapsed FP32 shapes (the same atoms in the same order: a = i_1 + n_1 j', j' = i_2 + n_2 (...)),
// else the n-mode kernel
template <typename T>
int tensor_code(const sdl_tensor_problem* p, const TPlan& tp, const Opt& o, hipStream_t st) {
  if constexpr (sizeof(T) == 4) {
    if (tp.collapsed) {
      TensorArgs<double> dd{};
      dd.nmodes = p->nmodes;
      for (int d = 0; d < kTensorMaxModes; ++d) {
        dd.m[d] = d < p->nmodes ? p->m[d] : 1;
        dd.n[d] = d < p->nmodes ? p->n[d] : 1;
        dd.D[d] = d < p->nmodes ? p->D[d] : nullptr;
      }
      HIP_TRY(launch_kron_tail(dd, tp.Dk64, st));
      HIP_TRY(launch_dict_prep<float>(tp.Dk64, tp.mk, tp.nk, (float*)tp.Dkc, tp.Gk64, (float*)tp.Gkc, st));
      OmpArgs<float> a{};
      a.m1 = p->m[0]; a.m2 = tp.mk; a.n1 = p->n[0]; a.n2 = tp.nk; a.s = p->s; a.N = p->N;
      a.Y = (const float*)p->Y;
      a.Yh = nullptr;
      a.D1 = (const float*)tp.Dc[0];
      a.D2 = (const float*)tp.Dkc;
      a.G1 = (const float*)tp.Gc[0];
      a.G2 = (const float*)tp.Gkc;
      a.supp = p->supp;
      a.coef = (float*)p->coef;
      a.res2 = (float*)p->res2;
      a.stop_rel = o.stop_rel; a.dep_eps = o.dep_eps; a.pivot_fp64 = o.pivot_fp64; a.err2 = o.err2;
      a.tie_band = o.tie_band;
      a.counters = tp.pl.counters;
      a.sums_side = 0;
      a.sums_part = nullptr;
      a.index = nullptr;
      a.count = nullptr;
      HIP_TRY(launch_omp_wave_collapsed(a, st));
      return SDL_OK;
    }
  }
  HIP_TRY(launch_tensor_omp<T>(tensor_args<T>(p, tp, o), st));
  return SDL_OK;
}

template <typename T>
int tensor_check_finite(const sdl_tensor_problem* p, const TPlan& tp, hipStream_t st) {
  HIP_TRY(launch_check_finite<T>((const T*)p->Y, p->N * tensor_elems(p->m, p->nmodes), tp.pl.status, st));
  for (int d = 0; d < p->nmodes; ++d)
    HIP_TRY(launch_check_finite<double>(p->D[d], (int64_t)p->m[d] * p->n[d], tp.pl.status, st));
  return SDL_OK;
}

// call: 0 sparse coding, 1 one mode's update (mode 0-based), 2 learning (K iterations)
template <typename T>
int tensor_impl(const sdl_tensor_problem* p, int call, int mode, int K, double* trace, const Opt& o, hipStream_t st) {
  Ctx* ctx;
  SDL_TRY(get_ctx(st, &ctx));
  TPlan tp;
  tensor_ws_layout(p, sizeof(T), K, nullptr, &tp);
  SDL_TRY_WS(ensure_ws(ctx, tp.bytes, st));
  tensor_ws_layout(p, sizeof(T), K, ctx->ws, &tp);
  std::vector<std::pair<int, int>> marks;
  SDL_TRY(begin_call(st, ctx, tp.pl, 1));
  if (o.check_finite) {
    SDL_TRY(tensor_check_finite<T>(p, tp, st));
    SDL_TRY(finish_call(st, ctx, tp.pl, o, marks, true));
  }
  SDL_TRY(tensor_prep<T>(p, tp, st));
  const double denom = (double)p->N * (double)tensor_elems(p->m, p->nmodes);
  if (call == 0) {
    SDL_TRY(tensor_code<T>(p, tp, o, st));
    return finish_call(st, ctx, tp.pl, o, marks, false);
  }
  if (call == 1) {
    if (p->N > 0) SDL_TRY(tensor_update_mode<T>(p, tp, o, mode, true, st));
    return finish_call(st, ctx, tp.pl, o, marks, true);
  }
  // Algorithm 1 with one sweep per mode: codes, then that mode's dictionary
  for (int it = 0; it < K && p->N > 0; ++it)
    for (int d = 0; d < p->nmodes; ++d) {
      SDL_TRY(tensor_code<T>(p, tp, o, st));
      if (d == 0 && p->res2)
        HIP_TRY(launch_rmse<T>((const T*)p->res2, p->N, denom, tp.rpart, tp.rblk, tp.pl.trace, 1, 0, tp.pl.iter, st));
      SDL_TRY(tensor_update_mode<T>(p, tp, o, d, false, st));
    }
  if (p->N > 0) {
    SDL_TRY(tensor_code<T>(p, tp, o, st));
    if (p->res2)
      HIP_TRY(launch_rmse<T>((const T*)p->res2, p->N, denom, tp.rpart, tp.rblk, tp.pl.trace, 1, 0, tp.pl.iter, st));
  }
  int rc = finish_call(st, ctx, tp.pl, o, marks, true);
  if (trace && (rc == SDL_OK || rc == SDL_E_SINGULAR)) {
    if (p->N > 0 && p->res2) {
      HIP_TRY(hipMemcpy(trace, tp.pl.trace, sizeof(double) * ((size_t)K + 1), hipMemcpyDeviceToHost));
    } else {
      for (int i = 0; i <= K; ++i) trace[i] = 0.0;
    }
  }
  return rc;
}

template <typename T>
int patches_to_image_impl(const sdl_problem* p, int H, int W, const Opt& o, void* image, hipStream_t st) {
  Ctx* ctx;
  SDL_TRY(get_ctx(st, &ctx));
  Plan pl;
  layout(p, 1, sizeof(T), 0, nullptr, &pl);
  void* wsb = nullptr;
  SDL_TRY(acquire_ws(ctx, o, pl.bytes, st, &wsb));
  layout(p, 1, sizeof(T), 0, wsb, &pl);
  std::vector<std::pair<int, int>> marks;
  Launcher L{st, false, ctx, &marks};
  SDL_TRY(run_prep<T>(p[0], pl.pb[0], L));
  HIP_TRY(launch_patches_to_image<T>(p->supp, (const T*)p->coef, (const T*)pl.pb[0].Dc1, (const T*)pl.pb[0].Dc2, H, W,
                                     p->m1, p->m2, p->n1, p->n2, p->s, (T*)image, st));
  return SDL_OK;
}

}  // namespace

extern "C" {

void sdl_default_options(sdl_options* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->prec = SDL_FP64;
  o->schedule = 0;
  o->use_graph = 1;
  o->check_finite = 0;
  o->timing = 0;
  o->kernel = 0;
  o->stop_rel = -1.0;
  o->dep_eps = -1.0;
  o->pivot_fp64 = -1.0;
  o->stats = nullptr;
  o->proposer = nullptr;
  o->tau = 0.0;
  o->err2 = 0.0;
  o->tie_band = 1.0 / 64.0;
  o->fallback_margin = 1.01;
  o->deterministic = 1;
  o->reserved0 = 0;
  o->workspace = nullptr;
  o->workspace_bytes = 0;
  o->method = 0;
  o->reserved1 = 0;
}

int sdl_sparse_code_noalloc(const sdl_problem* p, int32_t nprob, const sdl_options* o, void* stream) {
  g_err.clear();
  Opt opt = resolve(o);
  SDL_TRY(validate(p, nprob, opt, false));
  if (opt.timing) return fail(SDL_E_INVAL, "the allocation-free call does not time kernels (timing = 0)");
  if (opt.workspace) return fail(SDL_E_INVAL, "the allocation-free call uses its own scratch (workspace = NULL)");
  hipStream_t st = (hipStream_t)stream;
  return opt.prec == SDL_FP64 ? sparse_code_noalloc_impl<double>(p, nprob, opt, st)
                              : sparse_code_noalloc_impl<float>(p, nprob, opt, st);
}

int sdl_sparse_code_sums(const sdl_problem* p, int32_t side, double* sums, const sdl_options* o, void* stream) {
  g_err.clear();
  Opt opt = resolve(o);
  SDL_TRY(validate(p, 1, opt, false));
  if (side != 1 && side != 2) return fail(SDL_E_INVAL, "side = %d (1 or 2)", side);
  if (!sums) return fail(SDL_E_INVAL, "sums is NULL");
  if (p->N > 0 && !p->res2) return fail(SDL_E_INVAL, "sdl_sparse_code_sums needs res2");
  SDL_TRY(check_workspace(p, 1, 0, opt));
  hipStream_t st = (hipStream_t)stream;
  return opt.prec == SDL_FP64 ? sparse_code_sums_impl<double>(p, side, sums, opt, st)
                              : sparse_code_sums_impl<float>(p, side, sums, opt, st);
}

int sdl_image_to_patches(const void* image, int32_t H, int32_t W, int32_t m1, int32_t m2, int32_t prec,
                         void* patches, void* stream) {
  g_err.clear();
  if (prec != SDL_FP32 && prec != SDL_FP64) return fail(SDL_E_INVAL, "prec must be SDL_FP32 or SDL_FP64");
  if (m1 <= 0 || m2 <= 0 || m1 > SDL_MAX_M || m2 > SDL_MAX_M || H < m1 || W < m2)
    return fail(SDL_E_SHAPE, "need 0 < m1 <= H, 0 < m2 <= W and m1, m2 <= %d", SDL_MAX_M);
  if (!image || !patches) return fail(SDL_E_INVAL, "NULL pointer");
  hipStream_t st = (hipStream_t)stream;
  if (prec == SDL_FP64)
    HIP_TRY(launch_image_to_patches<double>((const double*)image, H, W, m1, m2, (double*)patches, st));
  else
    HIP_TRY(launch_image_to_patches<float>((const float*)image, H, W, m1, m2, (float*)patches, st));
  return SDL_OK;
}

int sdl_patches_to_image(const sdl_problem* p, int32_t H, int32_t W, const sdl_options* o, void* image,
                         void* stream) {
  g_err.clear();
  Opt opt = resolve(o);
  if (!p || !image) return fail(SDL_E_INVAL, "NULL pointer");
  if (opt.prec != SDL_FP32 && opt.prec != SDL_FP64) return fail(SDL_E_INVAL, "prec must be SDL_FP32 or SDL_FP64");
  sdl_problem q = *p;
  q.Y = q.Y ? q.Y : image;  // signals are not read
  SDL_TRY(validate(&q, 1, opt, false));
  if (H < p->m1 || W < p->m2 || (int64_t)(H - p->m1 + 1) * (W - p->m2 + 1) != p->N)
    return fail(SDL_E_SHAPE, "N = %lld is not (H - m1 + 1)(W - m2 + 1) for H = %d, W = %d", (long long)p->N, H, W);
  hipStream_t st = (hipStream_t)stream;
  return opt.prec == SDL_FP64 ? patches_to_image_impl<double>(&q, H, W, opt, image, st)
                              : patches_to_image_impl<float>(&q, H, W, opt, image, st);
}

int sdl_tensor_sparse_code(const sdl_tensor_problem* p, const sdl_options* o, void* stream) {
  g_err.clear();
  Opt opt = resolve(o);
  SDL_TRY(validate_tensor(p, opt, false));
  hipStream_t st = (hipStream_t)stream;
  return opt.prec == SDL_FP64 ? tensor_impl<double>(p, 0, 0, 0, nullptr, opt, st)
                              : tensor_impl<float>(p, 0, 0, 0, nullptr, opt, st);
}

int sdl_tensor_update(const sdl_tensor_problem* p, int32_t mode, const sdl_options* o, void* stream) {
  g_err.clear();
  Opt opt = resolve(o);
  SDL_TRY(validate_tensor(p, opt, true));
  if (mode < 1 || mode > p->nmodes) return fail(SDL_E_INVAL, "mode = %d (1..%d)", mode, p->nmodes);
  hipStream_t st = (hipStream_t)stream;
  return opt.prec == SDL_FP64 ? tensor_impl<double>(p, 1, mode - 1, 0, nullptr, opt, st)
                              : tensor_impl<float>(p, 1, mode - 1, 0, nullptr, opt, st);
}

int sdl_tensor_learn(const sdl_tensor_problem* p, int32_t K, double* rmse_trace, const sdl_options* o,
                     void* stream) {
  g_err.clear();
  Opt opt = resolve(o);
  SDL_TRY(validate_tensor(p, opt, true));
  if (K < 0) return fail(SDL_E_INVAL, "K = %d < 0", K);
  if (p->N > 0 && !p->res2) return fail(SDL_E_INVAL, "sdl_tensor_learn needs res2");
  hipStream_t st = (hipStream_t)stream;
  return opt.prec == SDL_FP64 ? tensor_impl<double>(p, 2, 0, K, rmse_trace, opt, st)
                              : tensor_impl<float>(p, 2, 0, K, rmse_trace, opt, st);
}

int sdl_mixed_supported(int32_t m1, int32_t m2, int32_t n1, int32_t n2, int32_t s) {
  return omp_mixed_supported(m1, m2, n1, n2, s) ? 1 : 0;
}

int sdl_workspace_bytes(const sdl_problem* p, int32_t nprob, int32_t call, int32_t K, const sdl_options* o,
                        size_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(SDL_E_INVAL, "bytes is NULL");
  Opt opt = resolve(o);
  SDL_TRY(validate(p, nprob, opt, false));
  if (call < 0 || call > 3) return fail(SDL_E_INVAL, "call = %d (0..3)", call);
  if (K < 0) return fail(SDL_E_INVAL, "K = %d < 0", K);
  if (call == 3 && nprob != 1) return fail(SDL_E_INVAL, "sdl_sparse_code_sums takes one problem");
  Plan pl;
  layout(p, nprob, opt.prec == SDL_FP64 ? 8 : 4, call == 2 ? K : 0, nullptr, &pl);
  *bytes = pl.bytes;
  return SDL_OK;
}

int sdl_sparse_code(const sdl_problem* p, int32_t nprob, const sdl_options* o, void* stream) {
  g_err.clear();
  Opt opt = resolve(o);
  SDL_TRY(validate(p, nprob, opt, false));
  SDL_TRY(check_workspace(p, nprob, 0, opt));
  hipStream_t st = (hipStream_t)stream;
  return opt.prec == SDL_FP64 ? sparse_code_impl<double>(p, nprob, opt, st) : sparse_code_impl<float>(p, nprob, opt, st);
}

int sdl_tmod_update(sdl_problem* p, int32_t nprob, uint32_t sides, const sdl_options* o, void* stream) {
  g_err.clear();
  Opt opt = resolve(o);
  SDL_TRY(validate(p, nprob, opt, true));
  if (sides < 1 || sides > 3) return fail(SDL_E_INVAL, "sides = %u (1, 2 or 3)", sides);
  SDL_TRY(check_workspace(p, nprob, 0, opt));
  hipStream_t st = (hipStream_t)stream;
  return opt.prec == SDL_FP64 ? tmod_update_impl<double>(p, nprob, sides, opt, st)
                              : tmod_update_impl<float>(p, nprob, sides, opt, st);
}

int sdl_learn(sdl_problem* p, int32_t nprob, int32_t K, double* rmse_trace, const sdl_options* o, void* stream) {
  g_err.clear();
  Opt opt = resolve(o);
  SDL_TRY(validate(p, nprob, opt, false));
  SDL_TRY(validate_learned(p, nprob, opt));
  if (K < 0) return fail(SDL_E_INVAL, "K = %d < 0", K);
  SDL_TRY(check_workspace(p, nprob, K, opt));
  hipStream_t st = (hipStream_t)stream;
  return opt.prec == SDL_FP64 ? learn_impl<double>(p, nprob, K, rmse_trace, opt, st)
                              : learn_impl<float>(p, nprob, K, rmse_trace, opt, st);
}

int sdl_autotune(const sdl_problem* p, int32_t nprob, int32_t reps, const sdl_options* o, void* stream) {
  g_err.clear();
  Opt opt = resolve(o);
  SDL_TRY(validate(p, nprob, opt, false));
  if (reps < 1) return fail(SDL_E_INVAL, "reps = %d < 1", reps);
  SDL_TRY(check_workspace(p, nprob, 0, opt));
  if (opt.prec == SDL_FP64 || opt.prec == SDL_MIXED_BF16) return SDL_OK;  // FP32 register-resident kernels only
  hipStream_t st = (hipStream_t)stream;
  Ctx* ctx;
  SDL_TRY(get_ctx(st, &ctx));
  Plan pl;
  layout(p, nprob, sizeof(float), 0, nullptr, &pl);
  void* wsb = nullptr;
  SDL_TRY(acquire_ws(ctx, opt, pl.bytes, st, &wsb));
  layout(p, nprob, sizeof(float), 0, wsb, &pl);
  pl.ybf16 = opt.prec == SDL_BF16 || opt.prec == SDL_MIXED_BF16;
  std::vector<std::pair<int, int>> marks;
  Launcher L{st, false, ctx, &marks};
  SDL_TRY(begin_call(st, ctx, pl, nprob));
  for (int q = 0; q < nprob; ++q) {
    if (p[q].N == 0 || !omp_fast_supported<float>(p[q].m1, p[q].m2, p[q].n1, p[q].n2, p[q].s)) continue;
    SDL_TRY(run_prep<float>(p[q], pl.pb[q], L));
    OmpArgs<float> a = omp_args<float>(p[q], pl.pb[q], opt, pl);
    // timed as the learning loop runs it: with the D1-update sums epilogue
    a.sums_side = 1;
    a.sums_part = pl.pb[q].part;
    int id;
    double ms;
    HIP_TRY(autotune_problem(a, st, reps, &id, &ms));
    if (id >= 0 && omp_wave_supported(p[q].m1, p[q].m2, p[q].n1, p[q].n2, p[q].s)) {
      // the alternative path: one wave per signal, then the standalone D1-side sums
      OmpArgs<float> aw = omp_args<float>(p[q], pl.pb[q], opt, pl);
      const TmodArgs<float> ta = tmod_args<float>(1, p[q], pl.pb[q], pl);
      double wms = 0.0;
      SDL_TRY(time_median(st, reps, &wms, [&]() -> hipError_t {
        hipError_t e = launch_omp_wave<float>(aw, st);
        return e != hipSuccess ? e : launch_tmod_sums<float>(ta, pl.pb[q].part, st);
      }));
      set_wave_choice(p[q].m1, p[q].m2, p[q].n1, p[q].n2, p[q].s, wms < ms, wms);
    }
  }
  HIP_TRY(hipStreamSynchronize(st));
  return SDL_OK;
}

int sdl_probe_hbm_copy(void* dst, const void* src, size_t bytes, int32_t reps, double* gbs, void* stream) {
  g_err.clear();
  if (!dst || !src || !gbs) return fail(SDL_E_INVAL, "NULL argument");
  if (bytes < 16 || reps < 1) return fail(SDL_E_INVAL, "need bytes >= 16 and reps >= 1");
  HIP_TRY(probe_hbm_copy(dst, src, bytes, reps, (hipStream_t)stream, gbs));
  return SDL_OK;
}

int sdl_probe_peak(int32_t kind, void* sink, int32_t reps, double* tflops, void* stream) {
  g_err.clear();
  if (!sink || !tflops) return fail(SDL_E_INVAL, "NULL argument");
  if (kind < 0 || kind > 6) return fail(SDL_E_INVAL, "kind = %d (0..6)", kind);
  if (reps < 1) return fail(SDL_E_INVAL, "reps = %d < 1", reps);
  HIP_TRY(probe_peak(kind, (float*)sink, reps, (hipStream_t)stream, tflops));
  return SDL_OK;
}

int sdl_tuned_config(int32_t m1, int32_t m2, int32_t n1, int32_t n2, int32_t s, int32_t* lanes_row,
                     int32_t* lanes_col, int32_t* waves_per_simd, int32_t* matrix_core, double* ms) {
  int lr = 0, lc = 0, wpe = 0, mf = 0;
  double t = 0.0;
  const bool fast = omp_fast_supported<float>(m1, m2, n1, n2, s);
  if ((!fast || wave_chosen(m1, m2, n1, n2, s)) && omp_wave_grid(m1, m2, n1, n2, s, &lr, &lc)) {
    mf = 2;  // standalone-sums path: one wave per signal, or four on matrix-core quadrants
    wpe = omp_quad_supported(m1, m2, n1, n2, s) ? 4 : 1;  // signals per wave
    t = wave_choice_ms(m1, m2, n1, n2, s);
  } else if (!tuned_config(m1, m2, n1, n2, s, &lr, &lc, &wpe, &mf, &t)) {
    return fail(SDL_E_UNSUPPORTED, "no register-resident kernel for this shape");
  }
  if (lanes_row) *lanes_row = lr;
  if (lanes_col) *lanes_col = lc;
  if (waves_per_simd) *waves_per_simd = wpe;
  if (matrix_core) *matrix_core = mf;
  if (ms) *ms = t;
  return SDL_OK;
}

int sdl_kernel_variants(int32_t m1, int32_t m2, int32_t n1, int32_t n2, int32_t s, int32_t* out, int32_t cap) {
  int ids[64];
  const int n = omp_fast_variants(m1, m2, n1, n2, s, ids, 64);
  for (int i = 0; i < n && i < cap && i < 64 && out; ++i)
    omp_fast_variant_info(ids[i], &out[4 * i], &out[4 * i + 1], &out[4 * i + 2], &out[4 * i + 3]);
  int lr, lc;
  if (!omp_wave_grid(m1, m2, n1, n2, s, &lr, &lc)) return n;
  if (out && n < cap) {
    out[4 * n] = lr;
    out[4 * n + 1] = lc;
    out[4 * n + 2] = omp_quad_supported(m1, m2, n1, n2, s) ? 4 : 1;  // signals per wave
    out[4 * n + 3] = 2;
  }
  return n + 1;
}

int sdl_set_kernel_variant(int32_t m1, int32_t m2, int32_t n1, int32_t n2, int32_t s, int32_t lanes_row,
                           int32_t lanes_col, int32_t waves_per_simd, int32_t matrix_core) {
  int ids[64];
  const int n = omp_fast_variants(m1, m2, n1, n2, s, ids, 64);
  for (int i = 0; i < n && i < 64; ++i) {
    int lr, lc, wpe, mf;
    omp_fast_variant_info(ids[i], &lr, &lc, &wpe, &mf);
    if (lr == lanes_row && lc == lanes_col && wpe == waves_per_simd && mf == matrix_core) {
      omp_fast_set_choice(m1, m2, n1, n2, s, ids[i]);
      set_wave_choice(m1, m2, n1, n2, s, false, 0.0);
      return SDL_OK;
    }
  }
  int lr, lc;
  if (matrix_core == 2 && omp_wave_grid(m1, m2, n1, n2, s, &lr, &lc) && lr == lanes_row && lc == lanes_col) {
    set_wave_choice(m1, m2, n1, n2, s, true, 0.0);
    return SDL_OK;
  }
  return fail(SDL_E_UNSUPPORTED, "no kernel variant (%d, %d, %d) for this shape", lanes_row, lanes_col,
              waves_per_simd);
}

int sdl_learned_sparse_code(sdl_proposer* P, const sdl_problem* p, int32_t nprob, int32_t* accept,
                            const sdl_options* o, void* stream) {
  g_err.clear();
  if (!P) return fail(SDL_E_INVAL, "proposer is NULL");
  Opt opt = resolve(o);
  opt.prec = SDL_FP32;
  opt.proposer = P;
  SDL_TRY(validate(p, nprob, opt, false));
  SDL_TRY(check_workspace(p, nprob, 0, opt));
  SDL_TRY(validate_learned(p, nprob, opt));
  if (accept && nprob != 1) return fail(SDL_E_INVAL, "accept needs nprob == 1");
  hipStream_t st = (hipStream_t)stream;
  Ctx* ctx;
  SDL_TRY(get_ctx(st, &ctx));
  Plan pl;
  layout(p, nprob, sizeof(float), 0, nullptr, &pl);
  void* wsb = nullptr;
  SDL_TRY(acquire_ws(ctx, opt, pl.bytes, st, &wsb));
  layout(p, nprob, sizeof(float), 0, wsb, &pl);
  pl.ybf16 = opt.prec == SDL_BF16 || opt.prec == SDL_MIXED_BF16;
  std::vector<std::pair<int, int>> marks;
  Launcher L{st, false, ctx, &marks};
  SDL_TRY(begin_call(st, ctx, pl, nprob));
  for (int q = 0; q < nprob; ++q) {
    if (p[q].N == 0) continue;
    SDL_TRY(run_prep<float>(p[q], pl.pb[q], L));
    // accepted and fallback counts accumulate in the call's device counters (read by finish_call)
    SDL_TRY(learned_code(P, p[q], opt.tau, accept, omp_args<float>(p[q], pl.pb[q], opt, pl), st, nullptr));
  }
  return finish_call(st, ctx, pl, opt, marks, opt.stats != nullptr);
}

int sdl_proposer_calibrate(sdl_proposer* P, const sdl_problem* prob, double violation, const sdl_options* opts,
                           double* tau_out, void* stream) {
  g_err.clear();
  if (!P || !prob || !tau_out) return fail(SDL_E_INVAL, "NULL argument");
  if (!(violation >= 0.0 && violation < 1.0)) return fail(SDL_E_INVAL, "violation must be in [0, 1)");
  const Opt copt = resolve(opts);
  if (!(copt.fallback_margin >= 1.0)) return fail(SDL_E_INVAL, "fallback_margin must be >= 1");
  const double margin = copt.fallback_margin;
  const sdl_problem& r = *prob;
  if (!r.res2) return fail(SDL_E_INVAL, "calibration needs res2");
  const int64_t N = r.N;
  hipStream_t st = (hipStream_t)stream;
  sdl_options o;
  sdl_default_options(&o);
  o.prec = SDL_FP32;
  o.tau = 1e300;  // accept every proposal: its residual is what we want
  SDL_TRY(sdl_learned_sparse_code(P, prob, 1, nullptr, &o, stream));
  std::vector<float> rp(N), ro(N), y((size_t)N * r.m1 * r.m2);
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipMemcpy(rp.data(), r.res2, sizeof(float) * N, hipMemcpyDeviceToHost));
  o.tau = 0.0;
  SDL_TRY(sdl_sparse_code(prob, 1, &o, stream));
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipMemcpy(ro.data(), r.res2, sizeof(float) * N, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(y.data(), r.Y, sizeof(float) * y.size(), hipMemcpyDeviceToHost));
  std::vector<std::pair<double, int>> q(N);
  for (int64_t k = 0; k < N; ++k) {
    double yy = 0.0;
    for (int e = 0; e < r.m1 * r.m2; ++e) yy += (double)y[k * r.m1 * r.m2 + e] * y[k * r.m1 * r.m2 + e];
    const double ratio = yy > 0 ? rp[k] / yy : 0.0;
    const int bad = (double)rp[k] > margin * (double)ro[k] ? 1 : 0;
    q[k] = {ratio, bad};
  }
  std::sort(q.begin(), q.end());
  double tau = 0.0;
  int64_t nbad = 0;
  for (int64_t i = 0; i < N; ++i) {
    nbad += q[i].second;
    if ((double)nbad <= violation * (double)(i + 1)) tau = q[i].first;
  }
  *tau_out = tau;
  return SDL_OK;
}

const char* sdl_last_error(void) { return g_err.c_str(); }

int sdl_abi_version(void) { return SDL_ABI_VERSION; }

}  // extern "C"
