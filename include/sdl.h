/* sdl.h -- C ABI of the MI355X (gfx950) separable dictionary learning library.
 *
 * Method: C. Rusu, P. Irofti, "Efficient and Parallel Separable Dictionary
 * Learning" (arXiv:2007.03800).  N two-dimensional signals Y_k (m1 x m2) are
 * approximated as Y_k ~ D1 X_k D2^T with s-sparse X_k (n1 x n2) and unit-norm
 * atoms (eq. (1)).  Sparse coding is 2D-OMP (Sec. III, step 1); the dictionary
 * updates are the least-squares solutions of Corollary 1 (D1) and
 * Result 1 (D2) followed by normalisation; learning iterates them as in
 * Algorithm 1.
 *
 * Layout: every matrix is column-major (the paper's vec, Sec. I).
 *   signal k, pixel (i,j):  Y[k*m1*m2 + i + j*m1]
 *   D1 (m1 x n1): D1[p + i*m1];  D2 (m2 x n2): D2[q + j*m2]; always FP64 (master copy)
 *   atom index a = i + n1*j, the column of D2 (x) D1 that multiplies vec X_k
 *   supp[k*s + t]: t-th atom chosen for signal k (selection order), -1 = unused slot
 *   coef[k*s + t]: its coefficient, 0 in unused slots
 * Element type of Y, coef and res2: double for SDL_FP64, float for SDL_FP32; for
 * SDL_BF16 and SDL_MIXED_BF16 Y holds bfloat16 values (16-bit patterns equal to the upper
 * half of the FP32 encoding) and coef/res2 are float.
 *
 * Pointers: every array pointer is a DEVICE pointer (HIP global memory) unless
 * marked "host".  The caller allocates and owns all of them and keeps them alive
 * until the work queued on `stream` has completed.  The library owns only its
 * internal workspace (allocated on first use per device and stream, grown on
 * demand, released at process exit).  Calls that share a stream are ordered;
 * calls on different streams must not share output buffers.
 *
 * Errors: nothing is thrown across this ABI.  Arguments are validated before any
 * work is queued; a negative status is returned and sdl_last_error() gives a
 * thread-local message.  SDL_E_SINGULAR (a dictionary update whose Gram sum is
 * not positive definite) leaves that dictionary unchanged and is reported after
 * the remaining work has run.
 */
#ifndef SDL_H
#define SDL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SDL_ABI_VERSION 9

/* SDL_FP64, SDL_FP32: the signals and every step in that precision (dictionary solves in FP64).
 * SDL_BF16: bfloat16 signals widened to FP32 where loaded; every step as SDL_FP32.
 * SDL_MIXED_BF16: bfloat16 signals; the correlations D1^T R_k D2 of every 2D-OMP step are
 *   contractions on the BF16 matrix cores with FP32 accumulation, every atom whose BF16
 *   |correlation| lies within tie_band (relative) of the largest is re-scored in FP32 before
 *   the pick, the residual, the chosen atom's correlation and the Cholesky factor are FP32, and
 *   the dictionary sums and solves are as for SDL_BF16.  Shapes: see sdl_mixed_supported. */
typedef enum { SDL_FP64 = 0, SDL_FP32 = 1, SDL_BF16 = 2, SDL_MIXED_BF16 = 3 } sdl_prec;

enum {
  SDL_OK = 0,
  SDL_E_INVAL = -1,       /* null pointer, bad enum, negative count */
  SDL_E_SHAPE = -2,       /* s > n1*n2, s > m1*m2, non-positive or too large sizes */
  SDL_E_DEVICE = -3,      /* a HIP call failed (message holds hipGetErrorString) */
  SDL_E_NOMEM = -4,       /* workspace allocation failed */
  SDL_E_SINGULAR = -5,    /* update Gram sum not positive definite; dictionary kept */
  SDL_E_NONFINITE = -6,   /* check_finite found NaN/Inf in Y or a dictionary */
  SDL_E_UNSUPPORTED = -7  /* valid but not supported by this library (see message) */
};

/* Limits of this library (per problem). */
#define SDL_MAX_M 64      /* m1, m2 */
#define SDL_MAX_N 64      /* n1, n2 */
#define SDL_MAX_S 32      /* s */
#define SDL_ORTHO_MAX_N 32  /* orthonormal variant (method 1): m1, m2 <= 32 and m1*m2 <= 256 */

/* One dictionary problem; an array of them is one (possibly uneven) batch. */
typedef struct sdl_problem {
  int32_t m1, m2, n1, n2, s;
  int32_t reserved;       /* must be 0 */
  int64_t N;              /* number of signals, >= 0 */
  const void* Y;          /* N*m1*m2 elements */
  double* D1;             /* m1*n1, unit-norm columns; input (sparse_code), in/out (update, learn) */
  double* D2;             /* m2*n2 */
  int32_t* supp;          /* N*s, output (sparse_code, learn), input (tmod_update) */
  void* coef;             /* N*s, output; rescaled in place by tmod_update */
  void* res2;             /* N, ||Y_k - D1 X_k D2^T||_F^2, output; may be NULL */
} sdl_problem;

/* Counters and timings filled when sdl_options.stats is set (host memory). */
typedef struct sdl_stats {
  int64_t early_stops;      /* signals that ended with fewer than s atoms */
  int64_t fp64_pivots;      /* FP32 path: Cholesky rows recomputed in FP64 (small pivot) */
  int64_t unused_atoms;     /* atoms kept unchanged because no code used them */
  int64_t singular_updates; /* dictionary updates skipped as not positive definite */
  /* Per-kernel device time when sdl_options.timing = 1, measured with HIP events on
   * the call's stream.  Index: 0 sparse coding (on the FP32 register-resident path it
   * also accumulates the next update's sums), 1 standalone TMOD sums, 2 fixed-order
   * reduction, 3 FP64 solve + normalise, 4 dictionary prep, 5 RMSE, 6 code rescale. */
  double kernel_ms[8];
  int64_t kernel_launches[8];
  int64_t proposals_accepted; /* learned path: signals whose proposal passed the test */
  int64_t fallbacks;          /* learned path: signals coded by the 2D-OMP fallback */
  int64_t near_tie_rescores;  /* SDL_MIXED_BF16: greedy steps (summed over signals) whose pick was
                                 decided among more than one candidate re-scored in FP32 */
  int64_t near_tie_overflows; /* SDL_MIXED_BF16: greedy steps where some lane of the signal had its
                                 second-largest BF16 |correlation| inside the band, so a third one of that
                                 lane, if also inside, was not re-scored (an upper bound on such misses) */
} sdl_stats;

/* Learned support proposal network (opaque; see sdl_proposer_* below). */
typedef struct sdl_proposer sdl_proposer;

typedef struct sdl_options {
  int32_t prec;             /* sdl_prec, default SDL_FP64 */
  int32_t schedule;         /* sdl_learn: 0 = Algorithm 1 (OMP, D1, OMP, D2), 1 = (OMP, D2, D1) */
  int32_t use_graph;        /* sdl_learn: replay one iteration as a HIP graph (default 1) */
  int32_t check_finite;     /* scan Y and dictionaries for NaN/Inf first (default 0) */
  int32_t timing;           /* fill stats->kernel_ms (eager launches with events; default 0) */
  int32_t kernel;           /* sparse-coding kernel: 0 auto, 1 generic, 2 register-resident multi-signal
                               (FP32), 3 register-resident with standalone sums (large shapes: one wave
                               per signal, or in FP32 four signals per wave on matrix-core quadrants
                               where compiled); auto picks 2, then 3, then 1, as compiled for the shape
                               and as the autotuner measured */
  double stop_rel;          /* OMP stops when max |corr| <= stop_rel*||Y_k||_F; default 1e-14 (FP64), 1e-6 (FP32) */
  double dep_eps;           /* OMP stops when the new Gram pivot <= dep_eps*G_aa; default 1e-10 */
  double pivot_fp64;        /* FP32: pivots below pivot_fp64*G_aa are recomputed in FP64; default 1e-3 */
  sdl_stats* stats;         /* host, optional */
  sdl_proposer* proposer;   /* sdl_learn: code with the learned proposal + 2D-OMP fallback (NULL = plain) */
  double tau;               /* acceptance threshold of the proposal: ||r||^2 <= tau*||Y||^2 (default 0) */
  double err2;              /* error-driven stop of the denoising experiments (Sec. IV): before each
                               greedy step, a signal whose residual energy ||Y_k - D1 X_k D2^T||_F^2 is
                               <= err2 takes no further atom; s stays the cap (the paper uses
                               eps = 1.15 sigma sqrt(m1 m2), err2 = eps^2, s = m1 m2 / 2).  0 = off
                               (default); negative or NaN: SDL_E_INVAL.  Runs on the one-wave-per-signal
                               kernel where one is compiled for the shape (among them the denoising
                               shapes 8x8 with 16x16 or 8x8 atoms at s = 32) and otherwise on the generic
                               kernel; kernel 2, kernel 3 without such a kernel, or a learned proposal,
                               with err2 > 0 is SDL_E_UNSUPPORTED */
  double tie_band;          /* SDL_MIXED_BF16: atoms whose BF16 |correlation| is at least (1 - tie_band) times
                               the largest are re-scored in FP32 and the pick is the largest FP32 |correlation|
                               among them (ties: smallest atom).  Default 2^-6; must be in [0, 0.5) */
  double fallback_margin;   /* learned proposal: sdl_proposer_calibrate counts a calibration signal as a
                               violation when its proposal's ||r||^2 exceeds fallback_margin times plain
                               2D-OMP's (default 1.01: "more than 1% worse"); must be >= 1 */
  int32_t deterministic;    /* 1 (default): results are bitwise reproducible run to run for the same inputs,
                               launch configuration and device.  Every path of this library already is (the
                               sums use fixed-order FP64 reductions and no floating-point atomics), so 0 is
                               accepted and gives the same results */
  int32_t reserved0;        /* must be 0 */
  void* workspace;          /* device memory the call uses instead of the library's own workspace (NULL: the
                               library allocates and keeps one per device and stream).  At least
                               sdl_workspace_bytes() bytes, 256-byte aligned, owned by the caller, not used by
                               calls that may overlap in time; its contents need not be preserved between calls.
                               Too small: SDL_E_NOMEM before any work is queued */
  size_t workspace_bytes;   /* size of workspace in bytes */
  int32_t method;           /* 0 (default): the general method (2D-OMP codes, least-squares dictionary updates).
                               1: the orthonormal variant of Remark 1 for square dictionaries with orthonormal
                               columns (n1 = m1, n2 = m2; SDL_ORTHO_MAX_N): sdl_sparse_code keeps the s entries of
                               D1^T Y_k D2 of largest magnitude (ties: smaller atom; listed in decreasing
                               magnitude; res2 from the explicit residual); sdl_tmod_update replaces D1 by the
                               orthogonal Procrustes solution U V^T of sum_k Y_k D2 X_k^T = U S V^T (D2 likewise from
                               sum_k Y_k^T D1 X_k; FP64 one-sided Jacobi SVD; the codes are not rescaled; a rank-
                               deficient sum leaves the dictionary and reports SDL_E_SINGULAR); sdl_learn iterates
                               these as Algorithm 1 does.  Reading of the paper's printed update, which multiplies
                               the sum by sum_k X_k X_k^T before the SVD: the polar factor of the sum alone, the
                               minimiser of eq. (1) over orthonormal dictionaries for fixed codes.  FP32 or FP64;
                               the caller's dictionaries must be orthonormal */
  int32_t reserved1;        /* must be 0 */
} sdl_options;

/* Fill *o with the defaults above (prec = SDL_FP64).  Passing NULL options to the
 * calls below means these defaults. */
void sdl_default_options(sdl_options* o);

/* 2D-OMP sparse coding (Sec. III step 1; 2D-OMP equals OMP on D2 (x) D1, Sec. II):
 * for every signal, s greedy steps choose the atom whose correlation with the
 * residual is largest in magnitude (ties: smallest a), then re-fit all chosen
 * coefficients by least squares.  Writes supp, coef, res2.  Asynchronous on
 * `stream` (a hipStream_t; NULL = default stream). */
int sdl_sparse_code(const sdl_problem* p, int32_t nprob, const sdl_options* o, void* stream);

/* TMOD dictionary update(s) from the codes in supp/coef (Algorithm 1 steps 2 and
 * 4; Corollary 1 for D1, Result 1 for D2).  sides: 1 = D1, 2 = D2, 3 = D1
 * then D2.  For each side: partial sums over all signals, FP64 solve on the
 * atoms used by some code, unit-norm normalisation, and rescaling of coef so
 * every product D1 X_k D2^T is unchanged.  Synchronises `stream` before
 * returning the status. */
int sdl_tmod_update(sdl_problem* p, int32_t nprob, uint32_t sides, const sdl_options* o, void* stream);

/* Algorithm 1: K iterations of (2D-OMP, D1 update, 2D-OMP, D2 update), then a
 * final 2D-OMP whose codes are returned in supp/coef/res2.  rmse_trace (host,
 * nprob*(K+1) doubles, may be NULL): for problem q, entry q*(K+1)+t is
 * sqrt(sum_k res2_k / (N*m1*m2)) of the 2D-OMP at the start of iteration t
 * (t = K: the final one).  D1, D2 are updated in place.  Synchronises. */
int sdl_learn(sdl_problem* p, int32_t nprob, int32_t K, double* rmse_trace, const sdl_options* o,
              void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): sdl_sparse_code with the same arguments, results and
 * kernels, whose workspace (status word, counters, compute-type dictionary copies and Gram
 * matrices) lives in a static device array of SDL_NOALLOC_SCRATCH_BYTES inside the library
 * instead of allocated memory.  It calls no hipMalloc/hipFree or other allocating routine; each
 * GPU the library runs on holds its own array until the process ends, set up on the first call on
 * that device.  Every call on a GPU shares that GPU's array: calls that overlap in time on one GPU
 * (other streams, other threads) race and must not be issued.  Each problem takes
 * (m1 n1 + m2 n2) e + (n1^2 + n2^2)(8 + e) bytes of the array (e = 8 for SDL_FP64, else 4, each
 * piece rounded up to 256 bytes; at most 192 KiB for the largest FP64 shape), plus about 1 KiB per
 * call; problems that do not fit are refused with SDL_E_NOMEM before any work is queued.
 * options->timing and options->workspace must be 0 / NULL (SDL_E_INVAL).  Asynchronous on
 * `stream` unless stats are requested. */
#define SDL_NOALLOC_SCRATCH_BYTES (1u << 20)
int sdl_sparse_code_noalloc(const sdl_problem* p, int32_t nprob, const sdl_options* o, void* stream);

/* The work of one node of Algorithm 1 in its step 1 (side 1) or step 3 (side 2): 2D-OMP of the
 * problem's signals as sdl_sparse_code does it (supp, coef and res2 written), then the sums that
 * node sends to the master, formed from the new codes:
 *   side 1 (Corollary 1):  T_k = X_k D2^T,  A = sum_k T_k T_k^T (n1 x n1),  B = sum_k Y_k T_k^T (m1 x n1)
 *   side 2 (Result 1):     Z_k = D1 X_k,    A = sum_k Z_k^T Z_k (n2 x n2),  B = sum_k Y_k^T Z_k (m2 x n2)
 * and the total squared residual sum_k res2_k.  sums (device, FP64, na*na + mr*na + 1 doubles with
 * na = n1, mr = m1 for side 1 and na = n2, mr = m2 for side 2): A column-major at sums[0], B
 * column-major at sums[na*na], the residual total last.  The sums are the ones sdl_learn solves:
 * on the register-resident FP32/BF16 kernels they are accumulated in the sparse-coding launch
 * itself (FP32 products, FP64 across workgroups), otherwise by the standalone sums kernel after
 * it; every reduction has a fixed order.  One problem; res2 must not be NULL.  On one GPU this is
 * what each GPU of a multi-GPU run would contribute to an all-reduce before the solve.
 * Asynchronous on `stream`. */
int sdl_sparse_code_sums(const sdl_problem* p, int32_t side, double* sums, const sdl_options* o, void* stream);

/* Device workspace bytes a call of kind `call` (0 sdl_sparse_code, 1 sdl_tmod_update,
 * 2 sdl_learn with K iterations, 3 sdl_sparse_code_sums) on these problems with these options
 * needs when sdl_options.workspace is given (the size the library would allocate itself).
 * Host only: queues no device work. */
int sdl_workspace_bytes(const sdl_problem* p, int32_t nprob, int32_t call, int32_t K, const sdl_options* o,
                        size_t* bytes);

/* 1 if SDL_MIXED_BF16 has a kernel for this shape (signal rows and columns and atom counts
 * multiples of 4 within the compiled set), else 0. */
int sdl_mixed_supported(int32_t m1, int32_t m2, int32_t n1, int32_t n2, int32_t s);

/* Denoising driver of the experiments in Sec. IV (overlapping patches of a noisy image coded by the
 * error-driven 2D-OMP, then put back together).  Step 1: all (H-m1+1)(W-m2+1) overlapping m1 x m2
 * patches of an H x W image (row-major, pixel (y, x) at y*W + x), stride 1, as signals in the layout
 * above: patch k = r*(W-m2+1) + c holds pixel (r+i, c+j) at its (i, j).  prec: SDL_FP32 or SDL_FP64,
 * the element type of both arrays (device pointers; patches holds (H-m1+1)(W-m2+1)*m1*m2 elements).
 * Asynchronous on `stream`.  Step 2 is sdl_sparse_code with options->err2 (eps^2) and s as the cap. */
int sdl_image_to_patches(const void* image, int32_t H, int32_t W, int32_t m1, int32_t m2, int32_t prec,
                         void* patches, void* stream);
/* Step 3: the H x W image rebuilt from the codes of those patches (p: m1, m2, n1, n2, s, D1, D2, supp,
 * coef and N = (H-m1+1)(W-m2+1); Y and res2 unused): every pixel is the plain average, over the patches
 * covering it, of D1 X_k D2^T at that pixel (a reading: the paper does not say how overlapping
 * estimates are combined).  options->prec (SDL_FP32 or SDL_FP64) is the type of coef and image.
 * Unused support slots (-1) may sit anywhere in a code.  The estimates are formed on chip, pixel
 * by pixel, and never stored: with options->workspace that buffer must hold what
 * sdl_workspace_bytes reports for sparse coding (call 0) of p (SDL_E_NOMEM otherwise).
 * Asynchronous on `stream`. */
int sdl_patches_to_image(const sdl_problem* p, int32_t H, int32_t W, const sdl_options* o, void* image,
                         void* stream);

/* n-dimensional signals (Remark 3).  A signal is a tensor Y_k of m[0] x ... x m[nmodes-1] entries,
 * stored first index fastest; the dictionary is separable over the modes, Y_k ~ X_k x_1 D_1 ... x_n
 * D_n with D_d (m[d] x n[d], column-major FP64, caller-owned, updated in place), so that it acts on
 * vec(Y_k) as D_n (x) ... (x) D_1 and atom a = i_0 + n[0] (i_1 + n[1] (i_2 + ...)).  Entries of m,
 * n and D beyond nmodes are ignored.  supp/coef/res2 as for sdl_problem (coef and res2 in the
 * element type of Y). */
#define SDL_TENSOR_MAX_MODES 4
#define SDL_TENSOR_MAX_ELEMS 4096 /* largest prod m[d] and prod n[d] */
typedef struct {
  int32_t nmodes; /* 2 .. SDL_TENSOR_MAX_MODES */
  int32_t s;      /* atoms per signal (cap) */
  int32_t m[SDL_TENSOR_MAX_MODES];
  int32_t n[SDL_TENSOR_MAX_MODES];
  int64_t N;
  const void* Y;
  double* D[SDL_TENSOR_MAX_MODES];
  int32_t* supp;
  void* coef;
  void* res2; /* optional for sdl_tensor_sparse_code, required by sdl_tensor_learn */
} sdl_tensor_problem;
/* Sparse coding of every signal by OMP on the Kronecker dictionary (Sec. II's equivalence, mode by
 * mode), with the stopping rules of sdl_sparse_code (stop_rel, dep_eps, pivot_fp64, err2).
 * options->prec: SDL_FP64 or SDL_FP32; kernel, method, schedule and proposer must be 0 and
 * workspace NULL (SDL_E_UNSUPPORTED otherwise).  Asynchronous unless stats is set. */
int sdl_tensor_sparse_code(const sdl_tensor_problem* p, const sdl_options* o, void* stream);
/* The update of mode `mode` (1..nmodes) from the codes in supp/coef (Remark 3: Corollary 1 with the
 * other modes' Kronecker product fixed): D_mode solves D A = B with A = sum_k W_k W_k^T,
 * B = sum_k Y_k(mode) W_k^T, W_k the mode-`mode` matricisation of X_k multiplied along every other
 * mode by its dictionary; atoms no code uses are kept; columns are normalised and the codes
 * rescaled.  SDL_E_SINGULAR leaves D unchanged.  Synchronous. */
int sdl_tensor_update(const sdl_tensor_problem* p, int32_t mode, const sdl_options* o, void* stream);
/* Algorithm 1 with one sweep per mode, K iterations: for each mode, sparse coding then that mode's
 * update; then a final sparse coding.  rmse_trace (host, optional, K + 1 values): the RMSE of each
 * iteration's first sweep and of the final one.  Synchronous. */
int sdl_tensor_learn(const sdl_tensor_problem* p, int32_t K, double* rmse_trace, const sdl_options* o,
                     void* stream);

/* Autotuner (no counterpart in the paper; a property of this GPU implementation):
 * for every FP32 problem whose shape has register-resident kernel variants
 * (different numbers of lanes per signal and register budgets), run each variant
 * `reps` times on the problem's own signals, timed with HIP events on `stream`
 * with the D1-update sums epilogue that sdl_learn fuses into the kernel, and keep
 * the fastest for all later calls in this process.  The problem's
 * supp/coef/res2 are overwritten with valid codes.  If the environment variable
 * SDL_TUNE_CACHE names a file, choices are loaded from it on first use and
 * appended after tuning.  FP64 problems and shapes without variants are skipped.
 * Synchronises. */
int sdl_autotune(const sdl_problem* p, int32_t nprob, int32_t reps, const sdl_options* o, void* stream);

/* Kernel configuration currently used for an FP32 shape: lanes per signal split
 * over atom rows (lanes_row) and columns (lanes_col), register budget in waves
 * per SIMD, the kind in matrix_core (0: multi-signal on the vector ALUs, 1: correlation
 * refresh on the matrix cores, 2: the standalone-sums path, whose dictionary sums run
 * in the standalone sums kernel: one wave per signal (in FP32 on 16x16 matrix-core tiles;
 * lanes_row x lanes_col is the lane grid of the FP64 form), or in FP32 at 12x12 signals
 * with 20x20 or 24x24 atoms four signals per wave on 4x4x1 matrix-core quadrants; for
 * kind 2 waves_per_simd reports the signals per wave, 1 or 4), and the tuned time in ms
 * (0 if not tuned; for kind 2
 * it includes the D1-side sums).  Returns 0 if the shape has a register-resident
 * kernel, SDL_E_UNSUPPORTED if it runs on the generic kernel.  The autotuner also times
 * kind 2 where it exists and keeps it if it beats the best fused variant. */
int sdl_tuned_config(int32_t m1, int32_t m2, int32_t n1, int32_t n2, int32_t s, int32_t* lanes_row,
                     int32_t* lanes_col, int32_t* waves_per_simd, int32_t* matrix_core, double* ms);

/* Register-resident kernel variants compiled for an FP32 shape: writes up to `cap`
 * quadruples (lanes_row, lanes_col, waves_per_simd, kind as in sdl_tuned_config) to out
 * (host, 4*cap int32) and returns how many exist (0: the shape runs on the generic kernel). */
int sdl_kernel_variants(int32_t m1, int32_t m2, int32_t n1, int32_t n2, int32_t s, int32_t* out, int32_t cap);

/* Force the variant used for an FP32 shape for the rest of the process (instead of
 * the autotuned or default one).  SDL_E_UNSUPPORTED if no such variant exists. */
int sdl_set_kernel_variant(int32_t m1, int32_t m2, int32_t n1, int32_t n2, int32_t s, int32_t lanes_row,
                           int32_t lanes_col, int32_t waves_per_simd, int32_t matrix_core);

/* ---- Learned support proposal (not part of the paper; an accelerator in front of 2D-OMP).
 * An MLP maps vec(Y_k)/||Y_k||_F (m1*m2 inputs) through two GELU layers of `hidden` units to
 * one logit per atom (n1*n2).  It is trained on the GPU by this library's own forward,
 * backward and Adam kernels with mean sigmoid cross-entropy against the supports that
 * 2D-OMP chose.  At inference the s largest logits (ties: smallest index) give the support,
 * least squares on it gives the coefficients and the explicit residual; the proposal is
 * accepted when ||r||^2 <= tau*||Y||^2, otherwise the signal is coded by 2D-OMP.
 * Supported: m1*m2 = 64, n1*n2 in {144, 256}, hidden a multiple of 64, s <= 16, FP32
 * signals; fp32_check = 1 runs the GEMMs in FP32 (for gradient checks), else BF16 with
 * FP32 accumulation.  Weights: FP32 masters, flat layout [W1 (hidden x m1m2, row = unit),
 * b1, W2 (hidden x hidden), b2, W3 (n1n2 x hidden), b3], seeded Kaiming-normal init.
 * Device pointers: Y (N x m1*m2 floats, column-major signals), supp (N x s int32),
 * logits (N x n1n2 floats), accept (N int32).  Calls are synchronous unless noted. */
int sdl_proposer_create(int32_t m1, int32_t m2, int32_t n1, int32_t n2, int32_t hidden, int32_t fp32_check,
                        uint64_t seed, sdl_proposer** out);
void sdl_proposer_destroy(sdl_proposer* p);
int64_t sdl_proposer_num_params(const sdl_proposer* p);
int sdl_proposer_get_params(const sdl_proposer* p, float* host);      /* np floats */
int sdl_proposer_set_params(sdl_proposer* p, const float* host);      /* also resets the Adam state */
/* Mean BCE loss and its gradient (host, np floats) on B signals (B % 64 == 0), no update. */
int sdl_proposer_gradient(sdl_proposer* p, const float* Y, const int32_t* supp, int32_t s, int64_t B,
                          float* grad_host, double* loss_host, void* stream);
/* Adam (lr, 0.9, 0.999, 1e-8) over `epochs` passes of floor(N/batch) shuffled batches;
 * loss_trace (host, epochs, may be NULL) gets each epoch's mean batch loss.  SDL_E_SHAPE
 * unless batch is a positive multiple of 64, batch <= N <= 2^31 - 1 and epochs >= 0. */
int sdl_proposer_train(sdl_proposer* p, const float* Y, const int32_t* supp, int32_t s, int64_t N, int32_t epochs,
                       int32_t batch, float lr, uint64_t seed, double* loss_trace, void* stream);
/* Logits of N signals (asynchronous on stream). */
int sdl_proposer_logits(sdl_proposer* p, const float* Y, int64_t N, float* logits, void* stream);
/* Learned sparse coding of FP32 problems (options->tau is the acceptance threshold):
 * proposal + least squares for every signal, register-resident 2D-OMP for the rejected
 * ones.  accept (device, N int32, may be NULL; only with nprob == 1) receives 1 where the
 * proposal was kept.  stats (if given) receives the accepted / fallback counts. */
int sdl_learned_sparse_code(sdl_proposer* p, const sdl_problem* prob, int32_t nprob, int32_t* accept,
                            const sdl_options* o, void* stream);
/* Choose tau on a calibration problem: run the proposal (accepting everything) and plain
 * 2D-OMP, sort signals by ||r_prop||^2/||Y||^2 and return the largest threshold such that at
 * most `violation` of the accepted signals have ||r_prop||^2 > m * ||r_omp||^2, with
 * m = o->fallback_margin (default 1.01; o may be NULL).  The problem's codes are overwritten. */
int sdl_proposer_calibrate(sdl_proposer* p, const sdl_problem* prob, double violation, const sdl_options* o,
                           double* tau_out, void* stream);

/* Save the network to a file: a fixed header (magic "SDLPROP1", m1, m2, n1, n2, hidden, fp32_check as
 * int32, the parameter count as int64) followed by the FP32 master weights in the flat layout above,
 * little-endian.  The Adam state is not saved.  SDL_E_INVAL for NULL arguments or an unwritable path. */
int sdl_proposer_save(const sdl_proposer* p, const char* path);
/* Create a network from a file written by sdl_proposer_save (weights restored, Adam state reset).
 * SDL_E_INVAL if the file cannot be read or is not such a file. */
int sdl_proposer_load(const char* path, sdl_proposer** out);

/* Measurement aids (no counterpart in the paper): achievable ceilings of the current
 * device, for quoting kernel fractions against measured as well as published peaks.
 * sdl_probe_hbm_copy copies bytes (rounded down to a multiple of 16) from src to dst
 * (device pointers, not overlapping, each at least `bytes` long) reps times with a
 * grid-stride kernel and stores the best rate, read plus write bytes, in *gbs (1e9 B/s).
 * sdl_probe_peak runs independent arithmetic chains on every SIMD and stores the best of
 * reps launches in *tflops: kind 0 = FP32 FMA on the vector ALUs (unpacked), 1 = FP32
 * MFMA 16x16x4, 2 = FP32 MFMA 4x4x1 (16 blocks), 3 = FP64 FMA, 4 = BF16 MFMA 4x4x4 (16 blocks),
 * 5 = BF16 MFMA 16x16x16, 6 = BF16 MFMA 16x16x32 (FP32 accumulation for 4-6).  sink: device, >= 8 bytes,
 * written only if a chain reaches a value it cannot reach.  Both synchronise the stream;
 * SDL_E_INVAL for NULL pointers, bytes < 16, reps < 1 or an unknown kind. */
int sdl_probe_hbm_copy(void* dst, const void* src, size_t bytes, int32_t reps, double* gbs, void* stream);
int sdl_probe_peak(int32_t kind, void* sink, int32_t reps, double* tflops, void* stream);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char* sdl_last_error(void);

/* SDL_ABI_VERSION of the built library. */
int sdl_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SDL_H */
