/*
 * ttr.h -- tensor-train (TT) arithmetic on one AMD MI355X (gfx950).
 *
 * C ABI of libttr.so.  Every entry point takes plain host structs whose core
 * pointers are DEVICE pointers (HIP global memory on the handle's device), and
 * enqueues its kernels on the handle's HIP stream.  No torch or C++ types
 * appear here.  The operations are those of "Parallel Algorithms for Tensor
 * Train Arithmetic" (Al Daas, Ballard, Benner):
 *   sum (§3.2.1), Hadamard product (§3.2.2), inner product (§3.2.3, eq. (4)),
 *   norms (§3.2.4), orthonormalization (§2.3 Alg. 1; §3.4 Alg. 5) and
 *   rounding (§2.4 Alg. 2; §3.5 Alg. 6).
 *
 * TT layout (§2.1, §3.1).  A TT tensor has N cores; core n (0-based here,
 * n = 0..N-1) is an R[n] x I[n] x R[n+1] array of doubles with R[0] = R[N] = 1,
 * stored in the paper's "natural descending" order: entry (a, i, b) at offset
 *     a + R[n] * (i + I[n] * b).
 * Both the horizontal unfolding H (R[n] x I[n]R[n+1]) and the vertical
 * unfolding V (R[n]I[n] x R[n+1]) are then column-major views of the buffer.
 *
 * Ownership.  The library never frees caller memory and keeps no caller
 * pointer after a call returns.  It owns a device workspace attached to the
 * handle (allocated with hipMalloc on first need, grown on demand, released by
 * ttr_destroy).  A rounding at ranks above 64 also keeps the products
 * C_n = X_n T_{n+1} of its orthonormalization sweep for the truncation sweep
 * (about the size of X more device memory, held like the workspace) when
 * that allocation succeeds, and forms them again when it does not.  A handle
 * is bound to one device and one stream; use one handle per host thread.
 *
 * Errors.  Every call returns TTR_OK (0) or a TTR_ERR_* code and records a
 * message readable with ttr_last_error().  Argument errors are detected on the
 * host before any device work is enqueued.  Calls marked "synchronizes" wait
 * for the stream before returning.
 */
#ifndef TTR_H
#define TTR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum ttr_status {
  TTR_OK = 0,
  TTR_ERR_INVALID_ARG = 1,  /* NULL pointer, rank/size <= 0, R[0] or R[N] != 1, tol < 0 or NaN */
  TTR_ERR_SHAPE = 2,        /* operands disagree on N or mode sizes */
  TTR_ERR_CAPACITY = 3,     /* an output core's cap[] is smaller than what the result needs */
  TTR_ERR_ALLOC = 4,        /* workspace allocation failed */
  TTR_ERR_HIP = 5,          /* a HIP runtime call failed */
  TTR_ERR_NUMERICAL = 6,    /* non-finite data or a small factorization that did not converge */
  TTR_ERR_UNSUPPORTED = 7   /* a rank above the supported maximum (TTR_MAX_RANK) */
};

enum { TTR_RIGHT = 0, TTR_LEFT = 1 };             /* orthonormalization side (§2.3) */
/* rounding sweep order and orthonormal factors (§4.3.2): RLR / LRL keep the
 * first sweep's orthonormal factors implicit (§3.5 Alg. 6); the _EXPLICIT
 * variants write the orthonormal cores first (§3.4 Alg. 5) and truncate over
 * the written cores */
enum { TTR_RLR = 0, TTR_LRL = 1, TTR_RLR_EXPLICIT = 2, TTR_LRL_EXPLICIT = 3 };
enum { TTR_NORM_ORTHO = 0, TTR_NORM_GRAM = 1, TTR_NORM_SYM = 2 };    /* norm method (§3.2.4) */
enum { TTR_FP64 = 0, TTR_MIXED = 1 };              /* arithmetic of the Gram passes */

/* Largest TT rank of the register/LDS-tiled matrix-core kernels.  Every entry
 * point accepts it; ttr_norm(TTR_NORM_SYM), ttr_dot_noalloc and
 * ttr_round_batched stop there (ttr_add, ttr_hadamard and ttr_apply_kron
 * state their own limits). */
#define TTR_MAX_RANK 64
/* Largest rank of ttr_round (every direction, TTR_FP64 and TTR_MIXED),
 * ttr_dot, ttr_norm (TTR_NORM_ORTHO, TTR_NORM_GRAM) and ttr_orthogonalize:
 * ranks 65..256 take the GEMM-shaped matrix-core path (one unfolding times a
 * small matrix per product, Gram matrices of whole unfoldings). */
#define TTR_MAX_RANK_LARGE 256

/* A TT tensor.  All arrays are HOST memory; core[n] are DEVICE pointers.
 *   N      number of cores (>= 1)
 *   I      N mode sizes (> 0)
 *   R      N+1 ranks; R[0] = R[N] = 1.  Output tensors get R overwritten.
 *   core   N device pointers, core n holding R[n]*I[n]*R[n+1] doubles
 *   cap    N capacities in doubles of the output cores (ignored for inputs,
 *          may be NULL there). */
typedef struct ttr_tt {
  int32_t N;
  const int64_t *I;
  int64_t *R;
  double **core;
  const int64_t *cap;
} ttr_tt;

typedef struct ttr_handle ttr_handle;

/* Creates a handle on HIP device `device` that enqueues on `stream`
 * (a hipStream_t passed as void*; NULL = the device's null stream). */
int ttr_create(ttr_handle **h, int device, void *stream);
int ttr_destroy(ttr_handle *h);
int ttr_set_stream(ttr_handle *h, void *stream);

/* Routes the handle's device workspaces (Gram partials, small factors,
 * materialized cores, the batched plan, the rank 65..256 scratch) through a
 * caller allocator, e.g. a framework's caching allocator: alloc(bytes, ctx)
 * returns device memory on the handle's device or NULL (the call that needed
 * it then fails with TTR_ERR_ALLOC); free(ptr, ctx) takes back what alloc gave.
 * Both NULL restores hipMalloc / hipFree.  Synchronizes the stream and returns
 * the current workspaces to the allocator they came from first, so memory is
 * never freed through the wrong one.  Memory is requested when a call needs
 * more than the handle holds and kept until the next larger request, this
 * call, or ttr_destroy.
 * Errors: TTR_ERR_INVALID_ARG if exactly one of alloc / free is NULL. */
int ttr_set_allocator(ttr_handle *h, void *(*alloc)(size_t bytes, void *ctx), void (*free)(void *ptr, void *ctx),
                      void *ctx);

/* Z = alpha*X + beta*Y, slice-wise (§3.2.1): first core [alpha X_1, beta Y_1],
 * interior slices blockdiag(X_n(i), Y_n(i)) with the X block first, last core
 * [X_N; Y_N]; ranks add.  For N = 1 the single core is alpha X_1 + beta Y_1.
 * Z's cores must not alias X's or Y's.  Z->R is written.  Asynchronous. */
int ttr_add(ttr_handle *h, double alpha, const ttr_tt *X, double beta, const ttr_tt *Y, ttr_tt *Z);

/* Z = X .* Y, slice-wise Kronecker products (§3.2.2):
 * Z_n(i) = X_n(i) (x) Y_n(i), row (a_x, a_y) -> a_x*R^Y + a_y, same for columns;
 * ranks multiply.  Z->R is written.  Asynchronous. */
int ttr_hadamard(ttr_handle *h, const ttr_tt *X, const ttr_tt *Y, ttr_tt *Z);

/* Matrix-vector product with a Kronecker product of matrices (§3.2.5):
 * vec(Y) = (A_1 (x) ... (x) A_N) vec(X), computed core by core as the mode-2
 * products Y_n(a, :, b) = A_n X_n(a, :, b); ranks are unchanged (Y->R = X->R).
 * A_n (I_n x I_n) is given in band storage with kl[n] sub- and ku[n]
 * super-diagonals: A_n(i, j) = A[n][(ku[n] + i - j) + (kl[n] + ku[n] + 1) j]
 * for max(0, j - ku[n]) <= i <= min(I_n - 1, j + kl[n]) (a dense A_n is the
 * band kl = ku = I_n - 1, whose cost grows with I_n^2).  A: N DEVICE pointers
 * (array in host memory); kl, ku: host arrays.  Y's cores need
 * cap[n] >= R[n] I[n] R[n+1] of X and must not alias X's.  Left ranks up to
 * 4096.  A sum of Kronecker products is applied term by term, then summed with
 * ttr_add and rounded with ttr_round.  Asynchronous. */
int ttr_apply_kron(ttr_handle *h, const double *const *A, const int64_t *kl, const int64_t *ku, const ttr_tt *X,
                   ttr_tt *Y);

/* *out = <X, Y> by the recursion W_n = sum_i Y_n(i)^T W_{n-1} X_n(i), W_0 = 1
 * (§3.2.3, eq. (4)).  `out` is host memory.  Ranks <= TTR_MAX_RANK_LARGE.
 * Synchronizes. */
int ttr_dot(ttr_handle *h, const ttr_tt *X, const ttr_tt *Y, double *out);

/* ttr_dot for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and summation order as ttr_dot, so the same value bit for bit,
 * but it allocates nothing and does not synchronize.  The partial sums live
 * in a fixed device array of the library (512 * 64 * 64 + 2 * 64 * 64
 * doubles, about 16.8 MB), one copy per device, held until the process ends.
 *   out_dev  DEVICE pointer to one double on the handle's device; receives
 *            <X, Y> when the stream reaches the end of the call.
 * Ranks <= TTR_MAX_RANK (TTR_ERR_UNSUPPORTED above, or if a step's partial
 * sums would not fit the array).  Every call on one device uses that
 * device's array and leaves it holding the last call's partial sums: calls
 * that overlap on one device (other streams or handles) race. */
int ttr_dot_noalloc(ttr_handle *h, const ttr_tt *X, const ttr_tt *Y, double *out_dev);

/* *out = ||X|| (§3.2.4).  TTR_NORM_GRAM: sqrt(<X, X>) (fast; cancellation for
 * small norms of difference tensors).  TTR_NORM_SYM: the same quantity with the
 * symmetry of the inner-product matrices exploited: W_n = V(Z_n)^T V(Z_n) with
 * Z_n(i) = F X_n(i) and F^T F = W_{n-1} from a pivoted Cholesky (§3.2.4), made
 * upper triangular so half of each product is skipped; same cancellation as
 * GRAM.  TTR_NORM_ORTHO: right-orthonormalization sweep (implicit, X
 * untouched) then ||X_1||_F (§2.3; accurate for small norms).  Ranks <=
 * TTR_MAX_RANK_LARGE (TTR_NORM_SYM: <= TTR_MAX_RANK, TTR_ERR_UNSUPPORTED
 * above).  Non-finite data give NaN.  Synchronizes. */
int ttr_norm(ttr_handle *h, const ttr_tt *X, int method, double *out);

/* In-place orthonormalization (§2.3 Alg. 1; explicit factors as in §3.4 Alg. 5).
 * TTR_RIGHT: H(X_n) row-orthonormal for n >= 2 and core 1 carries the norm;
 * TTR_LEFT: V(X_n) column-orthonormal for n <= N-1 and core N carries the norm.
 * The factorizations reveal numerical rank: a link whose unfolding is
 * numerically rank-deficient (e.g. Y + Y) gets its numerical rank (the
 * number of singular values above rounding level of the unfolding being
 * factored), where a Householder QR would keep the formal rank with
 * rounding-level diagonal entries; X->R is updated and the tensor is
 * preserved to rounding error.  Ranks <= TTR_MAX_RANK_LARGE.  `prec` is
 * TTR_FP64.  Synchronizes. */
int ttr_orthogonalize(ttr_handle *h, ttr_tt *X, int side, int prec);

/* Y = rounding of X to relative accuracy tol (§2.4 Alg. 2): ||X - Y|| <= tol ||X||.
 * TTR_RLR: right-orthonormalization sweep (orthonormal factors kept implicit,
 * §3.5), threshold delta = tol ||X|| / sqrt(N-1), then left-to-right truncation
 * with the smallest rank whose Frobenius tail of singular values is <= delta;
 * output cores 1..N-1 are left-orthonormal.  TTR_LRL: the mirror image.
 * X is read only; Y's cores need cap[n] >= R[n]*I[n]*R[n+1] of X (always
 * enough, ranks never grow).  Ranks up to TTR_MAX_RANK_LARGE, every direction.
 * Y->R receives the new ranks; *norm_out (host, nullable) receives the ||X||
 * used for delta.  tol = 0 keeps every direction above rounding level, so a
 * numerically rank-deficient input (Y + Y) gets its numerical ranks, as in
 * ttr_orthogonalize; N = 1 copies.  `prec`: TTR_FP64 or TTR_MIXED.
 * Synchronizes. */
int ttr_round(ttr_handle *h, const ttr_tt *X, double tol, int direction, int prec,
              ttr_tt *Y, double *norm_out);

/* Y = rounding of the Hadamard product A * B (§3.2.2) to relative accuracy
 * tol, without forming A * B: the closing remark of §3.2.2 (keep the product
 * implicit for the rounding that follows).  The result is that of
 * ttr_hadamard followed by ttr_round(TTR_RLR): every product of a core of
 * A * B with a small matrix, (A_n(i) (x) B_n(i)) T, is formed from the
 * factors' slices (two 16 x 16 products per slice and column instead of one
 * with the Kronecker slice), and only the last core A_N (x) B_N is formed.
 * Ranks of A and B <= 16 (so ranks of A * B <= 256); direction TTR_RLR
 * (TTR_ERR_UNSUPPORTED otherwise); prec TTR_FP64 or TTR_MIXED.  Y's cores need
 * cap[n] >= R^A_n R^B_n I_n R^A_{n+1} R^B_{n+1}.  Synchronizes. */
int ttr_round_hadamard(ttr_handle *h, const ttr_tt *A, const ttr_tt *B, double tol, int direction, int prec,
                       ttr_tt *Y, double *norm_out);

/* Batched rounding (the batched form of §2.4 Alg. 2): Y[t] = rounding of X[t]
 * to relative accuracy tol[t], t = 0..count-1, for tensors of uneven mode
 * sizes and ranks that share the number of cores N (2 <= N <= 16), RLR order.
 * Arithmetic, accuracy and `prec` are those of ttr_round.  The decisions that
 * ttr_round takes on the host (ranks, whether a factorization has settled) are
 * taken on the device, so the whole call is one fixed sequence of batched
 * launches; it is captured once into a HIP graph and every later call with the
 * same arguments (pointers, shapes, tolerances) replays it with one launch.
 * Asynchronous: no host synchronization once the plan exists.
 *   ranks_dev  DEVICE array of count*(N+1) int64: the ranks of Y[t] at
 *              ranks_dev[t*(N+1) .. t*(N+1)+N]; ranks_dev[t*(N+1)] is -1 when a
 *              small factorization of tensor t failed (non-finite data).
 *              Y[t].R (host) is not written.
 *   tune       nonzero: when the plan is built, time the captured graph for a
 *              few slices-per-workgroup and grid-cap settings on this batch and
 *              keep the fastest (ttr_get_batch_plan reports them).
 * Building a plan allocates its device workspace and synchronizes; the plan
 * of the previous batch on the handle is released.  X and Y are not copied:
 * the graph reads and writes the given core pointers when replayed. */
int ttr_round_batched(ttr_handle *h, int count, const ttr_tt *X, const double *tol, int direction, int prec,
                      ttr_tt *Y, int64_t *ranks_dev, int tune);

typedef struct ttr_batch_plan {
  int32_t count;           /* tensors in the cached plan (0: none) */
  int32_t spw_target;      /* slices per workgroup chosen */
  int32_t grid_cap;        /* persistent grid cap chosen (0: one workgroup per item) */
  int32_t graph_nodes;     /* launches in the captured graph */
  int64_t workspace_bytes;
  int32_t candidates;      /* autotuner candidates timed */
  int32_t cand_spw[16];
  int32_t cand_grid[16];
  double cand_ms[16];      /* one replay of each candidate's graph */
} ttr_batch_plan;

int ttr_get_batch_plan(const ttr_handle *h, ttr_batch_plan *out);

const char *ttr_status_string(int status);
const char *ttr_last_error(void);

/* Per-call statistics of the last ttr_round on this handle (host memory):
 * number of streaming Gram passes, materialization passes, small-factorization
 * launches, and for each of the first TTR_STATS_LINKS links (physical link
 * order, link l between cores l and l+1):
 *   sigma     the singular values of the truncation step (descending, up to
 *             TTR_STATS_SIGMA, zero padded; all zero when the step proved that
 *             nothing can be dropped and skipped the SVD)
 *   nsigma    how many of them are nonzero
 *   tail2     the sum of squares of the singular values the truncation
 *             discarded (Alg. 2: sqrt(tail2) <= delta at every link, so
 *             sqrt(sum of tail2) <= tol ||X||)
 *   sweeps    Jacobi sweeps of the truncation SVD (0: no SVD was needed) */
#define TTR_STATS_LINKS 64
#define TTR_STATS_SIGMA 256
typedef struct ttr_round_stats {
  int32_t gram_passes;
  int32_t apply_passes;
  int32_t small_launches;
  int32_t links;
  double norm;
  double delta;
  double sigma[TTR_STATS_LINKS * TTR_STATS_SIGMA];
  int32_t nsigma[TTR_STATS_LINKS];
  double tail2[TTR_STATS_LINKS];
  int32_t sweeps[TTR_STATS_LINKS];
} ttr_round_stats;

int ttr_get_round_stats(const ttr_handle *h, ttr_round_stats *out);

/* Opt-in kernel timing.  With profiling on, every streaming launch made by the
 * handle is bracketed by HIP events on the handle's stream and its duration,
 * count and algorithmic traffic/work are accumulated per kernel:
 *   0 k_gram_right_factor  Gram pass with a right factor (orthonormalization)
 *   1 k_gram_left_factor   Gram pass with a left factor (truncation)
 *   2 k_gram               staged generic Gram pass (longer factor chains)
 *   3 k_apply_mfma         output pass, matrix cores
 *   4 k_apply              staged generic output pass
 *   5 k_add  6 k_hadamard  7 k_dot (inner-product steps)  8 small one-workgroup kernels
 *   9 k_gram_fac           refinement Gram pass on a materialized core
 *  10 k_apply_fac2         output pass with two right factors (refined core)
 *  11 k_gram_right_factor  as 0, FP32 matrix cores (TTR_MIXED first pass)
 *  12 k_gram_left_factor   as 1, FP32 matrix cores (TTR_MIXED first pass)
 *  13 k_kron_apply         mode-2 products of ttr_apply_kron (bytes: core
 *                          read + written, band read; flops: 2 per band entry
 *                          and output)
 * Gram passes: bytes = the core read once, flops = the slice products plus the
 * symmetric Gram accumulation; output passes: bytes = core read + output
 * written, flops = the slice products; sum/Hadamard: bytes = inputs read +
 * output written.  Durations are resolved at the end of each synchronizing
 * call and by ttr_get_profile, which waits for the stream.
 * ttr_set_profiling(h, 1) also clears the accumulators. */
#define TTR_NPROF 14
typedef struct ttr_profile {
  int64_t count[TTR_NPROF];
  double ms[TTR_NPROF];
  double bytes[TTR_NPROF];
  double flops[TTR_NPROF];
} ttr_profile;

int ttr_set_profiling(ttr_handle *h, int on);
int ttr_get_profile(ttr_handle *h, ttr_profile *out);

#ifdef __cplusplus
}
#endif

#endif /* TTR_H */
