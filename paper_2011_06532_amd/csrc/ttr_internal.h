// Internal declarations shared by the host API and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define TTR_RMAX 64          // largest rank the small-matrix kernels hold in LDS
#define TTR_MAXWG 1024       // most workgroups a streaming pass uses (fixed-order reduction)

// Logical view of one core: slice M(i) is an ea x eb matrix.
//   trans = 0: M(r, c) = X(r, i, c) of a physical pa x I x pb core (ea = pa, eb = pb)
//   trans = 1: M(r, c) = X(c, i, r)                                 (ea = pb, eb = pa)
// Physical layout (a, i, b) -> a + pa*(i + I*b).
struct CoreView {
  const double *X;
  long long I;
  int pa, pb;
  int trans;
  __host__ __device__ int ea() const { return trans ? pb : pa; }
  __host__ __device__ int eb() const { return trans ? pa : pb; }
};

// Small dense transforms applied to every slice of a streaming pass, in
// stages: Z(i) = L_k ... L_1 M(i) R_1 ... R_m.  Left stages are applied first
// (in order), then right stages (in order), each product rounded on its own.
// Applying the factors of an ill-conditioned QR one stage at a time (rather
// than as one collapsed matrix), and identically in every pass that touches
// the same core, is what keeps the computed orthonormal factors orthonormal.
//   stage matrix S(r, c) = S[r*sr + c*sc]
//   left stage:  rows x (current rows) ;  right stage: (current cols) x cols
struct Stage {
  const double *S;
  int rows, cols;
  long long sr, sc;
  int lower;  // S is lower triangular (S(r, c) = 0 for c > r); 0 when unknown
};
constexpr int kMaxLeft = 4;
constexpr int kMaxRight = 5;
struct Stages {
  int nl, nr;
  Stage L[kMaxLeft];
  Stage R[kMaxRight];
};

enum GramMode { GRAM_LEFT = 0, GRAM_RIGHT = 1 };

// --- streaming kernels (ttr_stream.hip) -----------------------------------
void launch_add(hipStream_t s, int n, int N, double alpha, double beta, const double *X, int rx0, int rx1,
                const double *Y, int ry0, int ry1, long long I, double *Z);
void launch_hadamard(hipStream_t s, const double *X, int rx0, int rx1, const double *Y, int ry0, int ry1,
                     long long I, double *Z);
// Y = X for n doubles on stream s (16-byte loads, streaming stores; a plain
// device copy when a pointer is not 16-byte aligned).
void launch_copy(hipStream_t s, const double *X, long long n, double *Y);
// Y = X x_2 A for one core (a x I x b): A banded (kl, ku), band storage
// A(i, j) = AB[(ku + i - j) + (kl + ku + 1) j].  a <= 4096.
void launch_kron_apply(hipStream_t s, const double *X, int r0, int r1, long long I, const double *AB, int kl, int ku,
                       double *Y);
// Per-workgroup partial Grams sum_i Z(i) Z(i)^T (LEFT, gd = rows of Z) or
// Z(i)^T Z(i) (RIGHT, gd = cols of Z) into `partials` (TTR_MAXWG * gd * gd
// doubles).  Returns the workgroup count; launch_reduce then sums the partials
// in a fixed order into G (gd x gd, column-major).
int launch_gram(hipStream_t s, const CoreView &cv, const Stages &st, int mode, double *partials, double *G,
                int mixed);
// Y(r, i, c) = Z(i)(r, c) into a p x I x q core (trans_out = 0) or its
// transpose q x I x p (trans_out = 1).
void launch_reduce(hipStream_t s, const double *partials, int nwg, int ne, double *G);
void launch_apply(hipStream_t s, const CoreView &cv, const Stages &st, double *Y, int trans_out);
// Matrix-core paths (ttr_mfma.hip) on physical cores (a x I x b), dims <= 64.
// tri: the factor is triangular (Q lower / P upper), zero fragments are skipped.
// f32: the mixed-precision first pass (FP32 products and accumulation).
// fscale (f32, device, 3 doubles, nullable): the data and the factor are
// scaled by powers of two chosen from their largest entries before they are
// rounded to FP32, and the Gram is scaled back exactly (without it, FP32's
// range bounds the data).
int launch_gram_right_factor(hipStream_t s, const double *X, int a, int b, long long I, const double *Q, int q,
                             long long sQr, long long sQc, int tri, int f32, double *partials,
                             double *fscale = nullptr);
int launch_gram_left_factor(hipStream_t s, const double *X, int a, int b, long long I, const double *P, int p,
                            long long sPr, long long sPa, int tri, int f32, double *partials,
                            double *fscale = nullptr);
// tri: bit 0 = Q lower triangular, bit 1 = P upper triangular (their
// vanishing k-steps are skipped).
void launch_apply_mfma(hipStream_t s, const double *X, int a, int b, long long I, const double *P, int p,
                       long long sPr, long long sPa, const double *Q, int q, long long sQr, long long sQc, int tri,
                       double *Y);
// On the slice S_i = M_i (trans = 0) or M_i^T (trans = 1), sa x sb:
//   launch_gram_fac:   partial Grams of sum_i (S_i Q)^T (S_i Q), Q sb x q
//   launch_apply_fac2: Y_i = S_i Q1 Q2 written as sa x I x q2 (trans = 0) or
//                      q2 x I x sa (trans = 1); tri: Q1 lower triangular
int launch_gram_fac(hipStream_t s, const double *X, int a, int b, long long I, int trans, const double *Q, int q,
                    long long sQr, long long sQc, int tri, double *partials);
void launch_apply_fac2(hipStream_t s, const double *X, int a, int b, long long I, int trans, const double *Q1,
                       int q1, long long s1r, long long s1c, int tri, const double *Q2, int q2, long long s2r,
                       long long s2c, double *Y);
// The same step on the FP64 matrix cores: partial W_n (e x b, ld e) of each
// workgroup into `partials`; returns the workgroup count (launch_reduce sums
// them).  All ranks <= TTR_RMAX; X's slices a x b, Y's c x e, W (c x a, ld c).
// Workgroups (= partial matrices) launch_dot_mfma uses for I slices.
int dot_mfma_workgroups(long long I);
int launch_dot_mfma(hipStream_t s, const double *X, int a, int b, const double *Y, int c, int e, long long I,
                    const double *W, double *partials);

// --- rank 65..256 streaming kernels (ttr_lstream.hip) ----------------------
// Z (M x N) = X (M x K) B (K x N), K, N <= 256.  X: column-major (xcol, element
// (r, k) at X[r + ldx k]) or row-major (X[r ldx + k]); Z likewise (zcol, ldz).
// B(k, c) = B[k bsr + c bsc]; tri: 1 = B lower triangular, 2 = upper.  Bp:
// scratch of lg_packed_doubles(K, N) doubles for B in fragment order.  perm
// (device, K ints, nullable; xcol only): Z = X(:, perm) B(perm, :)-rows, i.e.
// column k of the operand is X(:, perm[k]) and row k of B is B(perm[k], :).
size_t lg_packed_doubles(int K, int N);
void launch_lg_gemm(hipStream_t s, const double *X, long long M, int K, long long ldx, int xcol, const double *B,
                    long long bsr, long long bsc, int N, int tri, double *Bp, double *Z, long long ldz, int zcol,
                    const int *perm = nullptr);
struct LGramGrid {
  int nwg;
  long long rpw;  // rows per workgroup (multiple of 16)
};
LGramGrid lg_gram_grid(long long M, int f32);
// Partial matrices of X1^T X2 (K1 x K2, column-major) over row ranges of
// lg_gram_grid(M, f32).rpw rows into part (nwg x K1 K2 doubles); X2 == nullptr:
// the Gram of X1 (symmetric; f32: FP32 products and accumulation).  Both
// operands share the layout xcol and have M rows.  Returns nwg.
// fscale (FP32 only, device): the scale pair of launch_lg_scale_probe.
int launch_lg_gram(hipStream_t s, const double *X1, const double *X2, long long M, int K1, int K2, long long ld1,
                   long long ld2, int xcol, int f32, double *part, const double *fscale = nullptr);
// C(i) = (A(i) (x) B(i)) T for every slice (Kronecker index a_x rB + a_y):
// A a0 x I x a1, B b0 x I x b1 (all <= 16), T (a1 b1) x k (ld ldt); C is the
// (a0 b0) x I x k core.
void launch_lg_kron_right(hipStream_t s, const double *A, int a0, int a1, const double *B, int b0, int b1, long long I,
                          const double *T, long long ldt, int k, double *C);
// out[0] = 2^-e, out[1] = 2^2e from the largest sampled |x| of X (n doubles).
void launch_lg_scale_probe(hipStream_t s, const double *X, long long n, double *out);
// C (m x n, ld ldc) = A B, A(i, k) = A[i ar + k ac], B(k, j) = B[k br + j bc].
void launch_lg_sgemm(hipStream_t s, const double *A, long long ar, long long ac, const double *B, long long br,
                     long long bc, int m, int n, int k, double *C, long long ldc);

// --- small dense kernels (ttr_small.hip) ----------------------------------
// One step of QR-by-Gram.  G (d x d) is the Gram of the current staged
// unfolding A*F_1*...*F_{j-1} (j = pass).  Writes the next stage F_j
// (d x k, ld d), the collapsed factor Rnext = R_j * Rc (k x b, ld k; Rc = I at
// pass 1) and, once done, Tdst = Rnext^T (b x k, ld b).
struct QrStepArgs {
  const double *G;
  int d;
  // optional post-transform: the input is G0 (tpr x tpr) and the Gram used is
  // G = T^T G0 T (d = tpc); cond_scale (>= 1) is kappa(T)^2, which tightens
  // the one-pass acceptance test
  const double *Tpost;
  int tpr, tpc;
  long long tsr, tsc;
  double cond_scale;
  double *ratio_out;   // receives t_max / t_min of this pass (may be nullptr)
  int pass;            // 1, 2 or 3
  int b;               // columns of the unfolding
  const double *Rc;    // d x b (ld d); nullptr at pass 1
  double *Fstep;       // d x k (ld d)
  double *Rnext;       // k x b (ld k)
  double *Tdst;        // when done: Rnext^T (b x k, ld b); may be nullptr
  int *dec;            // [0] k, [1] done, [2] error flags, [4] triangular factors, [5] no truncation
                       // proven, [6] settled at the first pass with mutually orthogonal rows of R
  // tau1: one pass is enough (and a refinement pass settles) when the Gram's
  // condition number, scaled by cond_scale, is at most 1/tau1; tau2: rank
  // revealing cut of the refinement passes
  double tau1, tau2;
  double ugram;        // unit roundoff of the arithmetic that formed G (FP64 or FP32)
  double gerr;         // |G_computed - G| <= gerr * trace(G), for the no-truncation proof
  int try_chol;        // pass 1: try the Cholesky route first
  int shift_pass;      // last pass that may take the shifted route (1; 2 in mixed
                       // precision, where pass 1's FP32 shift leaves directions
                       // below ~u32 that one FP64 pass cannot resolve)
  // truncation sweep only: with the Cholesky route, also prove that no
  // singular value can be dropped at this link (lambda_min(G) >= 1/||L^{-1}||_F^2
  // > margin * delta^2); delta is *delta_dev, or at the first link
  // tol^2 trace(G) / (N-1) = tol2_nm1 * trace(G).
  int notrunc_check;
  const double *delta_dev;
  int first;
  double tol2_nm1;
};
void launch_qr_step(hipStream_t s, const QrStepArgs &a);

// Truncation at one link: SVD of R (k x b), rank L, and the two small factors
// that carry the result: GU = Glast * U_R[:, :L] (d x L, ld d), the merged last
// right stage of the output core, and Pnext = Sigma_L V_R[:, :L]^T Fn^T
// (L x dn, ld L), the merged last left stage of the next core (Fn is the last
// orthonormalization stage of the next core, dn x b, ld dn).
struct TruncArgs {
  const double *R;   // k x b (ld k)
  int k, b;
  const double *Glast;  // d x k (ld d)
  int d;
  const double *Fn;     // dn x b (ld dn)
  int dn;
  double *GU;        // d x L
  double *Pnext;     // L x dn
  double *delta;     // device scalar: written at the first link, read afterwards
  double *norm;      // device scalar
  int first;
  double tol;
  int Nm1;
  double *sigma_out; // TTR_RMAX values (descending, zero padded)
  double *tail_out;  // nullable: sum of squares of the discarded singular values
  int *dec;          // [3] L, [2] error flags, [9] Jacobi sweeps (0: no SVD)
  int r_orth;        // rows of R are known to be orthogonal (skip the rotations)
  int identity;      // the step proved L = k: U = I and Sigma V^T = R (no SVD)
};
void launch_trunc_step(hipStream_t s, const TruncArgs &a);

// Utility: C (m x n, ld m) = A (m x k, ld m) * B (k x n, ld k); one workgroup.
void launch_small_gemm(hipStream_t s, const double *A, const double *B, double *C, int m, int k, int n);
// --- batched streaming launches ---------------------------------------------
// One TT's operands for a batched streaming launch, written on the device by
// the batched planner (ttr_batch.hip).  Fields unused by a kernel are ignored.
struct BDesc {
  int active;
  int a, b;               // physical slice dims of X
  long long I, spw;       // slices, slices per workgroup
  int nwg;                // workgroups of this TT (= ceil(I / spw))
  int tri;                // first factor triangular (see the single launchers)
  const double *X;
  const double *P;        // left factor (output pass)
  int p;
  long long sPr, sPa;
  const double *Q;        // (first) right factor
  int q;
  long long sQr, sQc;
  const double *Q2;       // second right factor (two-factor output pass)
  int q2;
  long long s2r, s2c;
  double *out;            // Gram partials (nwg x ne) or the output core
  int ne;                 // Gram entries (reduce)
  double *G;              // reduce target
};
struct WGItem {
  int tt, wg;
};
// The items of one tile class (NT) and one core: workgroup `blockIdx.x` walks
// items blockIdx.x, blockIdx.x + gridDim.x, ... (persistent when the grid is
// smaller than the item count).  f32 / trans select the variants as in the
// single launchers.
void launch_gram_right_factor_batched(hipStream_t s, int nt, int f32, const BDesc *d, const WGItem *items, int nitems,
                                      int grid);
void launch_gram_left_factor_batched(hipStream_t s, int nt, int f32, const BDesc *d, const WGItem *items, int nitems,
                                     int grid);
void launch_apply_mfma_batched(hipStream_t s, int nt, const BDesc *d, const WGItem *items, int nitems, int grid);
void launch_gram_fac_batched(hipStream_t s, int nt, int trans, const BDesc *d, const WGItem *items, int nitems,
                             int grid);
void launch_apply_fac2_batched(hipStream_t s, int nt, int trans, const BDesc *d, const WGItem *items, int nitems,
                               int grid);
// Sum of each active TT's partials (d[t].out, d[t].nwg x d[t].ne) into d[t].G.
void launch_reduce_batched(hipStream_t s, int count, const BDesc *d);

// Batched forms (one workgroup per item, skipped where active[item] == 0);
// the argument arrays live in device memory.
struct SmallGemmArgs {
  const double *A, *B;
  double *C;
  int m, k, n;
};
void launch_qr_step_batched(hipStream_t s, int count, const QrStepArgs *args, const int *active);
void launch_trunc_step_batched(hipStream_t s, int count, const TruncArgs *args, const int *active);
void launch_small_gemm_batched(hipStream_t s, int count, const SmallGemmArgs *args, const int *active);
// Square root of a 1x1 device value into out (for norms).
// F (d x d, ld d): upper triangular with F^T F = G (pivoted Cholesky, then a
// Householder QR of L^T P^T), zero rows past the numerical rank; d <= TTR_RMAX.
void launch_sym_factor(hipStream_t s, const double *G, int d, double *F);
// W (a x a) = P^T P for P (p x a, ld p), a, p <= TTR_RMAX.
void launch_ptp(hipStream_t s, const double *P, int p, int a, double *W);
void launch_sqrt_scalar(hipStream_t s, const double *in, double *out);
