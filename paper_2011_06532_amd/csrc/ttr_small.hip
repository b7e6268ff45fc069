// Small dense FP64 kernels, one workgroup each, matrices (<= 64 x 64) in LDS.
//
// They turn the Gram matrices produced by the streaming passes into the
// factors the sweeps pass between cores:
//   * k_qr_step: one step of a rank-revealing, shift-stabilized Cholesky-QR
//     realized with eigendecompositions.  For a tall-skinny unfolding A
//     (accessed only through streaming passes) it yields B (b x k) and R
//     (k x b) with A*B column-orthonormal and A = (A*B) R to rounding error.
//     This plays the role of the tall-skinny QR of §3.3 (TSQR) in Alg. 5/6.
//   * k_trunc_step: SVD of R, truncation rank with the Frobenius-tail rule and
//     threshold delta = tol ||X|| / sqrt(N-1) (Alg. 2), the right factor that
//     produces the output core (U-hat, §2.4) and the matrix Sigma-hat V-hat^T
//     passed into the next core.
// Eigen- and singular-value problems use one-sided (Hestenes) Jacobi with a
// round-robin parallel ordering: each wave rotates one column pair at a time,
// lanes holding one row each.
#include "ttr_internal.h"

#include <cfloat>

namespace {

constexpr int kThreads = 1024;   // 16 waves: one-sided Jacobi rotates all column pairs of a round at once
constexpr int kThreadsQR = 256;  // two-sided Jacobi: cheap barriers matter more than width
// rows of a rotation handled by one thread: blockDim / (d/2) threads share a
// pair, so with 256 threads and d <= 64 each owns at most 8
constexpr int kRows = 8;
constexpr int kWave = 64;
constexpr double kU = DBL_EPSILON / 2;  // unit roundoff 2^-53
// A pivoted cut falls off a clear gap when the last kept pivot is at least
// this many times the largest dropped one (a factor 1e3 in singular values).
constexpr double kPivGap = 1e6;

// Sums of three values over the wave; every lane gets lane 0's result so
// that branch decisions taken on them are uniform across the wave.
__device__ inline void wave_sum3(double &a, double &b, double &c) {
  for (int off = kWave / 2; off >= 1; off >>= 1) {
    a += __shfl_xor(a, off, kWave);
    b += __shfl_xor(b, off, kWave);
    c += __shfl_xor(c, off, kWave);
  }
  a = __shfl(a, 0, kWave);
  b = __shfl(b, 0, kWave);
  c = __shfl(c, 0, kWave);
}

// Round-robin (circle) pairing of nn (even) columns: round r, pair k.
__device__ inline void rr_pair(int r, int k, int nn, int *p, int *q) {
  if (k == 0) {
    *p = r;
    *q = nn - 1;
  } else {
    const int m = nn - 1;
    *p = (r + k) % m;
    *q = (r - k + m) % m;
  }
}

__device__ inline bool finite(double x) { return x == x && fabs(x) <= DBL_MAX; }

// Fixed-order sum over the workgroup (blockDim.x a multiple of 64, <= 1024):
// a butterfly within each wave (every lane ends with bitwise the same value,
// the two operands of each addition being the same in both lanes), then the
// wave results in wave order.  Every thread returns the result.
__device__ double block_sum(double v) {
  __shared__ double red[16];
  for (int off = kWave / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  const int wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
  if (threadIdx.x % kWave == 0) red[wave] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < nw; ++w) r += red[w];
  __syncthreads();
  return r;
}

__device__ double block_max(double v) {
  __shared__ double red[16];
  for (int off = kWave / 2; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  const int wave = threadIdx.x / kWave, nw = blockDim.x / kWave;
  if (threadIdx.x % kWave == 0) red[wave] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < nw; ++w) r = fmax(r, red[w]);
  __syncthreads();
  return r;
}

// ||M||_1 (largest column sum of |entries|) or ||M||_inf (largest row sum)
// of a d x d column-major matrix.
__device__ double norm1(const double *M, int d) {
  double v = 0.0;
  for (int c = threadIdx.x; c < d; c += blockDim.x) {
    double s = 0.0;
    for (int r = 0; r < d; ++r) s += fabs(M[r + d * c]);
    v = fmax(v, s);
  }
  return block_max(v);
}
__device__ double norminf(const double *M, int d) {
  double v = 0.0;
  for (int r = threadIdx.x; r < d; r += blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < d; ++c) s += fabs(M[r + d * c]);
    v = fmax(v, s);
  }
  return block_max(v);
}

__device__ double sumsq(const double *X, int n) {
  double s = 0.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) s += X[e] * X[e];
  return block_sum(s);
}

// One-sided Jacobi on A (m x n, column-major, lda = m) in LDS, accumulating the
// rotations into V (n x n, ldv = n, identity on entry).  On return the columns
// of A are mutually orthogonal to relative tolerance.  Returns the number of
// sweeps, or -1 without convergence.  m, n <= 64.
__device__ int jacobi_onesided(double *A, int m, int n, double *Vm, int *flag) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int nwaves = blockDim.x / kWave;
  const int nn = n + (n & 1);
  const double tol = kU * 4.0 * sqrt((double)(m > 1 ? m : 1));
  // Columns at rounding level of the whole matrix (exact null directions of a
  // rank-deficient input) are left alone: their mutual angles are noise and
  // would never settle.
  const double fro2 = sumsq(A, m * n);
  const double floor2 = (8.0 * (m + n) * kU) * (8.0 * (m + n) * kU) * fro2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (threadIdx.x == 0) *flag = 0;
    __syncthreads();
    int rotated = 0;
    for (int r = 0; r < nn - 1; ++r) {
      for (int k = wave; k < nn / 2; k += nwaves) {
        int p, q;
        rr_pair(r, k, nn, &p, &q);
        if (p >= n || q >= n) continue;
        const double ap = lane < m ? A[p * m + lane] : 0.0;
        const double aq = lane < m ? A[q * m + lane] : 0.0;
        double alpha = ap * ap, beta = aq * aq, gamma = ap * aq;
        wave_sum3(alpha, beta, gamma);
        if (alpha > floor2 && beta > floor2 && fabs(gamma) > tol * sqrt(alpha) * sqrt(beta)) {
          const double zeta = (beta - alpha) / (2.0 * gamma);
          const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t);
          const double s = c * t;
          if (lane < m) {
            A[p * m + lane] = c * ap - s * aq;
            A[q * m + lane] = s * ap + c * aq;
          }
          if (lane < n) {
            const double vp = Vm[p * n + lane];
            const double vq = Vm[q * n + lane];
            Vm[p * n + lane] = c * vp - s * vq;
            Vm[q * n + lane] = s * vp + c * vq;
          }
          rotated = 1;
        }
      }
      __syncthreads();
    }
    if (rotated) *flag = 1;
    __syncthreads();
    const int any = *flag;
    __syncthreads();
    if (!any) return sweep + 1;
  }
  return -1;
}

// Two-sided cyclic Jacobi for a symmetric A (d x d, column-major, LDS),
// accumulating the rotations into V (identity on entry): A <- J^T A J,
// V <- V J.  Each round rotates the disjoint pairs of the round-robin
// ordering at once: angles from (A_pp, A_qq, A_pq), then all column
// rotations, then all row rotations.  Off-diagonal entries at rounding level
// of the matrix (null directions of a rank-deficient Gram) are left alone.
// Returns the sweep count, or -1 without convergence.  Eigenvalues end on the
// diagonal of A.
__device__ int jacobi_sym(double *A, int d, double *V, int *flag) {
  __shared__ double cs[TTR_RMAX / 2], sn[TTR_RMAX / 2];
  __shared__ unsigned char pp[TTR_RMAX][TTR_RMAX / 2], qq[TTR_RMAX][TTR_RMAX / 2];
  const int nn = d + (d & 1);
  const int npair = nn / 2;
  const double tol = kU * 4.0 * sqrt((double)(d > 1 ? d : 1));
  // pair schedule of every round, computed once
  for (int e = threadIdx.x; e < (nn - 1) * npair; e += blockDim.x) {
    const int r = e / npair, k = e - r * npair;
    int p, q;
    rr_pair(r, k, nn, &p, &q);
    pp[r][k] = (unsigned char)p;
    qq[r][k] = (unsigned char)q;
  }
  const double fro2 = sumsq(A, d * d);
  const double floor_abs = 8.0 * d * kU * sqrt(fro2);
  // thread -> (pair kk, first row r0, row stride rs) for the rotation phases
  const int lanes_per_pair = blockDim.x / npair;
  const int kk = threadIdx.x % npair;
  const int r0 = threadIdx.x / npair;
  const bool active = r0 < lanes_per_pair;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (threadIdx.x == 0) *flag = 0;
    __syncthreads();
    for (int r = 0; r < nn - 1; ++r) {
      if (threadIdx.x < npair) {
        const int k = threadIdx.x;
        const int p = pp[r][k], q = qq[r][k];
        double c = 1.0, s = 0.0;
        if (p < d && q < d) {
          const double app = A[p + d * p], aqq = A[q + d * q], apq = A[p + d * q];
          if (fabs(apq) > floor_abs && fabs(apq) > tol * sqrt(fabs(app)) * sqrt(fabs(aqq))) {
            const double zeta = (aqq - app) / (2.0 * apq);
            const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            c = 1.0 / sqrt(1.0 + t * t);
            s = c * t;
            *flag = 1;
          }
        }
        cs[k] = c;
        sn[k] = s;
      }
      __syncthreads();
      // Each thread owns at most kRows rows (columns) of its pair; all its LDS
      // reads are issued before any arithmetic so their latencies overlap.
      if (active) {
        const double s = sn[kk];
        if (s != 0.0) {
          const double c = cs[kk];
          const int p = pp[r][kk], q = qq[r][kk];
          double *Ap = A + d * p, *Aq = A + d * q, *Vp = V + d * p, *Vq = V + d * q;
          double ap[kRows], aq[kRows], vp[kRows], vq[kRows];
#pragma unroll
          for (int m = 0; m < kRows; ++m) {  // columns: A <- A J, V <- V J
            const int row = r0 + m * lanes_per_pair;
            if (row < d) {
              ap[m] = Ap[row];
              aq[m] = Aq[row];
              vp[m] = Vp[row];
              vq[m] = Vq[row];
            }
          }
#pragma unroll
          for (int m = 0; m < kRows; ++m) {
            const int row = r0 + m * lanes_per_pair;
            if (row < d) {
              Ap[row] = c * ap[m] - s * aq[m];
              Aq[row] = s * ap[m] + c * aq[m];
              Vp[row] = c * vp[m] - s * vq[m];
              Vq[row] = s * vp[m] + c * vq[m];
            }
          }
        }
      }
      __syncthreads();
      if (active) {
        const double s = sn[kk];
        if (s != 0.0) {
          const double c = cs[kk];
          const int p = pp[r][kk], q = qq[r][kk];
          double ap[kRows], aq[kRows];
#pragma unroll
          for (int m = 0; m < kRows; ++m) {  // rows: A <- J^T A
            const int col = r0 + m * lanes_per_pair;
            if (col < d) {
              ap[m] = A[p + d * col];
              aq[m] = A[q + d * col];
            }
          }
#pragma unroll
          for (int m = 0; m < kRows; ++m) {
            const int col = r0 + m * lanes_per_pair;
            if (col < d) {
              A[p + d * col] = c * ap[m] - s * aq[m];
              A[q + d * col] = s * ap[m] + c * aq[m];
            }
          }
        }
      }
      __syncthreads();
    }
    const int any = *flag;
    __syncthreads();
    if (!any) return sweep + 1;
  }
  return -1;
}

// Descending ranks of key[0..n): perm[rank] = j.  Ties keep index order.
__device__ void sort_desc(const double *key, int n, int *perm) {
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    int rank = 0;
    for (int i = 0; i < n; ++i)
      if (key[i] > key[j] || (key[i] == key[j] && i < j)) ++rank;
    perm[rank] = j;
  }
  __syncthreads();
}



// X = L^{-1} (k x k, ld d) for the lower-triangular L in A (ld d), both in
// LDS: column-oriented forward substitution on all right-hand sides at once,
// one barrier per column of L.  Step m eliminates with row m of X (scaled on
// the fly); the row itself is scaled one step later, when no thread reads it.
__device__ void lower_inv(const double *A, double *X, int k, int d) {
  const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4, nc = blockDim.x >> 4;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int r = e % k, c = e / k;
    X[r + d * c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  double pprev = 0.0;
  for (int m = 0; m < k; ++m) {
    const double pm = 1.0 / A[m + d * m];
    if (m > 0)
      for (int c = threadIdx.x; c < m; c += blockDim.x) X[(m - 1) + d * c] *= pprev;
    for (int c = tc; c <= m; c += nc) {
      const double xm = X[m + d * c] * pm;
      for (int r = m + 1 + tr; r < k; r += 16) X[r + d * c] -= A[r + d * m] * xm;
    }
    pprev = pm;
    __syncthreads();
  }
  for (int c = threadIdx.x; c < k; c += blockDim.x) X[(k - 1) + d * c] *= pprev;
  __syncthreads();
}

// Unpivoted Cholesky G = L L^T of the symmetric d x d matrix in A (LDS), in
// place (lower triangle; the strict upper part is zeroed), one barrier per
// column.  Returns false, with A partly overwritten, as soon as a pivot is not
// above `thresh`.
__device__ bool chol_lower(double *A, int d, double thresh) {
  // threads as 16 rows x (blockDim/16) columns of the trailing updates
  const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4, nc = blockDim.x >> 4;
  // step j updates the trailing lower triangle with the unscaled column j
  // (L(r,j) L(c,j) = A(r,j) A(c,j) / A(j,j)) and scales column j-1, which no
  // thread reads during step j
  double lprev = 0.0;
  for (int j = 0; j < d; ++j) {
    const double pv = A[j + d * j];
    if (!(pv > thresh)) return false;  // the same value in every thread
    if (j > 0)
      for (int r = j - 1 + threadIdx.x; r < d; r += blockDim.x)
        A[r + d * (j - 1)] = (r == j - 1) ? lprev : A[r + d * (j - 1)] / lprev;
    const double rp = 1.0 / pv;
    for (int c = j + 1 + tc; c < d; c += nc) {
      const double acj = A[c + d * j] * rp;
      for (int r = c + tr; r < d; r += 16) A[r + d * c] -= A[r + d * j] * acj;
    }
    lprev = sqrt(pv);
    __syncthreads();
  }
  if (threadIdx.x == 0) A[(d - 1) + d * (d - 1)] = lprev;
  for (int e = threadIdx.x; e < d * d; e += blockDim.x)
    if (e % d < e / d) A[e] = 0.0;
  __syncthreads();
  return true;
}

// Cholesky G = L L^T of the symmetric d x d matrix in A (LDS), in place (lower
// triangle; the strict upper part is zeroed), then L^{-1} into Vm by forward
// substitution; both take one barrier per column.  Returns false when a pivot
// is not positive.  With G symmetric, ||G||_2 <= ||G||_1 and
// ||G^{-1}||_2 <= ||G^{-1}||_1 <= ||L^{-1}||_inf ||L^{-1}||_1, so
// *kappa = ||G||_1 ||L^{-1}||_1 ||L^{-1}||_inf bounds kappa_2(G) from above and
// *lmin_lb = 1 / min(||L^{-1}||_F^2, ||L^{-1}||_1 ||L^{-1}||_inf) bounds
// lambda_min(G) from below.
__device__ bool chol_inv(double *A, double *Vm, int d, double *kappa, double *lmin_lb) {
  const double g1 = norm1(A, d);
  if (!chol_lower(A, d, 0.0)) return false;
  lower_inv(A, Vm, d, d);
  const double lf2 = sumsq(Vm, d * d);
  const double l1 = norm1(Vm, d), li = norminf(Vm, d);
  *kappa = g1 * l1 * li;
  *lmin_lb = 1.0 / fmin(lf2, l1 * li);
  return true;
}

// Pivoted Cholesky of the d x d symmetric A (full storage, overwritten), the
// rank-revealing form: pivots in order perm[0..k), A(i, j) (i >= j, j < k)
// holds L with G(perm, perm) ~= L L^T; stops once the largest remaining
// diagonal entry is at most tau times the largest initial one.  Returns k.
// gap (nullable, every thread): the last kept pivot over the largest
// remaining diagonal entry at the stop (+inf when nothing was dropped); the
// pivots never grow, so a large ratio separates the kept directions from the
// dropped ones.
__device__ int pivoted_chol(double *A, int d, double tau, int *perm, double *gap = nullptr) {
  __shared__ int piv, stop;
  __shared__ double dmax0, pkeep, pdrop;
  for (int i = threadIdx.x; i < d; i += blockDim.x) perm[i] = i;
  double m = 0.0;
  for (int i = threadIdx.x; i < d; i += blockDim.x) m = fmax(m, A[i + d * i]);
  m = block_max(m);
  if (threadIdx.x == 0) dmax0 = m;
  __syncthreads();
  int k = d;
  for (int j = 0; j < d; ++j) {
    if (threadIdx.x < kWave) {
      // wave 0: the largest remaining diagonal entry (d <= 64), the first
      // one among ties
      const int i = j + threadIdx.x;
      double v = (i < d) ? A[i + d * i] : -DBL_MAX;
      int p = (i < d) ? i : d;
      for (int off = kWave / 2; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(v, off, kWave);
        const int op = __shfl_xor(p, off, kWave);
        if (ov > v || (ov == v && op < p)) {
          v = ov;
          p = op;
        }
      }
      if (threadIdx.x == 0) {
        piv = p;
        stop = !(v > tau * dmax0) || p >= d;
        if (j == 0) pkeep = pdrop = 0.0;
        if (stop) pdrop = (p < d && v > 0.0) ? v : 0.0;
        else pkeep = v;
      }
    }
    __syncthreads();
    if (stop) {
      k = j;
      break;
    }
    const int p = piv;
    if (p != j) {
      // symmetric interchange j <-> p, including the rows of L computed so far
      for (int c = threadIdx.x; c < d; c += blockDim.x) {
        const double t = A[j + d * c];
        A[j + d * c] = A[p + d * c];
        A[p + d * c] = t;
      }
      __syncthreads();
      for (int r = threadIdx.x; r < d; r += blockDim.x) {
        const double t = A[r + d * j];
        A[r + d * j] = A[r + d * p];
        A[r + d * p] = t;
      }
      if (threadIdx.x == 0) {
        const int t = perm[j];
        perm[j] = perm[p];
        perm[p] = t;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) A[j + d * j] = sqrt(A[j + d * j]);
    __syncthreads();
    const double ljj = A[j + d * j];
    for (int i = j + 1 + threadIdx.x; i < d; i += blockDim.x) A[i + d * j] /= ljj;
    __syncthreads();
    const int n = d - j - 1;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const int r = j + 1 + e % n, c = j + 1 + e / n;
      A[r + d * c] -= A[r + d * j] * A[c + d * j];
    }
    __syncthreads();
  }
  if (gap) *gap = (k < d && pdrop > 0.0) ? pkeep / pdrop : INFINITY;
  return k;
}

// ---------------------------------------------------------------------------
// QR-by-Gram step.  Input: G = Gram of the current staged unfolding
// A F_1 ... F_{j-1} and the collapsed factor Rc with A = (A F_1...F_{j-1}) Rc.
// Output: the next stage F_j and Rnext = R_j Rc.
//   pass 1: eigen-decomposition G = W diag(t) W^T.  If t_min >= tau1 t_max the
//           unfolding is well conditioned: F = W t^{-1/2}, R = t^{1/2} W^T, done.
//           Otherwise shift by s ~ d u t_max (so every direction survives the
//           square root) and ask for another pass: F = W (t+s)^{-1/2}.
//   pass 2, 3: keep the k directions with t_j >= tau2 t_1 (the rest is
//           rounding noise of a rank-deficient unfolding), F = W_k t_k^{-1/2};
//           done when t_k >= tau1 t_1 (or at pass 3).
// ---------------------------------------------------------------------------
__device__ void qr_step_body(const QrStepArgs a) {
  __shared__ double A[TTR_RMAX * TTR_RMAX];
  __shared__ double Vm[TTR_RMAX * TTR_RMAX];
  __shared__ double Bf[TTR_RMAX * TTR_RMAX];
  __shared__ double lam[TTR_RMAX];
  __shared__ double sc[TTR_RMAX];
  __shared__ double rs[TTR_RMAX];
  __shared__ int perm[TTR_RMAX];
  __shared__ int flag, kk, done, bad;
  const int d = a.d;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  if (a.Tpost) {
    // G = T^T G0 T with G0 (m x m), T (m x d): Vm <- G0 T, then A <- T^T Vm
    const int m = a.tpr;
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
      const double g = a.G[e];
      if (!finite(g)) bad = 1;
      A[e] = g;
    }
    for (int e = threadIdx.x; e < m * d; e += blockDim.x) {
      const int r = e % m, c = e / m;
      Bf[r + m * c] = a.Tpost[r * a.tsr + c * a.tsc];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m * d; e += blockDim.x) {
      const int r = e % m, c = e / m;
      double s = 0.0;
      for (int k = 0; k < m; ++k) s += A[r + m * k] * Bf[k + m * c];
      Vm[r + m * c] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
      const int r = e % d, c = e / d;
      double s = 0.0;
      for (int k = 0; k < m; ++k) s += Bf[k + m * r] * Vm[k + m * c];
      A[r + d * c] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
      const int r = e % d, c = e / d;
      if (r > c) {  // exact symmetry
        const double v = 0.5 * (A[r + d * c] + A[c + d * r]);
        A[r + d * c] = v;
        A[c + d * r] = v;
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
      const int r = e % d, c = e / d;
      Vm[e] = (r == c) ? 1.0 : 0.0;
    }
  } else {
    for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
      const double g = a.G[e];
      if (!finite(g)) bad = 1;
      A[e] = g;
      const int r = e % d, c = e / d;
      Vm[e] = (r == c) ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  if (bad) {
    if (threadIdx.x == 0) {
      a.dec[2] |= 1;
      a.dec[1] = 1;
      a.dec[0] = 1;
      a.dec[6] = 0;
    }
    return;
  }
  if (a.try_chol) {
    // Attempt by Cholesky, G = L L^T: F = L^{-T}, R = L^T Rc (T = L at pass 1).
    // Accepted when kappa(G) (bounded by Gershgorin or ||G||_1 ||L^{-1}||_1
    // ||L^{-1}||_inf, scaled by kappa(T)^2 when G came through a post-transform)
    // is at most 1/tau1, and, at the first pass of the truncation sweep, when
    // no singular value can fall below delta.  At a refinement pass G is close
    // to the identity and this is the second step of CholeskyQR2.
    __shared__ int accept, kap_ok;
    for (int e = threadIdx.x; e < d * d; e += blockDim.x) Bf[e] = A[e];  // keep G for a fallback
    double trace_part = 0.0;
    for (int j = threadIdx.x; j < d; j += blockDim.x) trace_part += A[j + d * j];
    const double trG = block_sum(trace_part);
    // Gershgorin: every eigenvalue of G lies in [min_r (G_rr - off_r), max_r (G_rr + off_r)],
    // off_r = sum_{c != r} |G_rc|; tight for the near-diagonal Grams of
    // well-conditioned unfoldings
    double glo = DBL_MAX, ghi = 0.0;
    for (int r = threadIdx.x; r < d; r += blockDim.x) {
      double off = 0.0;
      for (int c = 0; c < d; ++c)
        if (c != r) off += fabs(A[r + d * c]);
      glo = fmin(glo, A[r + d * r] - off);
      ghi = fmax(ghi, A[r + d * r] + off);
    }
    const double gmin = -block_max(-glo), gmax = block_max(ghi);
    double kappa = 0.0, lmin_lb = 0.0;
    const bool ok = chol_inv(A, Vm, d, &kappa, &lmin_lb);
    if (gmin > 0.0) {
      kappa = fmin(kappa, gmax / gmin);
      lmin_lb = fmax(lmin_lb, gmin);
    }
    if (threadIdx.x == 0) {
      int acc = ok && (kappa == kappa) && kappa * (a.cond_scale > 1.0 ? a.cond_scale : 1.0) * a.tau1 <= 1.0;
      kap_ok = acc;
      int notrunc = 0;
      if (acc && a.notrunc_check && a.pass == 1) {
        const double dl = a.first ? sqrt(a.tol2_nm1 * trG) : *a.delta_dev;
        const double cs = a.cond_scale > 1.0 ? a.cond_scale : 1.0;
        notrunc = (lmin_lb - a.gerr * cs * trG > 4.0 * dl * dl);
        acc = notrunc;
      }
      if (a.ratio_out) *a.ratio_out = ok ? kappa : 1e300;
      accept = acc;
      a.dec[5] = notrunc;
    }
    __syncthreads();
    if (accept) {
      // A holds L (lower), Vm holds L^{-1} (lower)
      const int b = a.b;  // == d at pass 1
      if (!a.Rc) {
        for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
          const int r = e % d, c = e / d;
          a.Fstep[r + d * c] = Vm[c + d * r];            // F = L^{-T}
          a.Rnext[r + d * c] = A[c + d * r];             // R = L^T
          if (a.Tdst) a.Tdst[r + b * c] = A[r + d * c];  // T = L
        }
      } else {
        for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
          const int r = e % d, c = e / d;
          a.Fstep[r + d * c] = Vm[c + d * r];  // F = L^{-T}
        }
        // R = L^T Rc (d x b), and T = R^T
        for (int e = threadIdx.x; e < d * b; e += blockDim.x) {
          const int r = e % d, c = e / d;
          double v = 0.0;
          for (int j = r; j < d; ++j) v += A[j + d * r] * a.Rc[j + d * c];
          a.Rnext[r + d * c] = v;
          if (a.Tdst) a.Tdst[c + b * r] = v;
        }
      }
      if (threadIdx.x == 0) {
        a.dec[0] = d;
        a.dec[1] = 1;
        a.dec[4] = a.Rc ? 0 : 1;  // triangular factors (first pass only)
        a.dec[6] = 0;
      }
      return;
    }
    bool shift_it = !kap_ok && a.pass <= a.shift_pass;
    if (shift_it && a.pass >= 2) {
      // A second shifted pass (mixed precision, after the FP32 one) is for a
      // spectrum graded across the pivoted cut; when the pivots fall off a
      // clear gap instead (an exactly rank-deficient unfolding such as Y + Y)
      // the cut drops only null directions and this pass takes it.
      for (int e = threadIdx.x; e < d * d; e += blockDim.x) A[e] = Bf[e];
      __syncthreads();
      double gap;
      pivoted_chol(A, d, a.tau2, perm, &gap);
      shift_it = !(gap >= kPivGap);
      __syncthreads();
    }
    if (shift_it) {
      // Shifted CholeskyQR: G + sI = L L^T with s ~ d u trace(G) gives A L^{-T}
      // the singular values sqrt(lambda / (lambda + s)), as the shifted eigen
      // route would, at the cost of one factorization; the next pass refines.
      const double shift = 2.0 * d * a.ugram * trG;
      for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
        const int r = e % d, c = e / d;
        A[e] = Bf[e] + ((r == c) ? shift : 0.0);
      }
      __syncthreads();
      double kap2 = 0.0, lmin2 = 0.0;
      const bool ok2 = (shift > 0.0) && chol_inv(A, Vm, d, &kap2, &lmin2);
      if (ok2) {
        for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
          const int r = e % d, c = e / d;
          a.Fstep[r + d * c] = Vm[c + d * r];  // F = L^{-T}
          if (!a.Rc) a.Rnext[r + d * c] = A[c + d * r];   // R = L^T (Rc = I at the first pass)
        }
        if (a.Rc) {
          // a shifted refinement pass (mixed precision): R = L^T Rc (d x b)
          __syncthreads();
          const int b = a.b;
          for (int e = threadIdx.x; e < d * b; e += blockDim.x) {
            const int r = e % d, c = e / d;
            double v = 0.0;
            for (int j = r; j < d; ++j) v += A[j + d * r] * a.Rc[j + d * c];
            a.Rnext[r + d * c] = v;
          }
        }
        if (threadIdx.x == 0) {
          if (a.ratio_out) *a.ratio_out = 1e300;
          a.dec[0] = d;
          a.dec[1] = 0;
          a.dec[4] = 0;
          a.dec[5] = 0;
          a.dec[6] = 0;
        }
        return;
      }
    }
    if (a.pass >= 2) {
      // Refinement pass: rank-revealing pivoted Cholesky of G (close to the
      // identity on the directions that carry content, at rounding level on
      // the null directions of a rank-deficient unfolding).
      for (int e = threadIdx.x; e < d * d; e += blockDim.x) A[e] = Bf[e];
      __syncthreads();
      const int k = pivoted_chol(A, d, a.tau2, perm);
      if (k > 0) {
      // X = L11^{-1} (k x k lower, ld d)
      lower_inv(A, Vm, k, d);
      // conditioning of the kept part: ||G11||_1 ||X||_1 ||X||_inf
      double g1 = 0.0, x1 = 0.0, xi = 0.0;
      for (int c = threadIdx.x; c < k; c += blockDim.x) {
        double sg = 0.0, sx = 0.0;
        for (int r = 0; r < k; ++r) {
          sg += fabs(Bf[perm[r] + d * perm[c]]);
          sx += fabs(Vm[r + d * c]);
        }
        g1 = fmax(g1, sg);
        x1 = fmax(x1, sx);
      }
      for (int r = threadIdx.x; r < k; r += blockDim.x) {
        double sx = 0.0;
        for (int c = 0; c < k; ++c) sx += fabs(Vm[r + d * c]);
        xi = fmax(xi, sx);
      }
      g1 = block_max(g1);
      x1 = block_max(x1);
      xi = block_max(xi);
      const int dn = (a.pass >= 3 || g1 * x1 * xi * a.tau1 <= 1.0) ? 1 : 0;
      // F (d x k): F(perm[i], c) = X(c, i);  R' (k x d): R'(c, perm[j]) = L(j, c)
      for (int e = threadIdx.x; e < d * k; e += blockDim.x) a.Fstep[e] = 0.0;
      __syncthreads();
      for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
        const int i = e % k, c = e / k;
        a.Fstep[perm[i] + d * c] = (c >= i) ? Vm[c + d * i] : 0.0;
      }
      const int b = a.b;
      for (int e = threadIdx.x; e < k * b; e += blockDim.x) {
        const int c = e % k, col = e / k;
        double v = 0.0;
        for (int j = c; j < d; ++j) v += A[j + d * c] * a.Rc[perm[j] + d * col];
        a.Rnext[c + k * col] = v;
        if (dn && a.Tdst) a.Tdst[col + b * c] = v;
      }
      if (threadIdx.x == 0) {
        a.dec[0] = k;
        a.dec[1] = dn;
        a.dec[4] = 0;
        a.dec[6] = 0;
      }
      return;
      }
      // a zero Gram: the eigen route below returns the rank-1 zero factor
    }
    // fall back: G again for the eigen route
    for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
      A[e] = Bf[e];
      const int r = e % d, c = e / d;
      Vm[e] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) a.dec[5] = 0;
  if (threadIdx.x == 0) a.dec[4] = 0;
  const int sweeps = jacobi_sym(A, d, Vm, &flag);
  for (int j = threadIdx.x; j < d; j += blockDim.x) lam[j] = A[j + d * j];
  __syncthreads();
  sort_desc(lam, d, perm);
  // sorted eigenvectors into A (no longer needed), sorted eigenvalues into sc
  for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
    const int r = e % d, c = e / d;
    A[r + d * c] = Vm[r + d * perm[c]];
  }
  if (threadIdx.x < d) sc[threadIdx.x] = lam[perm[threadIdx.x]];
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t1 = sc[0];
    const double tmin = sc[d - 1];
    int k = d;
    int dn = 0;
    if (sweeps < 0) a.dec[2] |= 2;
    if (!(t1 > 0.0)) {
      k = 0;  // zero (or non-positive) Gram: no content
      dn = 1;
    } else if (a.pass == 1) {
      const double cs = a.cond_scale > 1.0 ? a.cond_scale : 1.0;
      if (a.ratio_out) *a.ratio_out = (tmin > 0.0) ? t1 / tmin : 1e300;
      const double shift = (tmin >= a.tau1 * t1 * cs) ? 0.0 : 2.0 * d * a.ugram * t1 + 2.0 * (tmin < 0 ? -tmin : 0.0);
      for (int j = 0; j < d; ++j) {
        const double v = sc[j] + shift;
        rs[j] = sqrt(v);
        sc[j] = 1.0 / rs[j];
      }
      dn = (shift == 0.0);
    } else {
      k = 0;
      while (k < d && sc[k] >= a.tau2 * t1) ++k;
      if (k < 1) k = 1;
      const double tk = sc[k - 1];
      for (int j = 0; j < k; ++j) {
        rs[j] = sqrt(sc[j]);
        sc[j] = 1.0 / rs[j];
      }
      dn = (a.pass >= 3 || tk >= a.tau1 * t1) ? 1 : 0;
    }
    kk = k;
    done = dn;
  }
  __syncthreads();
  const int k = kk;
  const int b = a.b;
  if (k == 0) {
    // zero unfolding: rank 1 with a zero factor R; the stage keeps the first direction
    for (int e = threadIdx.x; e < d; e += blockDim.x) a.Fstep[e] = (e == 0) ? 1.0 : 0.0;
    for (int e = threadIdx.x; e < b; e += blockDim.x) {
      a.Rnext[e] = 0.0;
      if (a.Tdst) a.Tdst[e] = 0.0;
    }
    if (threadIdx.x == 0) {
      a.dec[0] = 1;
      a.dec[1] = 1;
      a.dec[6] = 1;
    }
    return;
  }
  // F (d x k) = W[:, :k] diag(sc)
  for (int e = threadIdx.x; e < d * k; e += blockDim.x) {
    const int r = e % d, c = e / d;
    a.Fstep[r + d * c] = A[r + d * c] * sc[c];
  }
  // Rnext (k x b) = diag(rs) W[:, :k]^T Rc (d x b)
  if (a.Rc) {
    for (int e = threadIdx.x; e < d * b; e += blockDim.x) Bf[e] = a.Rc[e];
    __syncthreads();
  }
  for (int e = threadIdx.x; e < k * b; e += blockDim.x) {
    const int r = e % k, c = e / k;
    double s;
    if (a.Rc) {
      s = 0.0;
      for (int j = 0; j < d; ++j) s += A[j + d * r] * Bf[j + d * c];
    } else {
      s = A[c + d * r];
    }
    s *= rs[r];
    a.Rnext[r + k * c] = s;
    if (done && a.Tdst) a.Tdst[c + b * r] = s;
  }
  if (threadIdx.x == 0) {
    a.dec[0] = k;
    a.dec[1] = done;
    a.dec[6] = (a.pass == 1 && done) ? 1 : 0;  // R = t^{1/2} W^T: rows mutually orthogonal
  }
}

// ---------------------------------------------------------------------------
// Truncation step: SVD of R (k x b) by one-sided Jacobi on R^T, rank L with
// the Frobenius-tail rule, GU = Glast U_R[:, :L] and
// Pnext = Sigma_L V_R[:, :L]^T Fn^T.
// ---------------------------------------------------------------------------
__device__ void trunc_step_body(const TruncArgs a) {
  __shared__ double A[TTR_RMAX * TTR_RMAX];   // R^T, b x k
  __shared__ double Um[TTR_RMAX * TTR_RMAX];  // k x k rotations = U_R
  __shared__ double sv[TTR_RMAX];
  __shared__ double ss[TTR_RMAX];
  __shared__ int perm[TTR_RMAX];
  __shared__ int flag, LL;
  const int k = a.k, b = a.b;
  int ident = a.identity;
  if (!ident && k == b && k > 0) {
    // R upper triangular (Cholesky-based factorizations): sigma_min(R) >=
    // 1 / ||R^{-1}||_F, so no direction can be dropped when that bound exceeds
    // 2 delta (the Frobenius tail of any truncation would exceed delta).
    __shared__ int tri_ok;
    if (threadIdx.x == 0) tri_ok = 1;
    __syncthreads();
    for (int e = threadIdx.x; e < k * k; e += blockDim.x)
      if (e % k > e / k && a.R[e] != 0.0) tri_ok = 0;
    __syncthreads();
    if (tri_ok) {
      for (int c = threadIdx.x; c < k; c += blockDim.x)
        for (int r = k - 1; r >= 0; --r) {
          if (r > c) {
            A[r + k * c] = 0.0;
            continue;
          }
          double v = (r == c) ? 1.0 : 0.0;
          for (int m = r + 1; m <= c; ++m) v -= a.R[r + k * m] * A[m + k * c];
          A[r + k * c] = v / a.R[r + k * r];
        }
      __syncthreads();
      const double xf2 = sumsq(A, k * k);
      const double n2 = sumsq(a.R, k * k);
      const double dl2 = a.first ? ((a.Nm1 > 0) ? a.tol * a.tol * n2 / (double)a.Nm1 : 0.0) : (*a.delta) * (*a.delta);
      ident = (xf2 > 0.0 && finite(xf2) && 1.0 / xf2 > 4.0 * dl2) ? 1 : 0;
      __syncthreads();
    }
  }
  if (ident) {
    // no truncation possible (proved here or by the step kernel): U = I, Sigma V^T = R
    const double n2 = sumsq(a.R, k * b);
    if (threadIdx.x == 0) {
      if (a.first) {
        const double nrm = sqrt(n2);
        *a.norm = nrm;
        *a.delta = (a.Nm1 > 0) ? a.tol * nrm / sqrt((double)a.Nm1) : 0.0;
      }
      for (int j = 0; j < TTR_RMAX; ++j) a.sigma_out[j] = 0.0;
      if (a.tail_out) *a.tail_out = 0.0;
      a.dec[3] = k;
      a.dec[9] = 0;
    }
    const int d = a.d;
    for (int e = threadIdx.x; e < d * k; e += blockDim.x) a.GU[e] = a.Glast[e];
    if (a.Pnext) {
      const int dn = a.dn;
      for (int e = threadIdx.x; e < k * dn; e += blockDim.x) {
        const int l = e % k, r = e / k;
        double s = 0.0;
        for (int j = 0; j < b; ++j) s += a.R[l + k * j] * a.Fn[r + dn * j];
        a.Pnext[l + k * r] = s;
      }
    }
    return;
  }
  for (int e = threadIdx.x; e < b * k; e += blockDim.x) {
    const int r = e % b, c = e / b;     // A(r, c) = R(c, r)
    A[r + b * c] = a.R[c + k * r];
  }
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) Um[e] = (e % k == e / k) ? 1.0 : 0.0;
  __syncthreads();
  // rows of R already orthogonal (one-pass eigen route, R = t^{1/2} W^T): no rotations needed
  const int sweeps = a.r_orth ? 1 : jacobi_onesided(A, b, k, Um, &flag);
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    double s = 0.0;
    for (int r = 0; r < b; ++r) s += A[r + b * j] * A[r + b * j];
    sv[j] = sqrt(s);
  }
  __syncthreads();
  sort_desc(sv, k, perm);
  if (threadIdx.x < k) ss[threadIdx.x] = sv[perm[threadIdx.x]];
  __syncthreads();
  if (threadIdx.x == 0) {
    if (sweeps < 0) a.dec[2] |= 2;
    if (a.first) {
      double n2 = 0.0;
      for (int j = k - 1; j >= 0; --j) n2 += ss[j] * ss[j];
      const double nrm = sqrt(n2);
      *a.norm = nrm;
      *a.delta = (a.Nm1 > 0) ? a.tol * nrm / sqrt((double)a.Nm1) : 0.0;
    }
    const double delta = *a.delta;
    // smallest L >= 1 whose Frobenius tail sqrt(sum_{j >= L} s_j^2) <= delta
    double tail = 0.0;
    int L = k;
    for (int j = k - 1; j >= 1; --j) {
      tail += ss[j] * ss[j];
      if (sqrt(tail) <= delta) L = j;
      else break;
    }
    LL = L;
    for (int j = 0; j < TTR_RMAX; ++j) a.sigma_out[j] = (j < k) ? ss[j] : 0.0;
    if (a.tail_out) {
      double t2 = 0.0;
      for (int j = k - 1; j >= L; --j) t2 += ss[j] * ss[j];
      *a.tail_out = t2;
    }
    a.dec[3] = L;
    a.dec[9] = sweeps < 0 ? -sweeps : sweeps;
  }
  __syncthreads();
  const int L = LL;
  const int d = a.d;
  // GU (d x L) = Glast (d x k) * U_R[:, perm[:L]]
  for (int e = threadIdx.x; e < d * L; e += blockDim.x) {
    const int r = e % d, c = e / d;
    const int pc = perm[c];
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += a.Glast[r + d * j] * Um[j + k * pc];
    a.GU[r + d * c] = s;
  }
  // Pnext (L x dn) = sigma_l v_l^T Fn^T with sigma_l v_l = A(:, perm[l])
  if (a.Pnext) {
    const int dn = a.dn;
    for (int e = threadIdx.x; e < L * dn; e += blockDim.x) {
      const int l = e % L, r = e / L;
      const int pc = perm[l];
      double s = 0.0;
      for (int j = 0; j < b; ++j) s += A[j + b * pc] * a.Fn[r + dn * j];
      a.Pnext[l + L * r] = s;
    }
  }
}

__device__ void small_gemm_body(const double *A, const double *B, double *C, int m, int k, int n) {
  for (int e = threadIdx.x; e < m * n; e += blockDim.x) {
    const int r = e % m, c = e / m;
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += A[r + m * j] * B[j + k * c];
    C[r + m * c] = s;
  }
}

// ---------------------------------------------------------------------------
// Factor of the symmetric inner-product norm (§3.2.4).  G (d x d, symmetric
// positive semi-definite, ld d) -> F (d x d, ld d) upper triangular with
// F^T F = G to rounding error and zero rows past the numerical rank k.
// When every pivot of the unpivoted Cholesky G = L L^T exceeds d u max G_jj,
// F = L^T.  Otherwise (G numerically singular) pivoted Cholesky gives
// G = P L L^T P^T, stopping at pivots <= d u max G_jj; B = L^T P^T (k x d)
// then has B^T B = G, and Householder QR of B, B = Q F, turns it into the
// upper-trapezoidal F with the same F^T F.  The triangle is what lets the
// streaming pass skip the zero half of F X_n(i).  Non-finite G gives an
// all-NaN F, so the norm comes out NaN.
// ---------------------------------------------------------------------------
__device__ void sym_factor_body(const double *__restrict__ G, int d, double *__restrict__ F) {
  __shared__ double A[TTR_RMAX * TTR_RMAX];
  __shared__ double Bm[TTR_RMAX * TTR_RMAX];
  __shared__ double vh[TTR_RMAX];
  __shared__ int perm[TTR_RMAX];
  __shared__ double hbeta;
  double bad = 0.0;
  for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
    const double g = G[e];
    A[e] = g;
    if (!finite(g)) bad = 1.0;
  }
  bad = block_max(bad);  // also the barrier after the loads
  if (bad > 0.0) {
    for (int e = threadIdx.x; e < d * d; e += blockDim.x) F[e] = NAN;
    return;
  }
  double m = 0.0;
  for (int i = threadIdx.x; i < d; i += blockDim.x) m = fmax(m, A[i + d * i]);
  m = block_max(m);
  if (chol_lower(A, d, (double)d * kU * m)) {
    for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
      const int r = e % d, c = e / d;
      F[e] = (c >= r) ? A[c + d * r] : 0.0;
    }
    return;
  }
  __syncthreads();  // every thread has left the factorization before A is reloaded
  for (int e = threadIdx.x; e < d * d; e += blockDim.x) A[e] = G[e];
  __syncthreads();
  const int k = pivoted_chol(A, d, (double)d * kU, perm);
  // B(r, perm[j]) = L(j, r) for j >= r, else 0 (ld TTR_RMAX)
  for (int e = threadIdx.x; e < k * d; e += blockDim.x) {
    const int r = e % k, j = e / k;
    Bm[r + TTR_RMAX * perm[j]] = (j >= r) ? A[j + d * r] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (threadIdx.x < kWave) {
      // reflector of column j below the diagonal: lane l holds row j + l
      const int i = j + threadIdx.x;
      const double x = (i < k) ? Bm[i + TTR_RMAX * j] : 0.0;
      double ss = x * x;
      for (int off = kWave / 2; off >= 1; off >>= 1) ss += __shfl_xor(ss, off, kWave);
      const double x0 = __shfl(x, 0, kWave);
      const double nx = sqrt(ss);
      const double alpha = (x0 >= 0.0) ? -nx : nx;
      if (i < k) vh[i] = (i == j) ? x0 - alpha : x;
      if (threadIdx.x == 0) hbeta = (nx > 0.0) ? 1.0 / (nx * (nx + fabs(x0))) : 0.0;  // 2 / v^T v
    }
    __syncthreads();
    const double beta = hbeta;
    for (int c = j + threadIdx.x; c < d; c += blockDim.x) {
      double sdot = 0.0;
      for (int i = j; i < k; ++i) sdot += vh[i] * Bm[i + TTR_RMAX * c];
      const double f = beta * sdot;
      for (int i = j; i < k; ++i) Bm[i + TTR_RMAX * c] -= f * vh[i];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
    const int r = e % d, c = e / d;
    F[e] = (r < k && c >= r) ? Bm[r + TTR_RMAX * c] : 0.0;
  }
}

__global__ __launch_bounds__(kThreadsQR) void k_qr_step(QrStepArgs a) { qr_step_body(a); }
__global__ __launch_bounds__(kThreadsQR) void k_sym_factor(const double *G, int d, double *F) {
  sym_factor_body(G, d, F);
}
__global__ __launch_bounds__(kThreads) void k_trunc_step(TruncArgs a) { trunc_step_body(a); }
// W (a x a) = P^T P for P (p x a, ld p), one workgroup: the Gram of a small
// left factor (its triangular factor F, F^T F = W, replaces P in a Gram pass).
__global__ __launch_bounds__(kThreadsQR) void k_ptp(const double *__restrict__ P, int p, int a,
                                                    double *__restrict__ W) {
  for (int e = threadIdx.x; e < a * a; e += blockDim.x) {
    const int r = e % a, c = e / a;
    double v = 0.0;
    for (int i = 0; i < p; ++i) v += P[i + (size_t)p * r] * P[i + (size_t)p * c];
    W[e] = v;
  }
}

__global__ void k_small_gemm(const double *A, const double *B, double *C, int m, int k, int n) {
  small_gemm_body(A, B, C, m, k, n);
}

// Batched forms: workgroup t handles item t when active[t] is set.
__global__ __launch_bounds__(kThreadsQR) void kb_qr_step(const QrStepArgs *args, const int *active) {
  if (!active[blockIdx.x]) return;
  qr_step_body(args[blockIdx.x]);
}
__global__ __launch_bounds__(kThreads) void kb_trunc_step(const TruncArgs *args, const int *active) {
  if (!active[blockIdx.x]) return;
  trunc_step_body(args[blockIdx.x]);
}
__global__ void kb_small_gemm(const SmallGemmArgs *args, const int *active) {
  if (!active[blockIdx.x]) return;
  const SmallGemmArgs g = args[blockIdx.x];
  small_gemm_body(g.A, g.B, g.C, g.m, g.k, g.n);
}

__global__ void k_sqrt_scalar(const double *in, double *out) {
  if (threadIdx.x == 0) {
    const double v = in[0];
    out[0] = v > 0 ? sqrt(v) : (v == v ? 0.0 : v);  // rounding residue below zero -> 0; NaN stays
  }
}

}  // namespace

void launch_qr_step(hipStream_t s, const QrStepArgs &a) {
  hipLaunchKernelGGL(k_qr_step, dim3(1), dim3(kThreadsQR), 0, s, a);
}

void launch_trunc_step(hipStream_t s, const TruncArgs &a) {
  hipLaunchKernelGGL(k_trunc_step, dim3(1), dim3(kThreads), 0, s, a);
}

void launch_small_gemm(hipStream_t s, const double *A, const double *B, double *C, int m, int k, int n) {
  hipLaunchKernelGGL(k_small_gemm, dim3(1), dim3(kThreads), 0, s, A, B, C, m, k, n);
}

void launch_qr_step_batched(hipStream_t s, int count, const QrStepArgs *args, const int *active) {
  hipLaunchKernelGGL(kb_qr_step, dim3(count), dim3(kThreadsQR), 0, s, args, active);
}
void launch_trunc_step_batched(hipStream_t s, int count, const TruncArgs *args, const int *active) {
  hipLaunchKernelGGL(kb_trunc_step, dim3(count), dim3(kThreads), 0, s, args, active);
}
void launch_small_gemm_batched(hipStream_t s, int count, const SmallGemmArgs *args, const int *active) {
  hipLaunchKernelGGL(kb_small_gemm, dim3(count), dim3(kThreads), 0, s, args, active);
}

void launch_sym_factor(hipStream_t s, const double *G, int d, double *F) {
  hipLaunchKernelGGL(k_sym_factor, dim3(1), dim3(kThreadsQR), 0, s, G, d, F);
}
void launch_ptp(hipStream_t s, const double *P, int p, int a, double *W) {
  hipLaunchKernelGGL(k_ptp, dim3(1), dim3(kThreadsQR), 0, s, P, p, a, W);
}
void launch_sqrt_scalar(hipStream_t s, const double *in, double *out) {
  hipLaunchKernelGGL(k_sqrt_scalar, dim3(1), dim3(64), 0, s, in, out);
}
