// Small dense FP64 kernels, one workgroup each, matrices (<= 64 x 64) in LDS.
//
// They turn the Gram matrices produced by the streaming passes into the
// factors the sweeps pass between cores:
//   * k_qr_step: one step of a rank-revealing, shift-stabilized Cholesky-QR
//     realized with eigendecompositions.  For a tall-skinny unfolding A
//     (accessed only through streaming passes) it yields B (b x k) and R
//     (k x b) with A*B column-orthonormal and A = (A*B) R to rounding error.
//     This plays the role of the tall-skinny QR of §3.3 (TSQR) in Alg. 5/6;
//     see the design doc for the derivation and accuracy argument.
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

constexpr int kThreads = 256;
constexpr int kWave = 64;
constexpr double kU = DBL_EPSILON / 2;  // unit roundoff 2^-53

__device__ inline double wave_sum(double v) {
  for (int off = kWave / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return __shfl(v, 0, kWave);  // one value for the whole wave
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
  __shared__ double fro2;
  if (threadIdx.x == 0) {
    double f = 0.0;
    for (int e = 0; e < m * n; ++e) f += A[e] * A[e];
    fro2 = f;
  }
  __syncthreads();
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
        const double alpha = wave_sum(ap * ap);
        const double beta = wave_sum(aq * aq);
        const double gamma = wave_sum(ap * aq);
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

__device__ inline bool finite(double x) { return x == x && fabs(x) <= DBL_MAX; }

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
__global__ __launch_bounds__(kThreads) void k_qr_step(QrStepArgs a) {
  __shared__ double A[TTR_RMAX * TTR_RMAX];
  __shared__ double Vm[TTR_RMAX * TTR_RMAX];
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
    __syncthreads();
    for (int e = threadIdx.x; e < m * d; e += blockDim.x) {
      const int r = e % m, c = e / m;
      double s = 0.0;
      for (int k = 0; k < m; ++k) s += A[r + m * k] * a.Tpost[k * a.tsr + c * a.tsc];
      Vm[r + m * c] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < d * d; e += blockDim.x) {
      const int r = e % d, c = e / d;
      double s = 0.0;
      for (int k = 0; k < m; ++k) s += a.Tpost[k * a.tsr + r * a.tsc] * Vm[k + m * c];
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
    }
    return;
  }
  const int sweeps = jacobi_onesided(A, d, d, Vm, &flag);
  // A = G V: eigenvalue j is the Rayleigh quotient v_j^T G v_j = v_j . A(:, j)
  for (int j = threadIdx.x; j < d; j += blockDim.x) {
    double s = 0.0;
    for (int r = 0; r < d; ++r) s += Vm[j * d + r] * A[j * d + r];
    lam[j] = s;
  }
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
      const double shift = (tmin >= a.tau1 * t1 * cs) ? 0.0 : 2.0 * d * kU * t1 + 2.0 * (tmin < 0 ? -tmin : 0.0);
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
    }
    return;
  }
  // F (d x k) = W[:, :k] diag(sc)
  for (int e = threadIdx.x; e < d * k; e += blockDim.x) {
    const int r = e % d, c = e / d;
    a.Fstep[r + d * c] = A[r + d * c] * sc[c];
  }
  // Rnext (k x b) = diag(rs) W[:, :k]^T Rc (d x b)
  for (int e = threadIdx.x; e < k * b; e += blockDim.x) {
    const int r = e % k, c = e / k;
    double s;
    if (a.Rc) {
      s = 0.0;
      for (int j = 0; j < d; ++j) s += A[j + d * r] * a.Rc[j + d * c];
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
  }
}

// ---------------------------------------------------------------------------
// Truncation step: SVD of R (k x b) by one-sided Jacobi on R^T, rank L with
// the Frobenius-tail rule, GU = Glast U_R[:, :L] and
// Pnext = Sigma_L V_R[:, :L]^T Fn^T.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_trunc_step(TruncArgs a) {
  __shared__ double A[TTR_RMAX * TTR_RMAX];   // R^T, b x k
  __shared__ double Um[TTR_RMAX * TTR_RMAX];  // k x k rotations = U_R
  __shared__ double sv[TTR_RMAX];
  __shared__ double ss[TTR_RMAX];
  __shared__ int perm[TTR_RMAX];
  __shared__ int flag, LL;
  const int k = a.k, b = a.b;
  for (int e = threadIdx.x; e < b * k; e += blockDim.x) {
    const int r = e % b, c = e / b;     // A(r, c) = R(c, r)
    A[r + b * c] = a.R[c + k * r];
  }
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) Um[e] = (e % k == e / k) ? 1.0 : 0.0;
  __syncthreads();
  const int sweeps = jacobi_onesided(A, b, k, Um, &flag);
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
    a.dec[3] = L;
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

__global__ void k_small_gemm(const double *A, const double *B, double *C, int m, int k, int n) {
  for (int e = threadIdx.x; e < m * n; e += blockDim.x) {
    const int r = e % m, c = e / m;
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += A[r + m * j] * B[j + k * c];
    C[r + m * c] = s;
  }
}

__global__ void k_sqrt_scalar(const double *in, double *out) {
  if (threadIdx.x == 0) {
    const double v = in[0];
    out[0] = v > 0 ? sqrt(v) : 0.0;
  }
}

}  // namespace

void launch_qr_step(hipStream_t s, const QrStepArgs &a) {
  hipLaunchKernelGGL(k_qr_step, dim3(1), dim3(kThreads), 0, s, a);
}

void launch_trunc_step(hipStream_t s, const TruncArgs &a) {
  hipLaunchKernelGGL(k_trunc_step, dim3(1), dim3(kThreads), 0, s, a);
}

void launch_small_gemm(hipStream_t s, const double *A, const double *B, double *C, int m, int k, int n) {
  hipLaunchKernelGGL(k_small_gemm, dim3(1), dim3(kThreads), 0, s, A, B, C, m, k, n);
}

void launch_sqrt_scalar(hipStream_t s, const double *in, double *out) {
  hipLaunchKernelGGL(k_sqrt_scalar, dim3(1), dim3(64), 0, s, in, out);
}
