// TT rounding for ranks above the register/LDS-tiled range (64 < R <= 256):
// the same algorithm as the single-tensor path (§2.4 Alg. 2, both sweep
// orders; QR-by-Gram for the tall-skinny QRs of §3.3-§3.5), with every
// streaming product a matrix-core GEMM on an unfolding (ttr_lstream.hip) and
// every small factorization done by one workgroup on matrices held in device
// memory.  Also the inner product, the orthonormalization norm, explicit
// orthonormalization and the rounding of an implicit Hadamard product at
// these ranks.
//
// Unfoldings of a core M (a x I x b, entry (i1, i, i2) at i1 + a*(i + I*i2)):
//   V(M) = (a*I) x b, H(M) = a x (I*b), both column-major views of the buffer.
// Products used (lg_gemm, B packed into fragment order once per call):
//   C = M x_3 T^T        V(C) = V(M) T
//   D = F^T x_1 C        H(D)^T = H(C)^T F
//   LEFT Gram            H(Z) H(Z)^T    (lg_gram over the row-major H(Z)^T)
//   RIGHT Gram           V(Z)^T V(Z)    (lg_gram over the column-major V(Z))
// Gram passes keep per-workgroup partial matrices summed in a fixed order.
// LRL rounding and left orthonormalization run the same code on the reversed
// train of transposed slices (LView).  Every refinement stage is applied to a
// materialized core, and the truncation sweep rebuilds the orthonormalization
// sweep's intermediates with the same calls, so each stage is applied to
// bitwise the data its Gram was measured on.
//
// Small factorizations (d <= 256): Cholesky with Gershgorin / norm bounds,
// shifted Cholesky and rank-revealing pivoted Cholesky run in one 1024-thread
// workgroup over device-memory scratch (L2-resident), Cholesky and triangular
// inverse blocked in 16-column panels; the products with the triangular
// factor (R = L^T Rc) are small matrix-core products (lg_sgemm).  The
// truncation SVD is a block one-sided Jacobi over many workgroups, one launch
// per round, converged when a sweep rotates nothing (checked on the device).
#include "ttr_host.h"

#include <algorithm>
#include <array>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

namespace {

constexpr int kLT = 1024;   // threads of the one-workgroup kernels
constexpr int kLMax = 256;  // largest rank of this path
constexpr double kU = 1.1102230246251565e-16;
constexpr double kTau1 = 1e-3;
constexpr double kTau2 = 1e-12;

__device__ inline bool lfinite(double x) { return x == x && fabs(x) <= DBL_MAX; }

// Block-wide sum and maximum: a butterfly within each wave (every lane ends
// with the same value), then the wave results added in wave order, so every
// thread returns the same value.
__device__ double lsum(double v) {
  __shared__ double part[kLT / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += part[w];
  __syncthreads();
  return r;
}

__device__ double lmax(double v) {
  __shared__ double part[kLT / 64];
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = part[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, part[w]);
  __syncthreads();
  return r;
}

// A (d x d, ld d) = the symmetric matrix whose lower triangle is that of G:
// each wave reads whole columns of G from the diagonal down (all its loads of
// a column in flight at once) and writes them and their mirror.  Returns true
// in every thread when an entry read was not finite.
__device__ bool lload_sym(const double *__restrict__ G, int d, double *__restrict__ A) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int bad = 0;
  for (int c = wave; c < d; c += nw) {
    double g[kLMax / 64];
#pragma unroll
    for (int m = 0; m < kLMax / 64; ++m) {
      const int r = c + lane + 64 * m;
      g[m] = (r < d) ? G[r + (size_t)d * c] : 0.0;
    }
#pragma unroll
    for (int m = 0; m < kLMax / 64; ++m) {
      const int r = c + lane + 64 * m;
      if (r < d) {
        if (!lfinite(g[m])) bad = 1;
        A[r + (size_t)d * c] = g[m];
        A[c + (size_t)d * r] = g[m];
      }
    }
  }
  return __syncthreads_or(bad) != 0;
}

// Y(j, i) = X(i, j) for X n x m (ld ldx) into Y (ld ldy): X read in order,
// four loads in flight per thread.
__device__ void ltrans(const double *__restrict__ X, int n, int m, int ldx, double *__restrict__ Y, int ldy) {
  const int tot = n * m, nt = blockDim.x;
  for (int e0 = threadIdx.x; e0 < tot; e0 += 4 * nt) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * nt;
      v[u] = (e < tot) ? X[e % n + (size_t)ldx * (e / n)] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * nt;
      if (e < tot) Y[e / n + (size_t)ldy * (e % n)] = v[u];
    }
  }
}

// Y = X for X n x m (ld ldx) into Y (ld ldy), four loads in flight per thread.
__device__ void lcopy(const double *__restrict__ X, int n, int m, int ldx, double *__restrict__ Y, int ldy) {
  const int tot = n * m, nt = blockDim.x;
  for (int e0 = threadIdx.x; e0 < tot; e0 += 4 * nt) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * nt;
      v[u] = (e < tot) ? X[e % n + (size_t)ldx * (e / n)] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * nt;
      if (e < tot) Y[e % n + (size_t)ldy * (e / n)] = v[u];
    }
  }
}

// Block-wide argmax: the largest v, the smallest p among equal v; the result
// is returned in every thread.
__device__ void largmax(double *v, int *p) {
  __shared__ double wv[kLT / 64];
  __shared__ int wp[kLT / 64];
  double bv = *v;
  int bp = *p;
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(bv, off, 64);
    const int op = __shfl_xor(bp, off, 64);
    if (ov > bv || (ov == bv && op < bp)) {
      bv = ov;
      bp = op;
    }
  }
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    wv[wave] = bv;
    wp[wave] = bp;
  }
  __syncthreads();
  bv = wv[0];
  bp = wp[0];
  for (int w = 1; w < nw; ++w)
    if (wv[w] > bv || (wv[w] == bv && wp[w] < bp)) {
      bv = wv[w];
      bp = wp[w];
    }
  __syncthreads();
  *v = bv;
  *p = bp;
}

constexpr int kNB = 16;                        // panel width of the blocked factorizations (registers: 1024-thread blocks leave 128 per lane)
constexpr int kLdsB = kLMax * (kNB + 1);       // doubles of LDS the blocked Cholesky's panel uses

// v from lane `lane` (uniform) of the wave, as a wave-uniform value.
__device__ inline double bcast(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Blocked right-looking Cholesky of the d x d symmetric A (device memory, ld
// d; lower triangle read) in place, strict upper part zeroed.  False if a
// pivot is not positive.  Per 16-column panel: wave 0 factors the diagonal
// block in registers (lane r holds row r; the pivot column is broadcast lane
// by lane), the rows below solve against it in parallel (one row per
// thread), and the trailing lower triangle takes the panel's rank-16 update
// with the panel held in LDS (S, kLdsB doubles).  Three barriers per panel.
typedef double lv4 __attribute__((ext_vector_type(4)));
__device__ bool lchol(double *A, int d, double *S) {
  __shared__ double Dk[kNB * kNB];
  __shared__ int okf;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) okf = 1;
  for (int k0 = 0; k0 < d; k0 += kNB) {
    const int nb = min(kNB, d - k0), k1 = k0 + nb;
    if (wave == 0) {
      const int r = lane;
      double a[kNB];
#pragma unroll
      for (int c = 0; c < kNB; ++c)
        a[c] = (r < nb && c <= r) ? A[(k0 + r) + (size_t)d * (k0 + c)] : 0.0;
      bool ok = true;
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        if (j < nb) {
          const double pv = bcast(a[j], j);
          if (!(pv > 0.0)) ok = false;
          const double sq = sqrt(pv);
          const double l = (r == j) ? sq : ((r > j) ? a[j] / sq : 0.0);
          a[j] = l;
#pragma unroll
          for (int c = j + 1; c < kNB; ++c) {
            const double lc = bcast(l, c);
            if (r >= c) a[c] -= l * lc;
          }
        }
      }
      if (r < kNB)
#pragma unroll
        for (int c = 0; c < kNB; ++c) Dk[r + kNB * c] = (c <= r && r < nb) ? a[c] : 0.0;
      if (r < nb)
#pragma unroll
        for (int c = 0; c < kNB; ++c)
          if (c <= r) A[(k0 + r) + (size_t)d * (k0 + c)] = a[c];
      if (r == 0 && !ok) okf = 0;
    }
    __syncthreads();
    if (!okf) return false;
    // panel below: L(i, k0:k1) = A(i, k0:k1) L_kk^{-T}, one row per thread
    // (d - k1 < blockDim: a single pass, so the reads of L_kk stay in the
    // loop body instead of being hoisted into registers)
    if (const int i = k1 + threadIdx.x; i < d) {
      double x[kNB];
#pragma unroll
      for (int c = 0; c < kNB; ++c) {
        double v = (c < nb) ? A[i + (size_t)d * (k0 + c)] : 0.0;
#pragma unroll
        for (int m = 0; m < c; ++m) v -= x[m] * Dk[c + kNB * m];
        x[c] = (c < nb) ? v / Dk[c + kNB * c] : 0.0;
      }
#pragma unroll
      for (int c = 0; c < kNB; ++c) {
        if (c < nb) A[i + (size_t)d * (k0 + c)] = x[c];
        S[(i - k1) * (kNB + 1) + c] = x[c];
      }
    }
    __syncthreads();
    // trailing update of the lower triangle, A(r, c) -= L(r, panel) L(c, panel)^T,
    // on the matrix cores: 16 x 16 tiles (ti >= tj) of the trailing matrix,
    // each the transposed product L(tj rows) (-L(ti rows))^T added to its
    // transposed tile, so that the 16 lanes of a row group hold 16
    // consecutive rows of one column (coalesced loads and stores)
    {
      const int g = lane >> 4, jj = lane & 15, nw = blockDim.x >> 6;
      const int T = (d - k1 + 15) / 16;
      for (int tix = wave; tix < T * T; tix += nw) {
        const int ti = tix / T, tj = tix % T;
        if (tj > ti) continue;
        const int row = k1 + 16 * ti + jj;
        lv4 acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = k1 + 16 * tj + 4 * r + g;
          acc[r] = (row < d && col < d) ? A[row + (size_t)d * col] : 0.0;
        }
#pragma unroll
        for (int ks = 0; ks < kNB / 4; ++ks)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(S[(16 * tj + jj) * (kNB + 1) + 4 * ks + g],
                                                     -S[(16 * ti + jj) * (kNB + 1) + 4 * ks + g], acc, 0, 0, 0);
        // register r: element (row, k1 + 16 tj + 4 r + g)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = k1 + 16 * tj + 4 * r + g;
          if (row < d && col < d && row >= col) A[row + (size_t)d * col] = acc[r];
        }
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < d * d; e += blockDim.x)
    if (e % d < e / d) A[e] = 0.0;
  __syncthreads();
  return true;
}

// X = L^{-1} (k x k lower, ld d) for the lower-triangular L in A (ld d).
// The diagonal 16-blocks are inverted by one wave each in registers (forward
// substitution on all columns at once, rows broadcast lane by lane); then
// blocks are paired and doubled, 16 -> 32 -> ... -> k: for L = [L00 0; L10
// L11] with X00, X11 known, X10 = -X11 (L10 X00), two products on the matrix
// cores per level.  W = L10 X00 is kept (transposed) in the strictly upper
// block X(B0, B1), which is cleared after the level, so X stays lower
// triangular between levels and the products skip its zero k-steps.
__device__ void linv(const double *A, double *X, int k, int d) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int nblk = (k + kNB - 1) / kNB;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int r = e % k, c = e / k;
    if (r < c) X[r + (size_t)d * c] = 0.0;
  }
  // nblk <= 16 = the waves of the workgroup: one diagonal block per wave
  if (const int bw = wave; bw < nblk) {
    const int b0 = bw * kNB, nb = min(kNB, k - b0);
    const int r = lane;
    double l[kNB], x[kNB];
#pragma unroll
    for (int c = 0; c < kNB; ++c) {
      l[c] = (r < nb && c <= r) ? A[(b0 + r) + (size_t)d * (b0 + c)] : 0.0;
      x[c] = (r == c) ? 1.0 : 0.0;
    }
#pragma unroll
    for (int m = 0; m < kNB; ++m) {
      if (m < nb) {
        const double pm = 1.0 / bcast(l[m], m);
#pragma unroll
        for (int c = 0; c <= m; ++c) {
          const double xm = bcast(x[c], m) * pm;  // row m of X, final
          if (r > m) x[c] -= l[m] * xm;
          else if (r == m) x[c] = xm;
        }
      }
    }
    if (r < nb)
#pragma unroll
      for (int c = 0; c < kNB; ++c)
        if (c <= r) X[(b0 + r) + (size_t)d * (b0 + c)] = x[c];
  }
  __syncthreads();
  const int g = lane >> 4, jj = lane & 15;
  auto lget = [&](int r, int c) { return (r < k && c < k) ? A[r + (size_t)d * c] : 0.0; };
  auto xget = [&](int r, int c) { return (r < k && c < k) ? X[r + (size_t)d * c] : 0.0; };
  for (int m = kNB; m < k; m *= 2) {
    const int tm = m / 16;                          // 16-tiles per block side
    const int npair = (k - m + 2 * m - 1) / (2 * m);  // pairs whose B1 = [i0 + m, i0 + 2m) is not empty
    const int ntile = npair * tm * tm;
    // W (B1 rows x B0 columns) = L(B1, B0) X(B0, B0): tile (tr, tc) of W
    for (int tix = wave; tix < ntile; tix += nw) {
      const int pr = tix / (tm * tm), tr = (tix % (tm * tm)) / tm, tc = tix % tm;
      const int i0 = 2 * m * pr, b1 = i0 + m;
      if (b1 + 16 * tr >= k) continue;
      lv4 acc = {0.0, 0.0, 0.0, 0.0};
      // X(B0, B0)(kk, c) = 0 for kk < c: k-steps from the tile's first column
#pragma unroll 4
      for (int ks = 4 * tc; ks < m / 4; ++ks)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(lget(b1 + 16 * tr + jj, i0 + 4 * ks + g),
                                                   xget(i0 + 4 * ks + g, i0 + 16 * tc + jj), acc, 0, 0, 0);
      // register r: W(16 tr + 4 r + g, 16 tc + jj), kept as X(i0 + 16 tc + jj, b1 + 16 tr + 4 r + g)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (b1 + 16 * tr + 4 * r + g < k) X[(i0 + 16 * tc + jj) + (size_t)d * (b1 + 16 * tr + 4 * r + g)] = acc[r];
    }
    __syncthreads();
    // X(B1, B0) = -X(B1, B1) W
    for (int tix = wave; tix < ntile; tix += nw) {
      const int pr = tix / (tm * tm), tr = (tix % (tm * tm)) / tm, tc = tix % tm;
      const int i0 = 2 * m * pr, b1 = i0 + m;
      if (b1 + 16 * tr >= k) continue;
      lv4 acc = {0.0, 0.0, 0.0, 0.0};
      // X(B1, B1)(r, kk) = 0 for kk > r: k-steps up to the tile's last row
#pragma unroll 4
      for (int ks = 0; ks < 4 * (tr + 1); ++ks)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xget(b1 + 16 * tr + jj, b1 + 4 * ks + g),
                                                   xget(i0 + 16 * tc + jj, b1 + 4 * ks + g), acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (b1 + 16 * tr + 4 * r + g < k) X[(b1 + 16 * tr + 4 * r + g) + (size_t)d * (i0 + 16 * tc + jj)] = -acc[r];
    }
    __syncthreads();
    // clear the kept W: X(B0, B1) back to the zero upper part
    for (int e = threadIdx.x; e < npair * m * m; e += blockDim.x) {
      const int pr = e / (m * m), r = (e % (m * m)) % m, c = (e % (m * m)) / m;
      const int i0 = 2 * m * pr;
      if (i0 + m + c < k) X[(i0 + r) + (size_t)d * (i0 + m + c)] = 0.0;
    }
    __syncthreads();
  }
}

// ||M||_1, ||M||_inf and ||M||_F^2 of the k x k matrix M (ld d).  Row sums
// run one row per thread (lanes read consecutive rows of a column), column
// sums one column per wave (lanes read down the column).
__device__ void lnorms(const double *M, int k, int d, double *n1, double *ni, double *f2) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double a1 = 0.0, ai = 0.0, af = 0.0;
  for (int r = threadIdx.x; r < k; r += blockDim.x) {
    double t = 0.0;
    for (int c = 0; c < k; ++c) {
      const double v = M[r + (size_t)d * c];
      t += fabs(v);
      af += v * v;
    }
    ai = fmax(ai, t);
  }
  for (int c = wave; c < k; c += nw) {
    double s = 0.0;
    for (int r = lane; r < k; r += 64) s += fabs(M[r + (size_t)d * c]);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    a1 = fmax(a1, s);
  }
  *n1 = lmax(a1);
  *ni = lmax(ai);
  *f2 = lsum(af);
}

// Rank-revealing pivoted Cholesky (as in the d <= 64 kernels), A in device
// memory: pivots in order perm[0..k), on return A(i, j) (i >= j, j < k) holds
// L with G(perm, perm) ~= L L^T; stops once the largest remaining diagonal
// entry is at most tau times the largest initial one.  Returns k.  Only the
// lower triangle is kept: the symmetric interchange of rows/columns j and p
// moves lower-triangle entries only, and step j updates the trailing lower
// triangle with the unscaled column j (L(r,j) L(c,j) = A(r,j) A(c,j) / A(j,j)),
// column j being scaled one step later (scaling commutes with the row
// interchanges of the next step).
__device__ int lpivchol(double *A, int d, double tau, int *perm) {
  __shared__ int piv, stop;
  __shared__ double dmax0;
  for (int i = threadIdx.x; i < d; i += blockDim.x) perm[i] = i;
  double m0 = 0.0;
  for (int i = threadIdx.x; i < d; i += blockDim.x) m0 = fmax(m0, A[i + (size_t)d * i]);
  m0 = lmax(m0);
  if (threadIdx.x == 0) dmax0 = m0;
  __syncthreads();
  const int tr = threadIdx.x & 31, tc = threadIdx.x >> 5, nc = blockDim.x >> 5;
  int k = d;
  double lprev = 0.0;  // L(j-1, j-1), for the deferred scaling of column j-1
  for (int j = 0; j < d; ++j) {
    {
      // the largest remaining diagonal entry, the first one among ties
      double v = -DBL_MAX;
      int p = d;
      for (int i = j + threadIdx.x; i < d; i += blockDim.x) {
        const double di = A[i + (size_t)d * i];
        if (di > v) {
          v = di;
          p = i;
        }
      }
      largmax(&v, &p);
      if (threadIdx.x == 0) {
        piv = p;
        stop = !(v > tau * dmax0) || p >= d;
      }
      __syncthreads();
    }
    if (stop) {
      k = j;
      break;
    }
    const int p = piv;
    if (p != j) {
      // symmetric interchange j <-> p (j < p) on the lower triangle
      for (int c = threadIdx.x; c < j; c += blockDim.x) {  // rows of L so far
        const double t = A[j + (size_t)d * c];
        A[j + (size_t)d * c] = A[p + (size_t)d * c];
        A[p + (size_t)d * c] = t;
      }
      for (int m = j + 1 + threadIdx.x; m < p; m += blockDim.x) {  // column j between <-> row p
        const double t = A[m + (size_t)d * j];
        A[m + (size_t)d * j] = A[p + (size_t)d * m];
        A[p + (size_t)d * m] = t;
      }
      for (int m = p + 1 + threadIdx.x; m < d; m += blockDim.x) {  // below p: columns j and p
        const double t = A[m + (size_t)d * j];
        A[m + (size_t)d * j] = A[m + (size_t)d * p];
        A[m + (size_t)d * p] = t;
      }
      if (threadIdx.x == 0) {
        const double t = A[j + (size_t)d * j];
        A[j + (size_t)d * j] = A[p + (size_t)d * p];
        A[p + (size_t)d * p] = t;
        const int ti = perm[j];
        perm[j] = perm[p];
        perm[p] = ti;
      }
      __syncthreads();
    }
    const double pv = A[j + (size_t)d * j];
    if (j > 0)
      for (int r = j - 1 + threadIdx.x; r < d; r += blockDim.x)
        A[r + (size_t)d * (j - 1)] = (r == j - 1) ? lprev : A[r + (size_t)d * (j - 1)] / lprev;
    const double rp = 1.0 / pv;
    for (int c = j + 1 + tc; c < d; c += nc) {
      const double acj = A[c + (size_t)d * j] * rp;
      for (int r = c + tr; r < d; r += 32) A[r + (size_t)d * c] -= A[r + (size_t)d * j] * acj;
    }
    lprev = sqrt(pv);
    __syncthreads();
  }
  if (k > 0) {
    for (int r = k - 1 + threadIdx.x; r < d; r += blockDim.x)
      A[r + (size_t)d * (k - 1)] = (r == k - 1) ? lprev : A[r + (size_t)d * (k - 1)] / lprev;
    __syncthreads();
  }
  return k;
}

struct LStepArgs {
  const double *G;     // d x d (its lower triangle is read)
  int d, pass, b;
  const double *Rc;    // d x b (ld d), nullptr at the first pass
  double *Fstep;       // d x k (ld d)
  double *Rnext;       // k x b (ld k)
  double *Tdst;        // b x k (ld b) once settled, or nullptr
  int *dec;            // [0] k, [1] settled, [2] error flags, [5] no truncation proven,
                       // [8] R left to the host: 1 = L^T Rc, 2 = L(:, 0:k)^T Rp
  double tau1, tau2, ugram, gerr;
  int shift_pass;      // last pass that may take the shifted route (2 in mixed precision)
  int notrunc_check;
  const double *delta_dev;
  int first;
  double tol2_nm1;
  double *W0, *W1;     // d x d scratch
  int *perm;           // d scratch
  double *Rp;          // d x b scratch: permuted rows of Rc (pivoted route)
};

// One QR-by-Gram step (the d <= 64 step's Cholesky-based routes).
__global__ __launch_bounds__(kLT) void lk_step(LStepArgs a) {
  const int d = a.d;
  double *A = a.W0, *X = a.W1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __shared__ int accept;
  if (lload_sym(a.G, d, A)) {
    if (threadIdx.x == 0) {
      a.dec[2] |= 1;
      a.dec[0] = 1;
      a.dec[1] = 1;
      a.dec[8] = 0;
    }
    return;
  }
  // Gershgorin bounds and ||G||_1 (= ||G||_inf) from the off-diagonal
  // absolute sums of the rows, which are those of the columns (G symmetric):
  // one wave per column, its loads in flight at once.  kappa(G) >= max_j G_jj
  // / min_j G_jj (each G_jj is a Rayleigh quotient): when that already
  // exceeds 1/tau1 the Cholesky route cannot be taken and is not tried.
  double tp = 0.0, glo = DBL_MAX, ghi = 0.0, g1 = 0.0, gdx = 0.0, gdn = DBL_MAX;
  for (int c = wave; c < d; c += nw) {
    double v[kLMax / 64];
#pragma unroll
    for (int m = 0; m < kLMax / 64; ++m) {
      const int r = lane + 64 * m;
      v[m] = (r < d && r != c) ? fabs(A[r + (size_t)d * c]) : 0.0;
    }
    double off = 0.0;
#pragma unroll
    for (int m = 0; m < kLMax / 64; ++m) off += v[m];
    for (int o = 32; o > 0; o >>= 1) off += __shfl_xor(off, o, 64);
    const double drr = A[c + (size_t)d * c];
    if (lane == 0) {
      tp += drr;
      glo = fmin(glo, drr - off);
      ghi = fmax(ghi, drr + off);
      g1 = fmax(g1, fabs(drr) + off);
      gdx = fmax(gdx, drr);
      gdn = fmin(gdn, drr);
    }
  }
  const double trG = lsum(tp), gmin = -lmax(-glo), gmax = lmax(ghi);
  g1 = lmax(g1);
  gdx = lmax(gdx);
  gdn = -lmax(-gdn);
  __shared__ double Sbuf[kLdsB];
  const bool ok = (gdn > 0.0 && gdx * a.tau1 <= gdn) && lchol(A, d, Sbuf);
  double kappa = 1e300, lmin_lb = 0.0;
  // kappa(G) = kappa(L)^2 >= (max_j L_jj / min_j L_jj)^2 (the diagonal of a
  // triangular matrix holds its eigenvalues): when that already exceeds
  // 1/tau1 the step is rejected without forming L^{-1}
  double dmx = 0.0, dmn = DBL_MAX;
  if (ok)
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
      dmx = fmax(dmx, A[j + (size_t)d * j]);
      dmn = fmin(dmn, A[j + (size_t)d * j]);
    }
  dmx = lmax(dmx);
  dmn = -lmax(-dmn);
  const double klow = (dmx / dmn) * (dmx / dmn);
  if (ok && !(klow * a.tau1 <= 1.0)) {
    kappa = klow;
  } else if (ok) {
    linv(A, X, d, d);
    double x1, xi, xf;
    lnorms(X, d, d, &x1, &xi, &xf);
    kappa = g1 * x1 * xi;
    lmin_lb = 1.0 / fmin(xf, x1 * xi);
    if (gmin > 0.0) {
      kappa = fmin(kappa, gmax / gmin);
      lmin_lb = fmax(lmin_lb, gmin);
    }
  }
  if (threadIdx.x == 0) {
    int acc = ok && kappa == kappa && kappa * a.tau1 <= 1.0;
    int nt = 0;
    if (acc && a.notrunc_check && a.pass == 1) {
      const double dl = a.first ? sqrt(a.tol2_nm1 * trG) : *a.delta_dev;
      nt = (lmin_lb - a.gerr * trG > 4.0 * dl * dl);
    }
    accept = acc;
    a.dec[5] = nt;
  }
  __syncthreads();
  const int b = a.b;
  if (accept) {
    ltrans(X, d, d, d, a.Fstep, d);  // F = L^{-T}
    // R = L^T (first pass), T = R^T = L; at a refinement pass R = L^T Rc is
    // left to the host (dec[8] = 1: one small product with L in W0)
    if (!a.Rc) {
      ltrans(A, b, d, d, a.Rnext, d);
      if (a.Tdst) lcopy(A, b, d, d, a.Tdst, b);
    }
    if (threadIdx.x == 0) {
      a.dec[0] = d;
      a.dec[1] = 1;
      a.dec[8] = a.Rc ? 1 : 0;
    }
    return;
  }
  // restore G
  lload_sym(a.G, d, A);
  if (a.pass <= a.shift_pass) {
    // shifted CholeskyQR: the next pass refines
    const double shift = 2.0 * d * a.ugram * trG;
    for (int j = threadIdx.x; j < d; j += blockDim.x) A[j + (size_t)d * j] += shift;
    __syncthreads();
    if (shift > 0.0 && lchol(A, d, Sbuf)) {
      linv(A, X, d, d);
      ltrans(X, d, d, d, a.Fstep, d);
      if (!a.Rc) ltrans(A, d, d, d, a.Rnext, d);  // R = L^T (Rc = I)
      if (threadIdx.x == 0) {
        a.dec[0] = d;
        a.dec[1] = 0;
        a.dec[5] = 0;
        a.dec[8] = a.Rc ? 1 : 0;  // a refinement pass: R = L^T Rc by the host's product
      }
      return;
    }
    // a Gram too far from positive definite for the shift: pivoted below
    lload_sym(a.G, d, A);
  }
  // rank-revealing pivoted Cholesky
  int k = lpivchol(A, d, a.tau2, a.perm);
  if (k == 0) {
    // zero Gram: rank 1, zero factor
    for (int e = threadIdx.x; e < d; e += blockDim.x) a.Fstep[e] = (e == 0) ? 1.0 : 0.0;
    for (int e = threadIdx.x; e < b; e += blockDim.x) {
      a.Rnext[e] = 0.0;
      if (a.Tdst) a.Tdst[e] = 0.0;
    }
    if (threadIdx.x == 0) {
      a.dec[0] = 1;
      a.dec[1] = 1;
      a.dec[5] = 0;
      a.dec[8] = 0;
    }
    return;
  }
  linv(A, X, k, d);
  double x1, xi, xf, gk = 0.0;
  lnorms(X, k, d, &x1, &xi, &xf);
  // ||G(perm, perm)(0:k, 0:k)||_1, one wave per column
  for (int c = wave; c < k; c += nw) {
    const int pc = a.perm[c];
    double v[kLMax / 64];
#pragma unroll
    for (int m = 0; m < kLMax / 64; ++m) {
      const int r = lane + 64 * m;
      const int pr = (r < k) ? a.perm[r] : 0;
      v[m] = (r < k) ? fabs((pr >= pc) ? a.G[pr + (size_t)d * pc] : a.G[pc + (size_t)d * pr]) : 0.0;
    }
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < kLMax / 64; ++m) s += v[m];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    gk = fmax(gk, s);
  }
  gk = lmax(gk);
  const int dn = (a.pass >= 3 || (a.pass >= 2 && gk * x1 * xi * a.tau1 <= 1.0)) ? 1 : 0;
  for (int e = threadIdx.x; e < d * k; e += blockDim.x) a.Fstep[e] = 0.0;
  __syncthreads();
  // F(perm[i], c) = X(c, i) for c >= i (the rest stays zero), X read in order
  for (int e0 = threadIdx.x; e0 < k * k; e0 += 4 * (int)blockDim.x) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * (int)blockDim.x, c = e % k, i = e / k;
      v[u] = (e < k * k && c >= i) ? X[c + (size_t)d * i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * (int)blockDim.x, c = e % k, i = e / k;
      if (e < k * k && c >= i) a.Fstep[a.perm[i] + (size_t)d * c] = v[u];
    }
  }
  // R' = L(:, 0:k)^T Rc(perm, :) (Rc = I at the first pass) is left to the
  // host (dec[8] = 2: one small product with L in W0 and the permuted rows in Rp);
  // the strict upper part of L's k columns still holds Schur-complement
  // entries and is cleared first
  for (int e = threadIdx.x; e < d * k; e += blockDim.x)
    if (e % d < e / d) A[e] = 0.0;
  for (int e0 = threadIdx.x; e0 < d * b; e0 += 4 * (int)blockDim.x) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * (int)blockDim.x, j = e % d, col = e / d;
      v[u] = (e < d * b) ? (a.Rc ? a.Rc[a.perm[j] + (size_t)d * col] : (a.perm[j] == col ? 1.0 : 0.0)) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * (int)blockDim.x;
      if (e < d * b) a.Rp[e] = v[u];
    }
  }
  if (threadIdx.x == 0) {
    a.dec[0] = k;
    a.dec[1] = dn;
    a.dec[5] = 0;
    a.dec[8] = 2;
  }
}

struct LTruncArgs {
  const double *R;      // k x b (ld k)
  int k, b;
  double *delta, *norm;
  int first;
  double tol;
  int Nm1;
  double *sigma_out;    // kLMax values (descending, zero padded)
  double *tail_out;     // sum of squares of the discarded singular values
  int *dec;             // [3] L, [2] error flags, [7] no truncation (set by lk_trunc_setup)
  int identity;         // no truncation already proven by the first Gram pass
  double *W0, *W1;      // scratch: W0 b x k (R^T, then A), W1 k x k (U)
  double *thr;          // [0] Jacobi rotation threshold, [1] column-norm floor
  double *sv;           // k
  int *perm;            // k
  double *Up, *Ap;      // gathered U(:, perm[0:L]) (k x L), A(:, perm[0:L]) (b x L)
};

// Truncation (Alg. 2 inner step), part 1.  Decides whether the SVD of R can
// be skipped (no singular value can fall below delta); if so sets the norm
// and threshold at the first link and dec[3] = k, dec[7] = 1.  Otherwise sets
// up the one-sided Jacobi SVD of R: W0 = A = R^T (b x k), W1 = U = I (k x k),
// and the rotation thresholds.
__global__ __launch_bounds__(kLT) void lk_trunc_setup(LTruncArgs a) {
  const int k = a.k, b = a.b;
  __shared__ int ident, tri_ok;
  if (threadIdx.x == 0) {
    ident = a.identity;
    tri_ok = 1;
  }
  __syncthreads();
  if (!ident && k == b) {
    // upper-triangular R: sigma_min >= 1 / ||R^{-1}||_F proves that nothing can be dropped
    for (int e = threadIdx.x; e < k * k; e += blockDim.x)
      if (e % k > e / k && a.R[e] != 0.0) tri_ok = 0;
    __syncthreads();
    if (tri_ok) {
      // ||R^{-1}||_F = ||(R^T)^{-1}||_F, R^T lower triangular
      for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
        const int r = e % k, c = e / k;
        a.W0[r + (size_t)k * c] = a.R[c + (size_t)k * r];
      }
      __syncthreads();
      bool okd = true;
      for (int j = 0; j < k; ++j) okd = okd && (a.R[j + (size_t)k * j] != 0.0);
      double xf = 0.0, rf = 0.0;
      if (okd) {
        linv(a.W0, a.W1, k, k);
        for (int e = threadIdx.x; e < k * k; e += blockDim.x) xf += a.W1[e] * a.W1[e];
      }
      for (int e = threadIdx.x; e < k * k; e += blockDim.x) rf += a.R[e] * a.R[e];
      xf = lsum(xf);
      rf = lsum(rf);
      if (threadIdx.x == 0) {
        const double dl2 = a.first ? ((a.Nm1 > 0) ? a.tol * a.tol * rf / (double)a.Nm1 : 0.0) : (*a.delta) * (*a.delta);
        ident = (okd && xf > 0.0 && lfinite(xf) && 1.0 / xf > 4.0 * dl2) ? 1 : 0;
      }
      __syncthreads();
    }
  }
  if (ident) {
    double n2 = 0.0;
    for (int e = threadIdx.x; e < k * b; e += blockDim.x) n2 += a.R[e] * a.R[e];
    n2 = lsum(n2);
    if (threadIdx.x == 0) {
      if (a.first) {
        const double nrm = sqrt(n2);
        *a.norm = nrm;
        *a.delta = (a.Nm1 > 0) ? a.tol * nrm / sqrt((double)a.Nm1) : 0.0;
      }
      for (int j = 0; j < kLMax; ++j) a.sigma_out[j] = 0.0;
      *a.tail_out = 0.0;
      a.dec[3] = k;
      a.dec[7] = 1;
    }
    return;
  }
  for (int e = threadIdx.x; e < b * k; e += blockDim.x) {
    const int r = e % b, c = e / b;
    a.W0[r + (size_t)b * c] = a.R[c + (size_t)k * r];
  }
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) a.W1[e] = (e % k == e / k) ? 1.0 : 0.0;
  double f2 = 0.0;
  for (int e = threadIdx.x; e < b * k; e += blockDim.x) f2 += a.R[e] * a.R[e];
  f2 = lsum(f2);
  if (threadIdx.x == 0) {
    a.thr[0] = kU * 4.0 * sqrt((double)(b > 1 ? b : 1));
    a.thr[1] = (8.0 * (b + k) * kU) * (8.0 * (b + k) * kU) * f2;
    a.dec[7] = 0;
  }
}

__device__ inline void lrr_pair(int r, int kq, int nn, int *p, int *q) {
  if (kq == 0) {
    *p = r;
    *q = nn - 1;
  } else {
    const int m = nn - 1;
    *p = (r + kq) % m;
    *q = (r - kq + m) % m;
  }
}

// One round of the block one-sided Jacobi SVD of A (b x k, b, k <= 256): the
// k columns form nbp (even) blocks of kJW; in round `round` workgroup `pair`
// holds block P and block Q of the round-robin pairing, and each 16-lane row
// of its waves one column pair (lane j: rows j, j + 16, ...), so a wave
// rotates four pairs at once.  The P columns stay; in kJW steps every (P, Q)
// column pair is rotated once, the Q columns moving between the rows of a
// wave by lane shuffles and between waves through LDS every fourth step.
// Round 0 of a sweep first rotates the pairs inside P and inside Q (kJW - 1
// steps in LDS), so a sweep of nbp - 1 rounds rotates each of the k(k-1)/2
// pairs once.  The three inner products of a pair are row
// sums by DPP (bitwise the same in the row's 16 lanes, so the rotation
// decision is uniform over the pair).  A pair is rotated when |a_p^T a_q| >
// thr[0] ||a_p|| ||a_q|| and both squared norms exceed thr[1].  The rotations
// are accumulated in a 2 kJW x 2 kJW orthogonal J (column c of J beside
// column c of A, rows j and j + 16 in lane j), and the round ends with
// U(:, P u Q) = U(:, P u Q) J on the matrix cores.  flags[sweep] is set when
// any rotation was applied; a launch of sweep s > 0 returns at once when sweep
// s - 1 applied none (converged), so the host can queue several sweeps before
// it looks.
constexpr int kJW = 16;             // columns per block
constexpr int kJC = 2 * kJW;        // columns held by a workgroup
constexpr int kJT = 256;            // kJW pairs, one per 16-lane row
constexpr int kJR = kLMax / 16;     // rows of a column per lane

template <int CTRL>
__device__ __forceinline__ double ldpp(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 16 lanes of a DPP row, the same value (bitwise) in each.
__device__ __forceinline__ double lrow_total(double x) {
  x += ldpp<0xB1>(x);   // quad_perm [1,0,3,2]
  x += ldpp<0x4E>(x);   // quad_perm [2,3,0,1]
  x += ldpp<0x141>(x);  // row_half_mirror
  x += ldpp<0x140>(x);  // row_mirror
  return x;
}

__device__ __forceinline__ bool ljac_rotate(double *x, double *y, double *jx, double *jy, double tol2,
                                            double floor2) {
  // two partial sums per product: half the dependent chain
  double al0 = 0.0, be0 = 0.0, ga0 = 0.0, al1 = 0.0, be1 = 0.0, ga1 = 0.0;
#pragma unroll
  for (int m = 0; m < kJR; m += 2) {
    al0 += x[m] * x[m];
    be0 += y[m] * y[m];
    ga0 += x[m] * y[m];
    al1 += x[m + 1] * x[m + 1];
    be1 += y[m + 1] * y[m + 1];
    ga1 += x[m + 1] * y[m + 1];
  }
  double al = al0 + al1, be = be0 + be1, ga = ga0 + ga1;
  al = lrow_total(al);
  be = lrow_total(be);
  ga = lrow_total(ga);
  // |ga| > tol sqrt(al be), squared (the Gram passes bound the data's range
  // well inside the squares' range)
  if (!(al > floor2 && be > floor2 && ga * ga > tol2 * (al * be))) return false;
  // the smaller rotation angle: t = tan(theta) = sign(zeta) / (|zeta| +
  // sqrt(1 + zeta^2)), zeta = (be - al) / (2 ga), without forming zeta
  const double df = be - al, ga2 = 2.0 * ga;
  const double t = (df >= 0 ? ga2 : -ga2) / (fabs(df) + sqrt(df * df + ga2 * ga2));
  const double c = rsqrt(1.0 + t * t);
  const double sn = c * t;
#pragma unroll
  for (int m = 0; m < kJR; ++m) {
    const double u = x[m], v = y[m];
    x[m] = c * u - sn * v;
    y[m] = sn * u + c * v;
  }
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const double u = jx[m], v = jy[m];
    jx[m] = c * u - sn * v;
    jy[m] = sn * u + c * v;
  }
  return true;
}

typedef double ld4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kJT) void lk_jacobi_round(double *__restrict__ A, double *__restrict__ U, int b, int k,
                                                       int nbp, int round, const double *__restrict__ thr,
                                                       int *__restrict__ flags, int sweep) {
  // hA: the 2 kJW columns in the within-block steps, then the exchange buffers
  // of the cross steps ([2][kJW][kLMax]); hJ likewise for J, then J itself
  // (hJ[column][row])
  __shared__ double hA[kJC][kLMax];
  __shared__ double hJ[kJC][kJC];
  int P, Q;
  lrr_pair(round, blockIdx.x, nbp, &P, &Q);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int pr = 4 * wv + g;  // the pair of this 16-lane row
  const double tol2 = thr[0] * thr[0], floor2 = thr[1];
  auto gcol = [&](int l) { return l < kJW ? P * kJW + l : Q * kJW + (l - kJW); };
  if (sweep > 0 && flags[sweep - 1] == 0) return;
  // U(:, P u Q) is read now, in flight during the rotations (only this
  // workgroup touches these columns in this round): wave wv takes the
  // 16-row tiles wv, wv + 4, ... of U (k x k, ld k); bf[ti][ks] = U(row, held
  // column 4 ks + g)
  constexpr int kTU = kLMax / 16 / (kJT / 64);
  double bf[kTU][kJC / 4];
#pragma unroll
  for (int ti = 0; ti < kTU; ++ti) {
    const int row = 16 * (wv + 4 * ti) + j;
#pragma unroll
    for (int ks = 0; ks < kJC / 4; ++ks) {
      const int c = gcol(4 * ks + g);
      bf[ti][ks] = (c < k && row < k) ? U[row + (size_t)k * c] : 0.0;
    }
  }
  int rotated = 0;
  double ap[kJR], aq[kJR], jp[2], jq[2];
  if (round == 0) {
    for (int e = threadIdx.x; e < kJC * kLMax; e += kJT) {
      const int l = e / kLMax, r = e % kLMax, c = gcol(l);
      hA[l][r] = (c < k && r < b) ? A[r + (size_t)b * c] : 0.0;
    }
    for (int e = threadIdx.x; e < kJC * kJC; e += kJT) hJ[e / kJC][e % kJC] = (e / kJC == e % kJC) ? 1.0 : 0.0;
    __syncthreads();
    // pairs inside P (rows 0..kJW/2-1) and inside Q (the others)
    const int off = (pr < kJW / 2) ? 0 : kJW;
    for (int st = 0; st < kJW - 1; ++st) {
      int p, q;
      lrr_pair(st, pr % (kJW / 2), kJW, &p, &q);
      p += off;
      q += off;
#pragma unroll
      for (int m = 0; m < kJR; ++m) {
        ap[m] = hA[p][j + 16 * m];
        aq[m] = hA[q][j + 16 * m];
      }
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        jp[m] = hJ[p][j + 16 * m];
        jq[m] = hJ[q][j + 16 * m];
      }
      if (ljac_rotate(ap, aq, jp, jq, tol2, floor2)) {
        rotated = 1;
#pragma unroll
        for (int m = 0; m < kJR; ++m) {
          hA[p][j + 16 * m] = ap[m];
          hA[q][j + 16 * m] = aq[m];
        }
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          hJ[p][j + 16 * m] = jp[m];
          hJ[q][j + 16 * m] = jq[m];
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < kJR; ++m) {
      ap[m] = hA[pr][j + 16 * m];
      aq[m] = hA[kJW + pr][j + 16 * m];
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      jp[m] = hJ[pr][j + 16 * m];
      jq[m] = hJ[kJW + pr][j + 16 * m];
    }
    __syncthreads();  // hA and hJ become the exchange buffers
  } else {
    const int c0 = gcol(pr), c1 = gcol(kJW + pr);
#pragma unroll
    for (int m = 0; m < kJR; ++m) {
      const int r = j + 16 * m;
      ap[m] = (c0 < k && r < b) ? A[r + (size_t)b * c0] : 0.0;
      aq[m] = (c1 < k && r < b) ? A[r + (size_t)b * c1] : 0.0;
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      jp[m] = (j + 16 * m == pr) ? 1.0 : 0.0;
      jq[m] = (j + 16 * m == kJW + pr) ? 1.0 : 0.0;
    }
  }
  // cross steps, four phases of four: in phase ph, step sg, pair pr = 4 wv + g
  // holds P column pr and Q column 4 ((wv + ph) & 3) + ((g + sg) & 3).  Within
  // a phase the Q columns move one 16-lane row up inside the wave (lane
  // shuffles, no barrier); between phases each wave takes the next wave's Q
  // columns through LDS, one row further on, so each (P, Q) pair meets once.
  static_assert(kJW == 16 && kJT == 256, "four waves of four pairs");
  double(*xA)[kJW][kLMax] = reinterpret_cast<double(*)[kJW][kLMax]>(&hA[0][0]);
  double(*xJ)[kJW][kJC] = reinterpret_cast<double(*)[kJW][kJC]>(&hJ[0][0]);
  for (int ph = 0; ph < 4; ++ph) {
    for (int sg = 0; sg < 4; ++sg) {
      if (ljac_rotate(ap, aq, jp, jq, tol2, floor2)) rotated = 1;
      if (sg < 3) {
        const int src = (lane + 16) & 63;
#pragma unroll
        for (int m = 0; m < kJR; ++m) aq[m] = __shfl(aq[m], src, 64);
#pragma unroll
        for (int m = 0; m < 2; ++m) jq[m] = __shfl(jq[m], src, 64);
      } else if (ph < 3) {
        const int buf = ph & 1, from = 4 * ((wv + 1) & 3) + ((g + 1) & 3);
#pragma unroll
        for (int m = 0; m < kJR; ++m) xA[buf][pr][j + 16 * m] = aq[m];
#pragma unroll
        for (int m = 0; m < 2; ++m) xJ[buf][pr][j + 16 * m] = jq[m];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kJR; ++m) aq[m] = xA[buf][from][j + 16 * m];
#pragma unroll
        for (int m = 0; m < 2; ++m) jq[m] = xJ[buf][from][j + 16 * m];
      }
    }
  }
  const int qw = kJW + 4 * ((wv + 3) & 3) + ((g + 3) & 3);  // local index of the Q column held at the end
  {
    const int c0 = gcol(pr), c1 = gcol(qw);
#pragma unroll
    for (int m = 0; m < kJR; ++m) {
      const int r = j + 16 * m;
      if (r < b) {
        if (c0 < k) A[r + (size_t)b * c0] = ap[m];
        if (c1 < k) A[r + (size_t)b * c1] = aq[m];
      }
    }
  }
  __syncthreads();  // the last exchange has been read: hJ takes J
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    hJ[pr][j + 16 * m] = jp[m];
    hJ[qw][j + 16 * m] = jq[m];
  }
  if (rotated && j == 0) flags[sweep] = 1;
  if (!__syncthreads_or(rotated)) return;  // J = I: U unchanged
  // U(:, P u Q) = U(:, P u Q) J, computed as its transpose J^T U^T
#pragma unroll
  for (int ti = 0; ti < kTU; ++ti) {
    const int row = 16 * (wv + 4 * ti) + j;
    if (16 * (wv + 4 * ti) >= k) break;
#pragma unroll
    for (int ct = 0; ct < kJC / 16; ++ct) {
      ld4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < kJC / 4; ++ks)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(hJ[16 * ct + j][4 * ks + g], bf[ti][ks], acc, 0, 0, 0);
      // register r: U(row, held column 16 ct + 4 r + g)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = gcol(16 * ct + 4 * r + g);
        if (c < k && row < k) U[row + (size_t)k * c] = acc[r];
      }
    }
  }
}

// Truncation, part 3 (after the Jacobi sweeps): singular values (column norms
// of A = R^T U = V Sigma), their descending order, the rank L (smallest with
// Frobenius tail <= delta), the norm and threshold at the first link, and the
// gathered columns Up = U(:, perm[0:L]), Ap = A(:, perm[0:L]) for the two
// products GU = Glast Up and Pnext = Ap^T Fn^T.
__global__ __launch_bounds__(kLT) void lk_trunc_finish(LTruncArgs a) {
  const int k = a.k, b = a.b;
  const double *A = a.W0, *U = a.W1;
  __shared__ int LL;
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    double s = 0.0;
    for (int r = 0; r < b; ++r) s += A[r + (size_t)b * j] * A[r + (size_t)b * j];
    a.sv[j] = sqrt(s);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    int rank = 0;
    for (int i = 0; i < k; ++i)
      if (a.sv[i] > a.sv[j] || (a.sv[i] == a.sv[j] && i < j)) ++rank;
    a.perm[rank] = j;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (a.first) {
      double n2 = 0.0;
      for (int j = k - 1; j >= 0; --j) n2 += a.sv[a.perm[j]] * a.sv[a.perm[j]];
      const double nrm = sqrt(n2);
      *a.norm = nrm;
      *a.delta = (a.Nm1 > 0) ? a.tol * nrm / sqrt((double)a.Nm1) : 0.0;
    }
    const double delta = *a.delta;
    double tail = 0.0;
    int L = k;
    for (int j = k - 1; j >= 1; --j) {
      const double s = a.sv[a.perm[j]];
      tail += s * s;
      if (sqrt(tail) <= delta) L = j;
      else break;
    }
    LL = L;
    for (int j = 0; j < kLMax; ++j) a.sigma_out[j] = (j < k) ? a.sv[a.perm[j]] : 0.0;
    double t2 = 0.0;
    for (int j = k - 1; j >= L; --j) t2 += a.sv[a.perm[j]] * a.sv[a.perm[j]];
    *a.tail_out = t2;
    a.dec[3] = L;
  }
  __syncthreads();
  const int L = LL;
  for (int e = threadIdx.x; e < k * L; e += blockDim.x) {
    const int r = e % k, c = e / k;
    a.Up[e] = U[r + (size_t)k * a.perm[c]];
  }
  for (int e = threadIdx.x; e < b * L; e += blockDim.x) {
    const int r = e % b, c = e / b;
    a.Ap[e] = A[r + (size_t)b * a.perm[c]];
  }
}

// D (cols x rows, ld ldd) = S^T for S (rows x cols, ld lds).
__global__ void lk_transpose(const double *__restrict__ S, int rows, int cols, int lds, double *__restrict__ D,
                             int ldd) {
  const long long n = (long long)rows * cols;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(e / rows), r = (int)(e % rows);
    D[c + (long long)ldd * r] = S[r + (long long)lds * c];
  }
}

// --- host -------------------------------------------------------------------
constexpr size_t kSlotL = (size_t)kLMax * kLMax;
constexpr int kMaxSweeps = 60;
constexpr int kSweepGroup = 4;  // Jacobi sweeps queued between host checks

// A logical core: slice M'(i) = M(i) (trans = 0) or M(i)^T (trans = 1) of the
// physical pa x I x pb core at X.  LRL rounding and left orthonormalization
// run the RLR / right algorithm on the reversed train of transposed slices.
struct LView {
  const double *X;
  long long I;
  int pa, pb, trans;
  int ea() const { return trans ? pb : pa; }
  int eb() const { return trans ? pa : pb; }
};

}  // namespace

struct LargeCtx {
  double *mem = nullptr;
  size_t bytes = 0;
  double *keep = nullptr;  // the orthonormalization sweep's products kept for the truncation sweep
  size_t keep_bytes = 0;
};

void ttr_large_release(ttr_handle *h) {
  if (!h || !h->large) return;
  LargeCtx *c = h->large;
  if (c->mem) ttr_dev_free(h, c->mem);
  if (c->keep) ttr_dev_free(h, c->keep);
  delete c;
  h->large = nullptr;
}

namespace {

constexpr double kU32 = 5.9604644775390625e-08;  // 2^-24
constexpr double kTauMix = 1e-5;

struct Large {
  ttr_handle *h = nullptr;
  // workspace
  double *G, *Ra, *Rb, *Gst[3], *P[2], *GU, *W0, *W1, *Up, *Ap, *Id, *scal, *sigma, *tails, *sv, *Bp, *part;
  double *tC, *tA, *tB;
  int *perm, *flags;
  std::vector<double *> T;                 // N+1 slots
  std::vector<std::array<double *, 3>> B;  // N x 3 slots
  int passes = 0, applies = 0, sweeps = 0;
  // implicit Hadamard product: the cores n < N-1 of X are A_n (x) B_n,
  // never formed (right products through launch_lg_kron_right)
  const ttr_tt *KA = nullptr, *KB = nullptr;
  double *xlast = nullptr;  // the formed last core of A * B

  // Room for the products C_n = M_n T_{n+1}, n = 1..N-2, of the
  // orthonormalization sweep, so that the truncation sweep reads them instead
  // of forming them again (one GEMM per link fewer).  Held by the handle like
  // the workspace; when the allocation fails they are formed again.
  std::vector<double *> keepC;
  void setup_keep(int N, size_t mc) {
    keepC.assign(N, nullptr);
    if (N < 3) return;
    mc = (mc + 63) & ~(size_t)63;
    const size_t need = (size_t)(N - 2) * mc * sizeof(double);
    LargeCtx *ctx = h->large;
    if (ctx->keep_bytes < need) {
      if (ctx->keep) {
        if (hipStreamSynchronize(h->stream) != hipSuccess) return;
        ttr_dev_free(h, ctx->keep);
        ctx->keep = nullptr;
        ctx->keep_bytes = 0;
      }
      void *m = nullptr;
      if (ttr_dev_alloc(h, &m, need) != TTR_OK) {
        (void)hipGetLastError();  // an out-of-memory result is not an error here
        return;
      }
      ctx->keep = static_cast<double *>(m);
      ctx->keep_bytes = need;
    }
    for (int n = 1; n <= N - 2; ++n) keepC[n] = ctx->keep + (size_t)(n - 1) * mc;
  }
  double *keep_slot(int n) const { return (n < (int)keepC.size()) ? keepC[n] : nullptr; }

  int setup(int N, size_t mc, size_t extra = 0) {
    mc = (mc + 63) & ~(size_t)63;
    const size_t need = (15 + (size_t)(N + 1) + 3 * (size_t)N) * kSlotL + 64 + (size_t)(N + 1) * (kLMax + 1) +
                        3 * (size_t)kLMax + lg_packed_doubles(kLMax, kLMax) + (size_t)512 * kSlotL + 3 * mc + extra +
                        256;
    if (!h->large) h->large = new LargeCtx();
    LargeCtx *ctx = h->large;
    if (ctx->bytes < need * sizeof(double)) {
      if (ctx->mem) {
        TTR_HIPCHK(hipStreamSynchronize(h->stream));
        ttr_dev_free(h, ctx->mem);
        ctx->mem = nullptr;
        ctx->bytes = 0;
      }
      void *m = nullptr;
      int arc;
      if ((arc = ttr_dev_alloc(h, &m, need * sizeof(double)))) return arc;
      ctx->mem = static_cast<double *>(m);
      ctx->bytes = need * sizeof(double);
    }
    double *p = ctx->mem;
    auto take = [&](size_t n) {
      double *q = p;
      p += (n + 31) & ~(size_t)31;
      return q;
    };
    G = take(kSlotL);
    Ra = take(kSlotL);
    Rb = take(kSlotL);
    for (int j = 0; j < 3; ++j) Gst[j] = take(kSlotL);
    for (int j = 0; j < 2; ++j) P[j] = take(kSlotL);
    GU = take(kSlotL);
    W0 = take(kSlotL);
    W1 = take(kSlotL);
    Up = take(kSlotL);
    Ap = take(kSlotL);
    Id = take(kSlotL);
    scal = take(64);
    sigma = take((size_t)(N + 1) * kLMax);
    tails = take((size_t)(N + 1));
    sv = take(kLMax);
    perm = reinterpret_cast<int *>(take(kLMax));
    flags = reinterpret_cast<int *>(take(kLMax));
    Bp = take(lg_packed_doubles(kLMax, kLMax));
    T.resize(N + 1);
    B.resize(N);
    for (int n = 0; n <= N; ++n) T[n] = take(kSlotL);
    for (int n = 0; n < N; ++n)
      for (int j = 0; j < 3; ++j) B[n][j] = take(kSlotL);
    part = take((size_t)512 * kSlotL);
    tC = take(mc);
    tA = take(mc);
    tB = take(mc);
    xlast = extra ? take(extra) : nullptr;
    for (int i = 0; i < 16; ++i) h->dec_host[i] = 0;
    TTR_HIPCHK(hipMemcpyAsync(h->dec_dev, h->dec_host, 16 * sizeof(int), hipMemcpyHostToDevice, h->stream));
    return TTR_OK;
  }

  // C (m x n, ld ldc) = op(A) op(B), op(A) m x k, A and B column-major
  void sgemm(bool ta, bool tb, int m, int n, int k, const double *A, long long lda, const double *Bm, long long ldb,
             double *C, long long ldc) {
    launch_lg_sgemm(h->stream, A, ta ? lda : 1, ta ? 1 : lda, Bm, tb ? ldb : 1, tb ? 1 : ldb, m, n, k, C, ldc);
  }
  // Z'(i) = M'(i) B (B(k, c) = B[k bsr + c bsc], eb x n) into `out`, in the
  // view's orientation; tri: B lower triangular.
  // perm (nullable, column-major views only): the product V(M)(:, perm) B(perm, :)
  // over the first n entries of perm (a pivoted factor F = P U: the gathered
  // columns times its upper-triangular rows).
  LView right(const LView &v, const double *Bm, long long bsr, long long bsc, int n, int tri, double *out,
              const int *perm = nullptr) {
    if (perm && !v.trans) {
      launch_lg_gemm(h->stream, v.X, (long long)v.pa * v.I, n, (long long)v.pa * v.I, 1, Bm, bsr, bsc, n, tri, Bp,
                     out, (long long)v.pa * v.I, 1, perm);
      return LView{out, v.I, v.pa, n, 0};
    }
    if (!v.trans) {
      // V(Z) = V(M) B
      launch_lg_gemm(h->stream, v.X, (long long)v.pa * v.I, v.pb, (long long)v.pa * v.I, 1, Bm, bsr, bsc, n, tri, Bp,
                     out, (long long)v.pa * v.I, 1);
      return LView{out, v.I, v.pa, n, 0};
    }
    // Z(i) = B^T M(i): H(Z)^T = H(M)^T B
    launch_lg_gemm(h->stream, v.X, v.I * v.pb, v.pa, v.pa, 0, Bm, bsr, bsc, n, tri, Bp, out, n, 0);
    return LView{out, v.I, n, v.pb, 1};
  }
  // Z'(i) = M'(i) T for core n of the tensor being rounded: for an implicit
  // Hadamard product (cores n < N-1) C(i) = (A_n(i) (x) B_n(i)) T formed
  // straight from the factors, otherwise right().
  LView right_core(int n, int N, const LView &v, const double *Tm, long long ldt, int k, int tri, double *out) {
    if (KA && n < N - 1 && !v.trans) {
      launch_lg_kron_right(h->stream, KA->core[n], (int)KA->R[n], (int)KA->R[n + 1], KB->core[n], (int)KB->R[n],
                           (int)KB->R[n + 1], v.I, Tm, ldt, k, out);
      return LView{out, v.I, v.pa, k, 0};
    }
    return right(v, Tm, 1, ldt, k, tri, out);
  }
  // Z'(i) = A M'(i) (A(r, c) = A[r asr + c asc], m x ea) into `out`.
  // tri = 2: A^T is upper triangular (a Cholesky-route stage factor F, A = F^T).
  LView left(const LView &v, const double *Am, long long asr, long long asc, int m, double *out, int tri = 0) {
    if (!v.trans) {
      // H(Z)^T = H(M)^T A^T
      launch_lg_gemm(h->stream, v.X, v.I * v.pb, v.pa, v.pa, 0, Am, asc, asr, m, tri, Bp, out, m, 0);
      return LView{out, v.I, m, v.pb, 0};
    }
    // Z(i) = M(i) A^T: V(Z) = V(M) A^T
    launch_lg_gemm(h->stream, v.X, (long long)v.pa * v.I, v.pb, (long long)v.pa * v.I, 1, Am, asc, asr, m, tri, Bp, out,
                   (long long)v.pa * v.I, 1);
    return LView{out, v.I, v.pa, m, 1};
  }
  // G (ea x ea) = sum_i M'(i) M'(i)^T (left) or (eb x eb) = sum_i M'(i)^T M'(i)
  // (right); *gerr = bound on the rounding error relative to the trace
  int gram(const LView &v, bool left_side, int f32, double *Gout, double *gerr) {
    // physical: H(M) H(M)^T (row-major H(M)^T) or V(M)^T V(M) (column-major V(M))
    const bool use_h = (left_side != (v.trans != 0));
    long long M;
    int K, nwg;
    double *fs = scal + 32;
    if (f32) launch_lg_scale_probe(h->stream, v.X, (long long)v.pa * v.I * v.pb, fs);
    if (use_h) {
      M = v.I * v.pb;
      K = v.pa;
      nwg = launch_lg_gram(h->stream, v.X, nullptr, M, K, K, v.pa, v.pa, 0, f32, part, fs);
    } else {
      M = (long long)v.pa * v.I;
      K = v.pb;
      nwg = launch_lg_gram(h->stream, v.X, nullptr, M, K, K, M, M, 1, f32, part, fs);
    }
    if (nwg > 512) return ttr_fail(TTR_ERR_HIP, "Gram partials exceed the workspace");
    launch_reduce(h->stream, part, nwg, K * K, Gout);
    const LGramGrid g = lg_gram_grid(M, f32);
    // per entry: the workgroup's sequential sum over its rows, then the
    // fixed-order sum of the partials (FP32: inputs rounded too)
    *gerr = 2.0 * ((double)g.rpw + (double)nwg + 18.0) * (f32 ? kU32 : kU);
    ++passes;
    return TTR_OK;
  }
  int sync_dec() {
    TTR_HIPCHK(hipMemcpyAsync(h->dec_host, h->dec_dev, 16 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    TTR_HIPCHK(hipStreamSynchronize(h->stream));
    TTR_HIPCHK(hipGetLastError());
    if (h->dec_host[2] != 0)
      return ttr_fail(TTR_ERR_NUMERICAL, "non-finite data or a small factorization did not converge");
    return TTR_OK;
  }
  // One-sided Jacobi SVD of A = W0 (b x k) with U = W1: sweeps of block
  // rounds until a sweep applies no rotation, checked on the device (a sweep
  // after the converged one returns at once); the host looks every few sweeps.
  int jacobi(long long b, int k) {
    const int nbp = std::max(2, 2 * ((k + 2 * kJW - 1) / (2 * kJW)));
    TTR_HIPCHK(hipMemsetAsync(flags, 0, kMaxSweeps * sizeof(int), h->stream));
    int hf[kMaxSweeps];
    for (int sweep = 0; sweep < kMaxSweeps;) {
      const int end = std::min(kMaxSweeps, sweep + kSweepGroup);
      for (; sweep < end; ++sweep)
        for (int r = 0; r < nbp - 1; ++r)
          hipLaunchKernelGGL(lk_jacobi_round, dim3(nbp / 2), dim3(kJT), 0, h->stream, W0, W1, (int)b, k, nbp, r,
                             scal + 8, flags, sweep);
      TTR_HIPCHK(hipGetLastError());
      h->stats.small_launches += (nbp - 1) * kSweepGroup;
      TTR_HIPCHK(hipMemcpyAsync(hf, flags, sweep * sizeof(int), hipMemcpyDeviceToHost, h->stream));
      TTR_HIPCHK(hipStreamSynchronize(h->stream));
      for (int s = 0; s < sweep; ++s)
        if (!hf[s]) {
          sweeps = s + 1;
          return TTR_OK;
        }
    }
    return ttr_fail(TTR_ERR_NUMERICAL, "the truncation SVD did not converge");
  }
  // One QR-by-Gram step on the Gram in G (d x d).  *pivoted is set when the
  // step took the pivoted route (its factor is not triangular).
  int mixed = 0;  // TTR_MIXED: FP32 first passes
  int step(const double *Rc, int d, int b, int pass, double *F, double *Rn, double *Tdst, double gerr, int check,
           int first, double tol2_nm1, int f32, int *pivoted, int *permuted = nullptr) {
    LStepArgs a;
    a.G = G;
    a.d = d;
    a.pass = pass;
    a.b = b;
    a.Rc = Rc;
    a.Fstep = F;
    a.Rnext = Rn;
    a.Tdst = Tdst;
    a.dec = h->dec_dev;
    const double u = f32 ? kU32 : kU;
    a.tau1 = f32 ? u / kTauMix : kTau1;
    a.tau2 = kTau2;
    a.ugram = u;
    a.gerr = gerr;
    a.shift_pass = mixed ? 2 : 1;
    a.notrunc_check = check;
    a.delta_dev = scal + 1;
    a.first = first;
    a.tol2_nm1 = tol2_nm1;
    a.W0 = W0;
    a.W1 = W1;
    a.perm = perm;
    a.Rp = Ap;
    hipLaunchKernelGGL(lk_step, dim3(1), dim3(kLT), 0, h->stream, a);
    h->stats.small_launches++;
    int rc;
    if ((rc = sync_dec())) return rc;
    const int how = h->dec_host[8], kk = h->dec_host[0];
    if (pivoted && (how == 2 || kk < d)) *pivoted = 1;
    if (permuted) *permuted = (how == 2);  // F = P U with P in `perm`, U upper triangular
    if (how == 0) return TTR_OK;
    // R = L^T Rc (d x b) or R' = L(:, 0:k)^T Rp (k x b), L lower in W0 (ld d)
    sgemm(true, false, kk, b, d, W0, d, how == 1 ? Rc : Ap, d, Rn, kk);
    if (Tdst && h->dec_host[1]) {
      hipLaunchKernelGGL(lk_transpose, dim3(64), dim3(256), 0, h->stream, Rn, kk, b, kk, Tdst, b);
      TTR_HIPCHK(hipGetLastError());
    }
    return TTR_OK;
  }
};

// Per-core factorization record of the orthonormalization sweep.
struct LFac {
  int nst = 1;
  int dim[4] = {0, 0, 0, 0};
  int tri = 0;                // T_n = R^T is lower triangular (no pivoted pass)
  int stri[4] = {0, 0, 0, 0};  // lg_gemm tri flag of stage j's F (2: upper triangular)
};

// Orthonormalization sweep over logical cores N-1..1 (§2.3 Alg. 1 order)
// with implicit factors (§3.5 Alg. 6): core n's QR-by-Gram of H(C_n)^T,
// C_n(i) = M_n(i) T_{n+1}; the stages F_j (slots B[n][j]) and T_n = R^T
// (slot T[n]) are kept.  `rev`: the mirror image (reversed train of
// transposed slices).  When `out` is given, each orthonormal core
// F_nst^T .. F_1^T C_n is written to out->core (in the view's orientation,
// §3.4 Alg. 5).
int orth_sweep_large(Large &L, const ttr_tt *X, int rev, int prec, std::vector<int> &k, std::vector<LFac> &fac,
                     ttr_tt *out, std::vector<LView> *kept = nullptr) {
  ttr_handle *h = L.h;
  const int N = X->N;
  auto phys = [&](int n) { return rev ? N - 1 - n : n; };
  auto view = [&](int n) {
    const int p = phys(n);
    return LView{X->core[p], X->I[p], (int)X->R[p], (int)X->R[p + 1], rev};
  };
  k.assign(N + 1, 1);
  fac.assign(N + 1, LFac());
  for (int n = 0; n <= N; ++n) k[n] = (int)(rev ? X->R[N - n] : X->R[n]);
  int rc;
  for (int n = N - 1; n >= 1; --n) {
    const LView v = view(n);
    const int a = v.ea(), b = v.eb();
    LView cur = v;
    if (n < N - 1) {
      double *dst = (kept && L.keep_slot(n)) ? L.keep_slot(n) : L.tC;
      cur = L.right_core(n, N, v, L.T[n + 1], b, k[n + 1], fac[n + 1].tri, dst);
      if (kept && dst != L.tC) (*kept)[n] = cur;
    }
    double *bufs[2] = {L.tA, L.tB};
    double *R[2] = {L.Ra, L.Rb};
    fac[n].dim[0] = a;
    int pass = 1, pivoted = 0;
    for (;; ++pass) {
      double gerr;
      const int f32 = (prec == TTR_MIXED && pass == 1);
      if ((rc = L.gram(cur, true, f32, L.G, &gerr))) return rc;
      int pv = 0;
      if ((rc = L.step(pass == 1 ? nullptr : R[pass & 1], cur.ea(), a, pass, L.B[n][pass - 1], R[(pass - 1) & 1],
                       L.T[n], gerr, 0, 0, 0.0, f32, &pv)))
        return rc;
      pivoted |= pv;
      fac[n].stri[pass - 1] = pv ? 0 : 2;
      const int kk = h->dec_host[0];
      fac[n].dim[pass] = kk;
      if (h->dec_host[1]) break;
      if (pass >= 3) return ttr_fail(TTR_ERR_NUMERICAL, "QR-by-Gram did not settle in three passes");
      // D = F_pass^T C (materialized; the next pass measures its Gram)
      cur = L.left(cur, L.B[n][pass - 1], cur.ea(), 1, kk, bufs[(pass - 1) & 1], fac[n].stri[pass - 1]);
    }
    fac[n].nst = pass;
    fac[n].tri = !pivoted;
    k[n] = fac[n].dim[pass];
    if (out) {
      // the orthonormal core: the last stage applied to what its Gram measured
      const int p = phys(n);
      L.left(cur, L.B[n][pass - 1], cur.ea(), 1, k[n], L.tB == cur.X ? L.tA : L.tB, fac[n].stri[pass - 1]);
      const double *src = (L.tB == cur.X) ? L.tA : L.tB;
      launch_copy(h->stream, src, (long long)k[n] * v.I * k[n + 1], out->core[p]);
      ++L.applies;
    }
  }
  return TTR_OK;
}

void fill_stats(ttr_handle *h, int N, int rev, const std::vector<double> &sig, const std::vector<double> &tails,
                const std::vector<int> &sweeps) {
  for (int l = 0; l < N - 1; ++l) {
    const int pl = rev ? (N - 1 - l) - 1 : l;
    if (pl >= TTR_STATS_LINKS) continue;
    int cnt = 0;
    for (int j = 0; j < kLMax; ++j) {
      h->stats.sigma[(size_t)pl * TTR_STATS_SIGMA + j] = sig[(size_t)l * kLMax + j];
      if (sig[(size_t)l * kLMax + j] > 0) cnt = j + 1;
    }
    h->stats.nsigma[pl] = cnt;
    h->stats.tail2[pl] = tails[l];
    h->stats.sweeps[pl] = sweeps[l];
  }
}

size_t max_core_of(const ttr_tt *X) {
  size_t mc = 0;
  for (int n = 0; n < X->N; ++n) mc = std::max(mc, (size_t)(X->R[n] * X->I[n] * X->R[n + 1]));
  return mc;
}

}  // namespace

// Rounding of X (ranks up to 256) into Y (§2.4 Alg. 2; implicit factors of
// §3.5 Alg. 6, or with explicit_factors the orthonormal cores written first,
// §3.4 Alg. 5, and the truncation sweep run over them); RLR or its mirror
// LRL; prec TTR_MIXED runs the first Gram pass of every factorization in FP32.
namespace {
int round_large_with(Large &L, ttr_handle *h, const ttr_tt *X, double tol, int direction, int prec,
                     int explicit_factors, ttr_tt *Y, double *norm_out);
}  // namespace

int ttr_round_large(ttr_handle *h, const ttr_tt *X, double tol, int direction, int prec, int explicit_factors,
                    ttr_tt *Y, double *norm_out) {
  Large L;
  L.h = h;
  L.mixed = (prec == TTR_MIXED);
  int rc;
  if ((rc = L.setup(X->N, max_core_of(X)))) return rc;
  return round_large_with(L, h, X, tol, direction, prec, explicit_factors, Y, norm_out);
}

namespace {
int round_large_with(Large &L, ttr_handle *h, const ttr_tt *X, double tol, int direction, int prec,
                     int explicit_factors, ttr_tt *Y, double *norm_out) {
  const int N = X->N;
  const int rev = (direction == TTR_LRL);
  int rc;
  auto phys = [&](int n) { return rev ? N - 1 - n : n; };
  auto view = [&](int n) {
    const int p = phys(n);
    return LView{X->core[p], X->I[p], (int)X->R[p], (int)X->R[p + 1], rev};
  };
  std::vector<int> k;
  std::vector<LFac> fac;
  std::vector<LView> kept;  // C_n of sweep 1 kept for sweep 2 (X == nullptr: form it again)
  const bool ex = explicit_factors != 0;
  if (ex) {
    // ---- sweep 1, explicit: Y <- X, orthonormal cores written into Y ----
    for (int n = 0; n < N; ++n) {
      launch_copy(h->stream, X->core[n], (long long)X->R[n] * X->I[n] * X->R[n + 1], Y->core[n]);
      Y->R[n] = X->R[n];
    }
    Y->R[N] = 1;
    if ((rc = orth_sweep_large(L, Y, rev, prec, k, fac, Y))) return rc;
    const int p0 = phys(0);
    const LView v0{Y->core[p0], Y->I[p0], (int)Y->R[p0], (int)Y->R[p0 + 1], rev};
    L.right(v0, L.T[1], 1, v0.eb(), k[1], fac[1].tri, L.tC);
    launch_copy(h->stream, L.tC, (long long)Y->I[p0] * k[1], Y->core[p0]);
    for (int l = 0; l <= N; ++l) Y->R[rev ? N - l : l] = k[l];
  } else {
    // ---- sweep 1: orthonormalization with implicit factors ----
    if (!L.KA) L.setup_keep(N, max_core_of(X));
    kept.assign(N, LView{nullptr, 0, 0, 0, 0});
    if ((rc = orth_sweep_large(L, X, rev, prec, k, fac, nullptr, &kept))) return rc;
  }
  auto yview = [&](int n) {
    const int p = phys(n);
    return LView{Y->core[p], Y->I[p], (int)Y->R[p], (int)Y->R[p + 1], rev};
  };
  // explicit: the next core's orthonormal factor is written into it, Fn = I
  double *Id = L.Id;  // cc x cc identity, built per link
  auto identity = [&](int m) -> int {
    std::vector<double> id((size_t)m * m, 0.0);
    for (int j = 0; j < m; ++j) id[(size_t)j * m + j] = 1.0;
    TTR_HIPCHK(hipStreamSynchronize(h->stream));
    TTR_HIPCHK(hipMemcpy(Id, id.data(), id.size() * sizeof(double), hipMemcpyHostToDevice));
    return TTR_OK;
  };
  // ---- sweep 2: truncation ----
  std::vector<int> Lr(N + 1, 1), sweeps(N, 0);
  const double *Pcur = nullptr;
  int Lprev = 1;
  for (int n = 0; n < N - 1; ++n) {
    const LView v = view(n);
    LView cur;
    int cc;
    if (ex) {
      // C'_n = P Y_n with the written orthonormal core Y_n
      cur = yview(n);
      cc = cur.eb();
      if (n >= 1) cur = L.left(cur, Pcur, 1, Lprev, Lprev, L.tA);
      if ((rc = identity(cc))) return rc;
    } else {
      // C_n = M_n T_{n+1}, then the left stages F_1^T .. F_{nst-1}^T and P
      // (the same calls as sweep 1, so each stage meets bitwise the data its
      // Gram was measured on)
      if (n < (int)kept.size() && kept[n].X) cur = kept[n];
      else cur = L.right_core(n, N, v, L.T[n + 1], v.eb(), k[n + 1], fac[n + 1].tri, L.tC);
      cc = k[n + 1];
      double *bufs[2] = {L.tA, L.tB};
      if (n >= 1) {
        for (int j = 1; j < fac[n].nst; ++j)
          cur = L.left(cur, L.B[n][j - 1], cur.ea(), 1, fac[n].dim[j], bufs[(j - 1) & 1], fac[n].stri[j - 1]);
        double *o = (cur.X == L.tC) ? L.tA : ((cur.X == L.tA) ? L.tB : L.tA);
        cur = L.left(cur, Pcur, 1, Lprev, Lprev, o);
      }
    }
    const int crow = cur.ea();
    // QR-by-Gram of V(C'_n)
    double *R[2] = {L.Ra, L.Rb};
    int g = 1, gd[4], notrunc = 0;
    gd[0] = cc;
    LView E = cur;
    for (;; ++g) {
      double gerr;
      const int f32 = (prec == TTR_MIXED && g == 1);
      if ((rc = L.gram(E, false, f32, L.G, &gerr))) return rc;
      int pv = 0, pm = 0;
      if ((rc = L.step(g == 1 ? nullptr : R[g & 1], gd[g - 1], cc, g, L.Gst[g - 1], R[(g - 1) & 1], nullptr, gerr, 1,
                       n == 0, tol * tol / (double)(N - 1), f32, &pv, &pm)))
        return rc;
      gd[g] = h->dec_host[0];
      if (g == 1) notrunc = h->dec_host[5];
      if (h->dec_host[1]) break;
      if (g >= 3) return ttr_fail(TTR_ERR_NUMERICAL, "QR-by-Gram did not settle in three passes");
      double *o = (E.X == L.tA) ? L.tB : L.tA;
      if (E.X == L.tC) o = L.tA;
      // a Cholesky-route factor is upper triangular; a pivoted one is P U:
      // gathered columns of E times U (the step's permutation is still in perm)
      if (pm && !E.trans) E = L.right(E, L.Gst[g - 1], 1, gd[g - 1], gd[g], 2, o, L.perm);
      else E = L.right(E, L.Gst[g - 1], 1, gd[g - 1], gd[g], pv ? 0 : 2, o);
    }
    // truncation: SVD of R (k x cc) unless no singular value can fall below delta
    const int kq = gd[g], dq = gd[g - 1];
    const double *Rq = R[(g - 1) & 1];
    const double *Fn = ex ? Id : L.B[n + 1][fac[n + 1].nst - 1];
    const int dn = ex ? cc : fac[n + 1].dim[fac[n + 1].nst - 1];
    double *Pn = L.P[n & 1];
    LTruncArgs ta;
    ta.R = Rq;
    ta.k = kq;
    ta.b = cc;
    ta.delta = L.scal + 1;
    ta.norm = L.scal + 2;
    ta.first = (n == 0);
    ta.tol = tol;
    ta.Nm1 = N - 1;
    ta.sigma_out = L.sigma + (size_t)n * kLMax;
    ta.tail_out = L.tails + n;
    ta.dec = h->dec_dev;
    ta.identity = (g == 1) ? notrunc : 0;
    ta.W0 = L.W0;
    ta.W1 = L.W1;
    ta.thr = L.scal + 8;
    ta.sv = L.sv;
    ta.perm = L.perm;
    ta.Up = L.Up;
    ta.Ap = L.Ap;
    hipLaunchKernelGGL(lk_trunc_setup, dim3(1), dim3(kLT), 0, h->stream, ta);
    h->stats.small_launches++;
    if ((rc = L.sync_dec())) return rc;
    int Ln;
    const double *GU;
    if (h->dec_host[7]) {
      // L = k: U = I, Pnext = R Fn^T
      Ln = kq;
      GU = L.Gst[g - 1];
      L.sgemm(false, true, kq, dn, cc, Rq, kq, Fn, dn, Pn, kq);
    } else {
      if ((rc = L.jacobi(cc, kq))) return rc;
      sweeps[n] = L.sweeps;
      hipLaunchKernelGGL(lk_trunc_finish, dim3(1), dim3(kLT), 0, h->stream, ta);
      h->stats.small_launches++;
      if ((rc = L.sync_dec())) return rc;
      Ln = h->dec_host[3];
      // GU = Glast U(:, perm[0:L]) (dq x L); Pnext = Sigma_L V_L^T Fn^T = A(:, perm[0:L])^T Fn^T
      L.sgemm(false, false, dq, Ln, kq, L.Gst[g - 1], dq, L.Up, kq, L.GU, dq);
      if (ex) L.sgemm(true, false, Ln, cc, cc, L.Ap, cc, Id, cc, Pn, Ln);  // Fn = I
      else L.sgemm(true, true, Ln, dn, cc, L.Ap, cc, Fn, dn, Pn, Ln);
      GU = L.GU;
    }
    Lr[n + 1] = Ln;
    // output core n: Y_n(i) = E(i) GU (explicit: through tC, Y_n is read)
    if (ex) {
      L.right(E, GU, 1, dq, Ln, 0, L.tC);
      launch_copy(h->stream, L.tC, (long long)E.ea() * E.I * Ln, Y->core[phys(n)]);
    } else {
      L.right(E, GU, 1, dq, Ln, 0, Y->core[phys(n)]);
    }
    ++L.applies;
    (void)crow;
    Pcur = L.P[n & 1];
    Lprev = Ln;
  }
  if (ex) {
    // last core: P Y_N
    const LView cur = yview(N - 1);
    L.left(cur, Pcur, 1, Lprev, Lprev, L.tC);
    launch_copy(h->stream, L.tC, (long long)Lprev * cur.I * cur.eb(), Y->core[phys(N - 1)]);
    ++L.applies;
  } else {
    // last core: P F_{nst-1}^T .. F_1^T M_N
    const int n = N - 1;
    LView cur = view(n);
    double *bufs[2] = {L.tA, L.tB};
    for (int j = 1; j < fac[n].nst; ++j)
      cur = L.left(cur, L.B[n][j - 1], cur.ea(), 1, fac[n].dim[j], bufs[(j - 1) & 1], fac[n].stri[j - 1]);
    L.left(cur, Pcur, 1, Lprev, Lprev, Y->core[phys(n)]);
    ++L.applies;
  }
  TTR_HIPCHK(hipGetLastError());
  TTR_HIPCHK(hipMemcpyAsync(h->scal_host, L.scal, 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  const int nsig = (N - 1) * kLMax;
  std::vector<double> sig(nsig), tails(N - 1);
  TTR_HIPCHK(hipMemcpyAsync(sig.data(), L.sigma, nsig * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  TTR_HIPCHK(hipMemcpyAsync(tails.data(), L.tails, (N - 1) * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  TTR_HIPCHK(hipStreamSynchronize(h->stream));
  for (int l = 0; l <= N; ++l) {
    const int pl = rev ? N - l : l;
    Y->R[pl] = (l == 0 || l == N) ? 1 : Lr[l];
  }
  h->stats.gram_passes = L.passes;
  h->stats.apply_passes = L.applies;
  h->stats.links = N - 1;
  h->stats.norm = h->scal_host[2];
  h->stats.delta = h->scal_host[1];
  fill_stats(h, N, rev, sig, tails, sweeps);
  if (norm_out) *norm_out = h->scal_host[2];
  return TTR_OK;
}

}  // namespace

// In-place orthonormalization at ranks above 64 (§2.3 Alg. 1; written cores
// as in §3.4 Alg. 5).  side TTR_LEFT runs the mirror image.
int ttr_orthogonalize_large(ttr_handle *h, ttr_tt *X, int side) {
  const int N = X->N;
  const int rev = (side == TTR_LEFT);
  Large L;
  L.h = h;
  int rc;
  if ((rc = L.setup(N, max_core_of(X)))) return rc;
  std::vector<int> k;
  std::vector<LFac> fac;
  if ((rc = orth_sweep_large(L, X, rev, TTR_FP64, k, fac, X))) return rc;
  // the first logical core absorbs T_2: C_1(i) = M_1(i) T_2
  const int p0 = rev ? N - 1 : 0;
  const LView v{X->core[p0], X->I[p0], (int)X->R[p0], (int)X->R[p0 + 1], rev};
  L.right(v, L.T[1], 1, v.eb(), k[1], fac[1].tri, L.tC);
  launch_copy(h->stream, L.tC, (long long)X->I[p0] * k[1], X->core[p0]);
  TTR_HIPCHK(hipStreamSynchronize(h->stream));
  TTR_HIPCHK(hipGetLastError());
  for (int l = 0; l <= N; ++l) {
    const int pl = rev ? N - l : l;
    X->R[pl] = k[l];
  }
  return TTR_OK;
}

// ||X|| by the orthonormalization sweep (implicit factors) and ||X_1 T_2||_F
// (end of §2.3; the second method of §3.2.4), ranks above 64.
int ttr_norm_ortho_large(ttr_handle *h, const ttr_tt *X, double *out) {
  const int N = X->N;
  Large L;
  L.h = h;
  int rc;
  if ((rc = L.setup(N, max_core_of(X)))) return rc;
  std::vector<int> k;
  std::vector<LFac> fac;
  if ((rc = orth_sweep_large(L, X, 0, TTR_FP64, k, fac, nullptr))) return rc;
  const LView v{X->core[0], X->I[0], 1, (int)X->R[1], 0};
  LView c0 = v;
  if (N > 1) c0 = L.right(v, L.T[1], 1, v.eb(), k[1], fac[1].tri, L.tC);
  double gerr;
  if ((rc = L.gram(c0, true, 0, L.G, &gerr))) return rc;  // 1 x 1: ||C_1||_F^2
  launch_sqrt_scalar(h->stream, L.G, L.scal);
  TTR_HIPCHK(hipGetLastError());
  TTR_HIPCHK(hipMemcpyAsync(h->scal_host, L.scal, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  TTR_HIPCHK(hipStreamSynchronize(h->stream));
  *out = h->scal_host[0];
  return TTR_OK;
}

// <X, Y> by the recursion W_n = sum_i Y_n(i)^T W_{n-1} X_n(i) (§3.2.3, eq. (4))
// at ranks above 64: Z_n(i) = W_{n-1} X_n(i) is formed as a core, then
// W_n = V(Y_n)^T V(Z_n).
int ttr_dot_large(ttr_handle *h, const ttr_tt *X, const ttr_tt *Y, double *out) {
  const int N = X->N;
  size_t mz = 0;
  for (int n = 0; n < N; ++n) mz = std::max(mz, (size_t)(Y->R[n] * X->I[n] * X->R[n + 1]));
  Large L;
  L.h = h;
  int rc;
  if ((rc = L.setup(N, std::max(mz, max_core_of(X))))) return rc;
  double *Wb[2] = {L.P[0], L.P[1]};
  h->scal_host[0] = 1.0;
  TTR_HIPCHK(hipMemcpyAsync(Wb[0], h->scal_host, sizeof(double), hipMemcpyHostToDevice, h->stream));
  for (int n = 0; n < N; ++n) {
    const int rx0 = (int)X->R[n], rx1 = (int)X->R[n + 1], ry0 = (int)Y->R[n], ry1 = (int)Y->R[n + 1];
    const LView vx{X->core[n], X->I[n], rx0, rx1, 0};
    // Z_n(i) = W (ry0 x rx0, ld ry0) X_n(i)
    const LView z = L.left(vx, Wb[n & 1], 1, ry0, ry0, L.tA);
    // W_n (ry1 x rx1) = V(Y_n)^T V(Z_n)
    const long long M = (long long)ry0 * X->I[n];
    const int nwg = launch_lg_gram(h->stream, Y->core[n], z.X, M, ry1, rx1, M, M, 1, 0, L.part);
    launch_reduce(h->stream, L.part, nwg, ry1 * rx1, Wb[(n + 1) & 1]);
  }
  TTR_HIPCHK(hipGetLastError());
  TTR_HIPCHK(hipMemcpyAsync(h->scal_host + 1, Wb[N & 1], sizeof(double), hipMemcpyDeviceToHost, h->stream));
  TTR_HIPCHK(hipStreamSynchronize(h->stream));
  *out = h->scal_host[1];
  return TTR_OK;
}

// Rounding of the Hadamard product A * B without forming it (the closing
// remark of §3.2.2: keep the product implicit for rounding): RLR rounding of
// X = A * B (§2.4 Alg. 2) where every product of an original core with a
// small matrix, C_n(i) = (A_n(i) (x) B_n(i)) T_{n+1}, runs on the factors'
// slices (launch_lg_kron_right); only the last core A_N (x) B_N is formed.
// Factor ranks <= 16, ranks of A * B <= 256; RLR only.
int ttr_round_hadamard_large(ttr_handle *h, const ttr_tt *A, const ttr_tt *B, double tol, int prec, ttr_tt *Y,
                             double *norm_out) {
  const int N = A->N;
  std::vector<int64_t> R(N + 1), I(N);
  for (int n = 0; n <= N; ++n) R[n] = A->R[n] * B->R[n];
  for (int n = 0; n < N; ++n) I[n] = A->I[n];
  size_t mc = 0;
  for (int n = 0; n < N; ++n) mc = std::max(mc, (size_t)(R[n] * I[n] * R[n + 1]));
  const size_t last = (size_t)R[N - 1] * I[N - 1];
  Large L;
  L.h = h;
  L.mixed = (prec == TTR_MIXED);
  L.KA = A;
  L.KB = B;
  int rc;
  if ((rc = L.setup(N, mc, (last + 63) & ~(size_t)63))) return rc;
  // a shape-only description of X = A * B; only its last core is formed
  std::vector<double *> cores(N, nullptr);
  launch_hadamard(h->stream, A->core[N - 1], (int)A->R[N - 1], 1, B->core[N - 1], (int)B->R[N - 1], 1, I[N - 1],
                  L.xlast);
  cores[N - 1] = L.xlast;
  ttr_tt X;
  X.N = N;
  X.I = I.data();
  X.R = R.data();
  X.core = cores.data();
  X.cap = nullptr;
  return round_large_with(L, h, &X, tol, TTR_RLR, prec, 0, Y, norm_out);
}
