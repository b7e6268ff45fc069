// Streaming kernels of the rank 65..256 path (the unfoldings of §2.2 with
// ranks too large for a whole slice in registers), on the matrix cores:
//
//   lg_gemm   Z = X B     X a huge unfolding (M rows, K <= 256 columns), B a
//                         small K x N matrix (N <= 256); the products of the
//                         orthonormalization and truncation sweeps (§2.3 Alg. 1,
//                         §2.4 Alg. 2): V(M) T, F^T H(C), P H(M), V(E) G, ...
//   lg_gram   G = X1^T X2 the Gram matrix of a huge unfolding (X1 = X2, only the
//                         lower blocks are formed) or the cross product of two
//                         (the inner-product step of eq. (4)); per-workgroup
//                         partial matrices, summed in a fixed order by
//                         launch_reduce.
//   lg_sgemm  C = op(A) op(B) for the small (<= 256) factor products.
//
// A huge operand is either column-major (a vertical unfolding V(M): element
// (r, k) at r + ld k) or row-major (the transpose of a horizontal unfolding,
// H(M)^T: element (r, k) at k + ld r).  Both are staged through LDS with
// coalesced loads (consecutive lanes read consecutive addresses in either
// layout) into the layout the matrix-core fragments read without bank
// conflicts.
//
// v_mfma_f64_16x16x4f64 (and the f32 form) take A[l%16][k0 + l/16] and
// B[k0 + l/16][l%16] in lane l; result register j of lane l holds
// D[4j + l/16][l%16] (FP64) or D[4(l/16) + j][l%16] (FP32).  A GEMM whose
// output is column-major computes Z^T = B^T X^T by swapping the two operand
// registers, which puts sixteen consecutive rows of Z in sixteen lanes (128-
// byte stores); a row-major output keeps the plain order (sixteen consecutive
// columns per lane group).
#include "ttr_internal.h"

#include <algorithm>
#include <cstdint>

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline d4 mma(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline f4 mma(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// ---------------------------------------------------------------------------
// B packed into fragment order: k-step s (rows 4s..4s+3), column tile t
// (columns 16t..16t+15): Bp[(s * NT + t) * 64 + l] = B(4s + l/16, 16t + l%16),
// zero outside K x N.  B(k, c) = B[k' * sr + c * sc], k' = rperm[k] when a
// row permutation is given, else k.
// ---------------------------------------------------------------------------
__global__ void lg_pack_b(const double *__restrict__ B, int K, int N, long long sr, long long sc,
                          const int *__restrict__ rperm, double *__restrict__ Bp) {
  const int KS = (K + 3) / 4, NT = (N + 15) / 16;
  const long long total = (long long)KS * NT * 64;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int l = (int)(e & 63);
    const long long st = e >> 6;
    const int t = (int)(st % NT), s = (int)(st / NT);
    const int k = 4 * s + l / 16, c = 16 * t + l % 16;
    Bp[e] = (k < K && c < N) ? B[(rperm ? rperm[k] : k) * sr + c * sc] : 0.0;
  }
}

typedef double d2 __attribute__((ext_vector_type(2)));

// Two consecutive doubles p[0], p[1] where both exist (`n` of them are in
// range: 0, 1 or 2); one 16-byte load when `vec` (the caller guarantees the
// alignment).
template <bool VEC>
__device__ inline d2 load2(const double *__restrict__ p, int n) {
  if (n >= 2) {
    if (VEC) return *reinterpret_cast<const d2 *>(p);
    return d2{p[0], p[1]};
  }
  return d2{n >= 1 ? p[0] : 0.0, 0.0};
}

// ---------------------------------------------------------------------------
// Skinny GEMM.  Workgroup = 128 rows of Z, 16 waves: wave w takes row half
// w / 8 and a 32-column block (the four waves of a SIMD get blocks c, c + 4,
// 7 - c and 3 - c, which balances the work a lower-triangular B skips).  K is consumed in
// chunks of 16: the X chunk (128 x 16) is staged in LDS as [k][row] with
// 16-byte loads (two consecutive rows of a column, or two consecutive k of a
// row), double buffered, the next chunk's loads in flight during the current
// products; B's fragments come from the packed copy (L2), one k-step ahead.
// VEC: X is 16-byte aligned with an even leading dimension.
// kperm (XCOL only, nullable): column k of the operand is column kperm[k] of
// X (a gathered operand: X(:, kperm) B).
// tri: 1 = B is lower triangular (B(k, c) = 0 for k < c), 2 = upper
// triangular (B(k, c) = 0 for k > c); its zero k-steps are skipped (adding
// the zero products changes no bit of a finite result).
// ---------------------------------------------------------------------------
constexpr int kGT = 1024;      // threads
constexpr int kGM = 128;       // rows per workgroup
constexpr int kGC = 16;        // k per chunk
constexpr int kGP = kGM + 2;   // LDS pitch (doubles) of a k row
constexpr int kLMaxG = 256;    // largest K

template <bool XCOL, bool ZCOL, bool VEC>
__global__ __launch_bounds__(kGT) void lg_gemm(const double *__restrict__ X, long long M, int K, long long ldx,
                                               const double *__restrict__ Bp, int N, int tri,
                                               double *__restrict__ Z, long long ldz,
                                               const int *__restrict__ kperm) {
  __shared__ double Xs[2][kGC][kGP];
  __shared__ int kp[kLMaxG + kGC];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int rh = w >> 3, cbi = w & 7, cb = rh ? 7 - cbi : cbi;
  const int NT = (N + 15) / 16;
  const int KS = (K + 3) / 4;
  const bool active = cb * 2 < NT;
  const long long row0 = (long long)blockIdx.x * kGM;
  const int nch = (K + kGC - 1) / kGC;
  // staging: 1024 pairs per chunk, one per thread
  //   XCOL: pair (k, rows 2p, 2p+1), k = e / 64, p = e % 64
  //   XROW: pair (row, k 2q, 2q+1),  row = e / 8, q = e % 8
  constexpr int NJ = kGM * kGC / 2 / kGT;
  int sr[NJ], sk[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int e = tid + j * kGT;
    if (XCOL) {
      sk[j] = e >> 6;
      sr[j] = 2 * (e & 63);
    } else {
      sr[j] = e >> 3;
      sk[j] = 2 * (e & 7);
    }
  }
  const long long rows_left = M - row0;
  if (XCOL && kperm) {
    for (int e = tid; e < kLMaxG + kGC; e += kGT) kp[e] = (e < K) ? kperm[e] : 0;
    __syncthreads();
  }
  d2 pre[NJ];
  auto load = [&](int c) {
    const int k0 = c * kGC;
    const bool full = rows_left >= kGM && k0 + kGC <= K;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const long long gr = row0 + sr[j];
      const int gk = k0 + sk[j];
      const double *p = XCOL ? X + gr + ldx * (kperm ? kp[gk] : gk) : X + gr * ldx + gk;
      int n;
      if (full) n = 2;
      else if (XCOL) n = (gk < K) ? (int)std::max(0LL, std::min(2LL, M - gr)) : 0;
      else n = (gr < M) ? std::max(0, std::min(2, K - gk)) : 0;
      pre[j] = load2<VEC>(p, n);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      if (XCOL) {
        *reinterpret_cast<d2 *>(&Xs[buf][sk[j]][sr[j]]) = pre[j];
      } else {
        Xs[buf][sk[j]][sr[j]] = pre[j][0];
        Xs[buf][sk[j] + 1][sr[j]] = pre[j][1];
      }
    }
  };
  const double *Bw = Bp + (long long)(cb * 2) * 64 + lane;  // + (ks NT + ct) 64
  auto loadb = [&](int ks, double *bf) {
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
      bf[ct] = (active && ks < KS && cb * 2 + ct < NT) ? Bw[((long long)ks * NT + ct) * 64] : 0.0;
  };
  d4 acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  double bcur[2], bnext[2];
  loadb(0, bcur);
  load(0);
  store(0);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) load(c + 1);
#pragma unroll
    for (int s = 0; s < kGC / 4; ++s) {
      const int ks = c * (kGC / 4) + s;
      loadb(ks + 1, bnext);
      if (active && ks < KS) {
        double af[4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) af[rt] = Xs[buf][4 * s + lane / 16][rh * 64 + rt * 16 + lane % 16];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          const int t = cb * 2 + ct;
          if (t >= NT) continue;
          if (tri == 1 && 4 * ks + 3 < 16 * t) continue;   // B(k, c) = 0 for k < c
          if (tri == 2 && 4 * ks > 16 * t + 15) continue;  // B(k, c) = 0 for k > c
#pragma unroll
          for (int rt = 0; rt < 4; ++rt)
            acc[rt][ct] = ZCOL ? mma(bcur[ct], af[rt], acc[rt][ct]) : mma(af[rt], bcur[ct], acc[rt][ct]);
        }
      }
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) bcur[ct] = bnext[ct];
    }
    if (c + 1 < nch) {
      store(buf ^ 1);
      __syncthreads();
    }
  }
  if (!active) return;
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int t = cb * 2 + ct;
      if (t >= NT) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        long long r;
        int col;
        if (ZCOL) {
          r = row0 + rh * 64 + rt * 16 + lane % 16;
          col = t * 16 + 4 * j + lane / 16;
        } else {
          r = row0 + rh * 64 + rt * 16 + 4 * j + lane / 16;
          col = t * 16 + lane % 16;
        }
        if (r < M && col < N) {
          if (ZCOL) Z[r + ldz * col] = acc[rt][ct][j];
          else Z[r * ldz + col] = acc[rt][ct][j];
        }
      }
    }
}

// ---------------------------------------------------------------------------
// Skinny Gram.  Workgroup (x, y) sums rows [x rpw, (x+1) rpw) of X1^T X2 for
// the 64 x 64 blocks 4y .. 4y+3 of the result (SYM: the lower blocks pb >= qb
// only, numbered row by row, a diagonal block whole, an off-diagonal block
// also written transposed) into part + x K1 K2 (column-major K1 x K2).  Eight
// waves, two per block: wave w takes the 32-column half w % 2 of block
// 4y + w / 2.  Rows are consumed in chunks of 16, staged in LDS as [row][k]
// (double buffered, the next chunk's loads in flight).  T = float: FP32
// products and per-wave FP32 accumulation over the workgroup's rows (the
// mixed-precision first passes), written to the partials in FP64.
// ---------------------------------------------------------------------------
constexpr int kRC = 16;          // rows per chunk
constexpr int kRP = 256 + 2;     // LDS pitch of a staged row
constexpr int kGrT = 512;        // threads (8 waves)

template <class T>
struct AccOf;
template <>
struct AccOf<double> {
  typedef d4 type;
};
template <>
struct AccOf<float> {
  typedef f4 type;
};

__host__ __device__ inline int lg_nblocks(int nb1, int nb2, bool sym) { return sym ? nb1 * (nb1 + 1) / 2 : nb1 * nb2; }

// fscale (FP32 only): fscale[0] = 2^-e multiplies every element before it is
// rounded to FP32 (keeps tiny or huge data inside FP32's range), fscale[1] =
// 2^2e multiplies the FP64 partials (exact: powers of two).
template <class T, bool XCOL, bool SYM, bool VEC>
__global__ __launch_bounds__(kGrT) void lg_gram(const double *__restrict__ X1, const double *__restrict__ X2,
                                                long long M, int K1, int K2, long long ld1, long long ld2,
                                                long long rpw, double *__restrict__ part,
                                                const double *__restrict__ fscale) {
  const double sin = (sizeof(T) == 4) ? fscale[0] : 1.0, sout = (sizeof(T) == 4) ? fscale[1] : 1.0;
  typedef typename AccOf<T>::type V;
  constexpr int NOP = SYM ? 1 : 2;
  __shared__ T S[NOP][2][kRC][kRP];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nb1 = (K1 + 63) / 64, nb2 = (K2 + 63) / 64;
  const int bi = 4 * blockIdx.y + (w >> 1), half = w & 1;
  const bool active = bi < lg_nblocks(nb1, nb2, SYM);
  int pb = 0, qb = 0;
  if (SYM) {
    int ww = bi;
    for (pb = 0; pb < nb1; ++pb) {
      if (ww <= pb) {
        qb = ww;
        break;
      }
      ww -= pb + 1;
    }
  } else {
    pb = bi / nb2;
    qb = bi % nb2;
  }
  const int q0 = 64 * qb + 32 * half;  // this wave's 32 columns
  const long long r0 = (long long)blockIdx.x * rpw;
  const long long r1 = std::min(M, r0 + rpw);
  const int nch = r1 > r0 ? (int)((r1 - r0 + kRC - 1) / kRC) : 0;
  const int Kp[2] = {(K1 + 15) & ~15, (K2 + 15) & ~15};
  const int Kv[2] = {K1, K2};
  const double *Xo[2] = {X1, X2};
  const long long ldo[2] = {ld1, ld2};
  // staging: pairs of consecutive elements, kPairs per thread per operand
  //   XCOL: (column k, rows 2p, 2p+1), k = e / 8, p = e % 8 (8 Kp pairs)
  //   XROW: (row, columns 2q, 2q+1), row = e / 128, q = e % 128 (16 x 128)
  constexpr int kPairs = kRC * 256 / 2 / kGrT;
  d2 pre[NOP][kPairs];
  auto pair_of = [&](int e, int *r, int *k) {
    if (XCOL) {
      *k = e >> 3;
      *r = 2 * (e & 7);
    } else {
      *r = e >> 7;
      *k = 2 * (e & 127);
    }
  };
  auto load = [&](int o, long long rb) {
#pragma unroll
    for (int j = 0; j < kPairs; ++j) {
      int r, k;
      pair_of(tid + j * kGrT, &r, &k);
      const long long gr = rb + r;
      int n = 0;
      if (k < Kp[o]) {
        if (XCOL) n = (k < Kv[o]) ? (int)std::max(0LL, std::min(2LL, r1 - gr)) : 0;
        else n = (gr < r1) ? std::max(0, std::min(2, Kv[o] - k)) : 0;
      }
      const double *p = XCOL ? Xo[o] + gr + ldo[o] * k : Xo[o] + gr * ldo[o] + k;
      pre[o][j] = load2<VEC>(p, n);
    }
  };
  auto store = [&](int o, int buf) {
#pragma unroll
    for (int j = 0; j < kPairs; ++j) {
      int r, k;
      pair_of(tid + j * kGrT, &r, &k);
      if (k < Kp[o]) {
        if (XCOL) {
          S[o][buf][r][k] = (T)(sin * pre[o][j][0]);
          S[o][buf][r + 1][k] = (T)(sin * pre[o][j][1]);
        } else {
          S[o][buf][r][k] = (T)(sin * pre[o][j][0]);
          S[o][buf][r][k + 1] = (T)(sin * pre[o][j][1]);
        }
      }
    }
  };
  V acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = V{0, 0, 0, 0};
  if (nch > 0) {
#pragma unroll
    for (int o = 0; o < NOP; ++o) {
      load(o, r0);
      store(o, 0);
    }
  }
  __syncthreads();
  const int np = active ? std::min(4, (K1 - 64 * pb + 15) / 16) : 0;
  const int nq = active ? std::max(0, std::min(2, (K2 - q0 + 15) / 16)) : 0;
  const int ob = SYM ? 0 : 1;
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) {
#pragma unroll
      for (int o = 0; o < NOP; ++o) load(o, r0 + (long long)(c + 1) * kRC);
    }
    if (nq > 0) {
#pragma unroll
      for (int s = 0; s < kRC / 4; ++s) {
        T af[4], bf[2];
#pragma unroll
        for (int pt = 0; pt < 4; ++pt)
          af[pt] = (pt < np) ? S[0][buf][4 * s + lane / 16][64 * pb + 16 * pt + lane % 16] : T(0);
#pragma unroll
        for (int qt = 0; qt < 2; ++qt)
          bf[qt] = (qt < nq) ? S[ob][buf][4 * s + lane / 16][q0 + 16 * qt + lane % 16] : T(0);
#pragma unroll
        for (int pt = 0; pt < 4; ++pt)
#pragma unroll
          for (int qt = 0; qt < 2; ++qt)
            if (pt < np && qt < nq) acc[pt][qt] = mma(af[pt], bf[qt], acc[pt][qt]);
      }
    }
    if (c + 1 < nch) {
      // the other buffer was last read before the previous barrier
#pragma unroll
      for (int o = 0; o < NOP; ++o) store(o, buf ^ 1);
      __syncthreads();
    }
  }
  if (nq <= 0) return;
  double *P = part + (long long)blockIdx.x * K1 * K2;
#pragma unroll
  for (int pt = 0; pt < 4; ++pt)
#pragma unroll
    for (int qt = 0; qt < 2; ++qt)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int p, q;
        if (sizeof(T) == 8) {
          p = 64 * pb + 16 * pt + 4 * j + lane / 16;
          q = q0 + 16 * qt + lane % 16;
        } else {
          p = 64 * pb + 16 * pt + 4 * (lane / 16) + j;
          q = q0 + 16 * qt + lane % 16;
        }
        const double v = sout * (double)acc[pt][qt][j];
        if (p < K1 && q < K2) {
          P[p + (long long)K1 * q] = v;
          if (SYM && pb != qb) P[q + (long long)K1 * p] = v;
        }
      }
}

// ---------------------------------------------------------------------------
// Small GEMM: C (m x n, ld ldc) = A B with A(i, k) = A[i ar + k ac],
// B(k, j) = B[k br + j bc] (any transposes through the strides); one wave per
// 16 x 16 tile of C, fragments straight from global memory (L2-resident).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void lg_sgemm(const double *__restrict__ A, long long ar, long long ac,
                                               const double *__restrict__ B, long long br, long long bc, int m,
                                               int n, int k, double *__restrict__ C, long long ldc) {
  const int lane = threadIdx.x;
  const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
  const int i = i0 + lane % 16, j = j0 + lane % 16;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < k; k0 += 4) {
    const int kk = k0 + lane / 16;
    const double a = (i < m && kk < k) ? A[i * ar + kk * ac] : 0.0;
    const double b = (j < n && kk < k) ? B[kk * br + j * bc] : 0.0;
    acc = mma(a, b, acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ci = i0 + 4 * r + lane / 16, cj = j0 + lane % 16;
    if (ci < m && cj < n) C[ci + ldc * cj] = acc[r];
  }
}

// ---------------------------------------------------------------------------
// Right product of a slice-wise Kronecker product (the implicit Hadamard
// product of §3.2.2): C(i) = (A(i) (x) B(i)) T for every slice i, with
// A(i) rA0 x rA1, B(i) rB0 x rB1 (all <= 16) and T (rA1 rB1) x k, never
// forming A(i) (x) B(i).  Column t of C(i) is vec(B(i) T_t A(i)^T), T_t the
// rB1 x rA1 reshape of T(:, t) (T_t(by, bx) = T(bx rB1 + by, t)), so per slice
// and column two 16 x 16 x 16 products replace a (rA0 rB0) x (rA1 rB1) one:
//   D1 = T_t^T B(i)^T = W_t^T   (rA1 x rB0; its result registers are the
//                                operand fragments of the next product)
//   D2 = A(i) W_t^T  = O_t^T    (rA0 x rB0): C(ax rB0 + ay, i, t) = D2(ax, ay)
// Wave = four columns t (their T fragments held in registers) over the
// workgroup's run of slices; the slices' A and B fragments are read once per
// slice and wave (L2-shared by the waves of other columns).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void lg_kron_right(const double *__restrict__ A, int a0, int a1,
                                                     const double *__restrict__ B, int b0, int b1, long long I,
                                                     const double *__restrict__ T, long long ldt, int k, long long spw,
                                                     double *__restrict__ C) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int t0 = (blockIdx.y * 4 + w) * 4;  // this wave's four columns
  if (t0 >= k) return;
  const int r16 = lane % 16, g = lane / 16;
  // T_t^T fragments: A-operand rows bx = r16, k-step s covers by = 4s + g
  double tf[4][4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int t = t0 + j, bx = r16, by = 4 * s + g;
      tf[j][s] = (t < k && bx < a1 && by < b1) ? T[(bx * b1 + by) + ldt * t] : 0.0;
    }
  const long long i0 = (long long)blockIdx.x * spw, i1 = std::min(I, i0 + spw);
  const long long cs = (long long)a0 * b0;  // rows of C
  for (long long i = i0; i < i1; ++i) {
    // B(i)^T as B-operand of D1: rows by = 4s + g (k), columns ay = r16
    // A(i) as A-operand of D2: rows ax = r16, k-step s covers bx = 4s + g
    double bf[4], af[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int by = 4 * s + g, bx = 4 * s + g;
      bf[s] = (r16 < b0 && by < b1) ? B[r16 + (long long)b0 * (i + I * by)] : 0.0;
      af[s] = (r16 < a0 && bx < a1) ? A[r16 + (long long)a0 * (i + I * bx)] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int t = t0 + j;
      if (t >= k) break;
      d4 d1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4; ++s) d1 = mma(tf[j][s], bf[s], d1);
      // d1 register s = W_t^T(bx = 4s + g, ay = r16): the B-operand of k-step s
      d4 d2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4; ++s) d2 = mma(af[s], d1[s], d2);
      // d2 register r = O_t^T(ax = 4r + g, ay = r16)
      double *Ct = C + cs * (i + I * t);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ax = 4 * r + g;
        if (ax < a0 && r16 < b0) Ct[ax * b0 + r16] = d2[r];
      }
    }
  }
}

}  // namespace

void launch_lg_kron_right(hipStream_t s, const double *A, int a0, int a1, const double *B, int b0, int b1, long long I,
                          const double *T, long long ldt, int k, double *C) {
  // about 16 waves' worth of slices per workgroup column group, >= 1024 workgroups
  const long long gy = (k + 15) / 16;
  long long gx = std::max(1LL, std::min(I, (4096 + gy - 1) / gy));
  const long long spw = (I + gx - 1) / gx;
  gx = (I + spw - 1) / spw;
  hipLaunchKernelGGL(lg_kron_right, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s, A, a0, a1, B, b0, b1, I, T, ldt,
                     k, spw, C);
}

size_t lg_packed_doubles(int K, int N) { return (size_t)((K + 3) / 4) * ((N + 15) / 16) * 64; }

void launch_lg_gemm(hipStream_t s, const double *X, long long M, int K, long long ldx, int xcol, const double *B,
                    long long bsr, long long bsc, int N, int tri, double *Bp, double *Z, long long ldz, int zcol,
                    const int *perm) {
  const long long np = (long long)lg_packed_doubles(K, N);
  hipLaunchKernelGGL(lg_pack_b, dim3((unsigned)std::min<long long>(1024, (np + 255) / 256)), dim3(256), 0, s, B, K,
                     N, bsr, bsc, perm, Bp);
  if (!xcol) perm = nullptr;  // the gathered form is column-major only (callers check)
  const dim3 grid((unsigned)((M + kGM - 1) / kGM));
  const bool vec = ((uintptr_t)X % 16 == 0) && (ldx % 2 == 0);
#define TTR_GEMM(XC, ZC, V) \
  hipLaunchKernelGGL((lg_gemm<XC, ZC, V>), grid, dim3(kGT), 0, s, X, M, K, ldx, Bp, N, tri, Z, ldz, perm)
  if (vec) {
    if (xcol && zcol) TTR_GEMM(true, true, true);
    else if (xcol) TTR_GEMM(true, false, true);
    else if (zcol) TTR_GEMM(false, true, true);
    else TTR_GEMM(false, false, true);
  } else {
    if (xcol && zcol) TTR_GEMM(true, true, false);
    else if (xcol) TTR_GEMM(true, false, false);
    else if (zcol) TTR_GEMM(false, true, false);
    else TTR_GEMM(false, false, false);
  }
#undef TTR_GEMM
}

LGramGrid lg_gram_grid(long long M, int f32) {
  // about 1024 rows per workgroup at least, at most 512 workgroups (FP64 and
  // FP32 alike: the callers' partial-matrix workspaces hold 512)
  (void)f32;
  const long long cap = 512;
  long long nwg = std::max(1LL, std::min(cap, (M + 1023) / 1024));
  LGramGrid g;
  g.rpw = (M + nwg - 1) / nwg;
  g.rpw = (g.rpw + kRC - 1) / kRC * kRC;
  g.nwg = (int)std::max(1LL, (M + g.rpw - 1) / g.rpw);
  return g;
}

namespace {

// Scale of an FP32 Gram: the largest finite |x| over up to 4096 evenly
// spaced samples of the n doubles at X, m, gives out[0] = 2^-e with
// 2^e <= m < 2^(e+1) and out[1] = 2^(2e) (1 and 1 when m = 0).  Only the
// exponent matters, so a sample suffices; each thread issues its 16 loads
// at once.
__global__ __launch_bounds__(256) void lg_scale_probe(const double *__restrict__ X, long long n, double *out) {
  __shared__ double red[256];
  constexpr int kPer = 16;
  const long long ns = std::min(n, 256LL * kPer);
  const long long stride = std::max(1LL, n / std::max(ns, 1LL));
  double m = 0.0;
  double v[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const long long j = threadIdx.x + 256LL * q;
    v[q] = (j < ns) ? fabs(X[j * stride]) : 0.0;
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q)
    if (v[q] <= 1.7976931348623157e308) m = fmax(m, v[q]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mx = red[0];
    if (mx > 0.0) {
      const int e = ilogb(mx);
      out[0] = ldexp(1.0, -e);
      out[1] = ldexp(1.0, 2 * e);
    } else {
      out[0] = 1.0;
      out[1] = 1.0;
    }
  }
}

}  // namespace

void launch_lg_scale_probe(hipStream_t s, const double *X, long long n, double *out) {
  hipLaunchKernelGGL(lg_scale_probe, dim3(1), dim3(256), 0, s, X, n, out);
}

int launch_lg_gram(hipStream_t s, const double *X1, const double *X2, long long M, int K1, int K2, long long ld1,
                   long long ld2, int xcol, int f32, double *part, const double *fscale) {
  const LGramGrid g = lg_gram_grid(M, f32);
  const bool sym = (X2 == nullptr);
  const int nb1 = (K1 + 63) / 64, nb2 = (K2 + 63) / 64;
  const int ngrp = (lg_nblocks(nb1, nb2, sym) + 3) / 4;
  const dim3 grid(g.nwg, ngrp), block(kGrT);
  // 16-byte loads need aligned operands with even leading dimensions (and
  // row-range starts: rpw is a multiple of 16)
  const bool vec = ((uintptr_t)X1 % 16 == 0) && (ld1 % 2 == 0) &&
                   (sym || (((uintptr_t)X2 % 16 == 0) && (ld2 % 2 == 0)));
#define TTR_LG(T, XC, SY)                                                                                        \
  do {                                                                                                           \
    if (vec)                                                                                                     \
      hipLaunchKernelGGL((lg_gram<T, XC, SY, true>), grid, block, 0, s, X1, sym ? X1 : X2, M, K1, sym ? K1 : K2, \
                         ld1, sym ? ld1 : ld2, g.rpw, part, fscale);                                             \
    else                                                                                                         \
      hipLaunchKernelGGL((lg_gram<T, XC, SY, false>), grid, block, 0, s, X1, sym ? X1 : X2, M, K1,               \
                         sym ? K1 : K2, ld1, sym ? ld1 : ld2, g.rpw, part, fscale);                              \
  } while (0)
  if (sym) {
    if (f32) {
      if (xcol) TTR_LG(float, true, true);
      else TTR_LG(float, false, true);
    } else {
      if (xcol) TTR_LG(double, true, true);
      else TTR_LG(double, false, true);
    }
  } else {
    if (xcol) TTR_LG(double, true, false);
    else TTR_LG(double, false, false);
  }
#undef TTR_LG
  return g.nwg;
}

void launch_lg_sgemm(hipStream_t s, const double *A, long long ar, long long ac, const double *B, long long br,
                     long long bc, int m, int n, int k, double *C, long long ldc) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(lg_sgemm, dim3((m + 15) / 16, (n + 15) / 16), dim3(64), 0, s, A, ar, ac, B, br, bc, m, n, k, C,
                     ldc);
}
