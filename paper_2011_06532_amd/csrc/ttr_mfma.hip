// Matrix-core (MFMA) streaming kernels of the QR-by-Gram factorizations and
// of the output pass (FP64, and FP32 for the mixed-precision first Gram
// pass), on cores stored in the paper's layout (§3.1): entry (a, i, b) of an
// R0 x I x R1 core at a + R0*(i + I*b).
//
// v_mfma_f64_16x16x4f64 on gfx950: lane l supplies A[l%16][k0 + l/16] and
// B[k0 + l/16][l%16]; the 16x16 result sits in four registers per lane with
// register r of lane l holding D[4r + l/16][l%16].  Register r of a result tile
// is therefore exactly the operand fragment of k-step 4r..4r+3 for a product
// that contracts over the tile's row index, so the chains below
//   Gram, right factor:  Wt = Q^T M^T,  G  += Wt^T Wt   (contract over c)
//   Gram, left factor:   Y  = P M,      G0 += Y^T Y     (contract over rho)
//   output:              W  = M Q,      Y^T = W^T P^T   (contract over alpha)
// feed one product's accumulators straight into the next, without LDS; a
// product with its operands swapped gives bitwise the transposed result.
// The small factors (<= 64 x 64) sit in LDS pre-arranged as per-lane
// fragments; slices are read from HBM once, 16 consecutive rows per lane
// group, or two consecutive rows per lane (16-byte loads) where the product
// contracts over rows.  Products accumulate one 16-row or 16-column band at a
// time where the band's contribution is complete on its own, which keeps the
// live accumulators to NT tiles and the FP64 kernels at two waves per SIMD.
//
// Each workgroup (4 waves) owns a contiguous range of slices; the waves take
// slices round-robin, keep their own partial Gram in registers, and combine
// them in LDS in a fixed order, so results are reproducible run to run.
#include "ttr_internal.h"

#include <algorithm>
#include <type_traits>

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kWaves = 4;

// Arithmetic of a matrix-core chain.  Both 16x16x4 forms take operands the
// same way (lane l supplies A[l%16][k0 + l/16] and B[k0 + l/16][l%16]); they
// differ in where the result lands: register r of lane l holds row
// row(l/16, r) of column l%16.
struct F64 {
  using T = double;
  using V = d4;
  __device__ static V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __host__ __device__ static constexpr int row(int g, int r) { return 4 * r + g; }
};
struct F32 {
  using T = float;
  using V = f4;
  __device__ static V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __host__ __device__ static constexpr int row(int g, int r) { return 4 * g + r; }
};

__device__ inline d4 mfma(double a, double b, d4 c) { return F64::mma(a, b, c); }

// A-operand fragments of S (rows x cols): frag[(t*KS + ks)*64 + l] = S(t*16 + l%16, ks*4 + l/16).
// S(r, c) = S[r*sr + c*sc]; S == nullptr means the identity.  Zero outside.
template <class T = double>
__device__ void build_afrag(T *frag, const double *S, int rows, int cols, long long sr, long long sc, int nt,
                            int KS, double scale = 1.0) {
  const int total = nt * KS * 64;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int l = e & 63;
    const int ks = (e >> 6) % KS;
    const int t = (e >> 6) / KS;
    const int r = t * 16 + (l & 15);
    const int c = ks * 4 + (l >> 4);
    double v = 0.0;
    if (r < rows && c < cols) v = S ? S[r * sr + c * sc] : (r == c ? 1.0 : 0.0);
    frag[e] = (sizeof(T) == 4) ? (T)(v * scale) : (T)v;
  }
}

// B-operand fragments of S (rows x cols): frag[(t*KS + ks)*64 + l] = S(ks*4 + l/16, t*16 + l%16).
template <class T = double>
__device__ void build_bfrag(T *frag, const double *S, int rows, int cols, long long sr, long long sc, int nt,
                            int KS) {
  const int total = nt * KS * 64;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int l = e & 63;
    const int ks = (e >> 6) % KS;
    const int t = (e >> 6) / KS;
    const int r = ks * 4 + (l >> 4);
    const int c = t * 16 + (l & 15);
    double v = 0.0;
    if (r < rows && c < cols) v = S ? S[r * sr + c * sc] : (r == c ? 1.0 : 0.0);
    frag[e] = (T)v;
  }
}

// Adds this wave's Gram tiles (lower block triangle, tile (u, v) with u >= v)
// into the workgroup's dense gd x gd matrix in LDS (FP64), waves in a fixed
// order.
template <int NT, class A>
__device__ void reduce_gram(const typename A::V (&G)[NT][NT], int nt, int gd, double *Gs, double *out,
                            double post = 1.0) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  for (int e = threadIdx.x; e < gd * gd; e += blockDim.x) Gs[e] = 0.0;
  __syncthreads();
  for (int w = 0; w < kWaves; ++w) {
    if (wave == w) {
#pragma unroll
      for (int u = 0; u < NT; ++u)
#pragma unroll
        for (int v = 0; v < NT; ++v)
          if (v <= u && u < nt) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = u * 16 + A::row(g, r);
              const int col = v * 16 + j;
              if (row < gd && col < gd && row >= col) Gs[row + gd * col] += (double)G[u][v][r];
            }
          }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < gd * gd; e += blockDim.x) {
    const int row = e % gd, col = e / gd;
    const double v = (row >= col) ? Gs[row + gd * col] : Gs[col + gd * row];
    out[e] = (sizeof(typename A::T) == 4) ? v * post : v;
  }
}

// Loads the operand fragments of one slice: buf[ks][t] = M(t*16 + l%16, ks*4 + l/16)
// (ROWS16 = true) or M(ks*4 + l/16, t*16 + l%16) (ROWS16 = false), zero outside
// the a x b slice.  M(alpha, beta) = Xi[alpha + col*beta].  Data are FP64 in
// memory; T = float rounds them on load.
template <int NT, int KS, bool ROWS16, class T = double>
__device__ inline void load_slice(const double *__restrict__ Xi, long long col, int a, int b, int g, int j,
                                  T (&buf)[KS][NT]) {
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int r = ROWS16 ? t * 16 + j : ks * 4 + g;   // alpha
      const int c = ROWS16 ? ks * 4 + g : t * 16 + j;   // beta
      double v = 0.0;
      if (r < a && c < b) v = Xi[r + col * c];
      buf[ks][t] = (T)v;
    }
}

// Loads one 16-row band t of the operand fragments of a slice:
// buf[ks] = M(t*16 + l%16, ks*4 + l/16) (ROWS16) or M(ks*4 + l/16, t*16 + l%16),
// zero outside the a x b slice.
template <int KS, bool ROWS16>
__device__ inline void load_band(const double *__restrict__ Xi, long long col, int a, int b, int g, int j, int t,
                                 double (&buf)[KS]) {
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int r = ROWS16 ? t * 16 + j : ks * 4 + g;
    const int c = ROWS16 ? ks * 4 + g : t * 16 + j;
    buf[ks] = (r < a && c < b) ? Xi[r + col * c] : 0.0;
  }
}

// Products that contract over alpha (the fast index of a slice) take their
// k-steps in "pair order": k-step ks covers alpha = 8 (ks/2) + 2 g + ks%2, so a
// lane holds two consecutive alpha of one column and reads them with one
// 16-byte load (V2: a even and a 16-byte aligned core).  Any order of the
// contraction index is valid as long as both operands use it.
__device__ __host__ inline int pair_alpha(int ks, int g) { return 8 * (ks >> 1) + 2 * g + (ks & 1); }

// buf[ks][t] = M(pair_alpha(ks, g), 16t + j), zero outside the a x b slice.
template <int NT, int KP, bool V2, class T = double>
__device__ inline void load_slice_pairs(const double *__restrict__ Xi, long long col, int a, int b, int g, int j,
                                        T (&buf)[KP][NT]) {
#pragma unroll
  for (int kk = 0; kk < KP / 2; ++kk)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int r = 8 * kk + 2 * g, c = 16 * t + j;
      double v0 = 0.0, v1 = 0.0;
      if (V2) {
        // a even: r < a implies r + 1 < a
        if (r < a && c < b) {
          const double2 v = *reinterpret_cast<const double2 *>(Xi + r + col * c);
          v0 = v.x;
          v1 = v.y;
        }
      } else {
        if (r < a && c < b) v0 = Xi[r + col * c];
        if (r + 1 < a && c < b) v1 = Xi[r + 1 + col * c];
      }
      buf[2 * kk][t] = (T)v0;
      buf[2 * kk + 1][t] = (T)v1;
    }
}

// A-operand fragments of S (rows x cols) with the column index in pair order:
// frag[(t*KP + ks)*64 + l] = S(t*16 + l%16, pair_alpha(ks, l/16)).
template <class T = double>
__device__ void build_afrag_pairs(T *frag, const double *S, int rows, int cols, long long sr, long long sc, int nt,
                                  int KP, double scale = 1.0) {
  const int total = nt * KP * 64;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int l = e & 63;
    const int ks = (e >> 6) % KP;
    const int t = (e >> 6) / KP;
    const int r = t * 16 + (l & 15);
    const int c = pair_alpha(ks, l >> 4);
    double v = 0.0;
    if (r < rows && c < cols) v = S ? S[r * sr + c * sc] : (r == c ? 1.0 : 0.0);
    frag[e] = (sizeof(T) == 4) ? (T)(v * scale) : (T)v;
  }
}

// Writes column tile c (columns 16c..16c+15) of an nrow x ncol block of one
// output slice, held as NT accumulator tiles: register r of yc[u] holds row
// 16u + row(g, r), column 16c + j; column c of the slice starts at Yi + ocol*c
// with its rows contiguous.  The tile goes through the wave's LDS buffer Lw
// (ld LDP) so that the stores leave as runs of consecutive rows, not 16
// scattered 32-byte pieces.
template <int NT, class A, class VT>
__device__ inline void store_col(const VT (&yc)[NT], int c, int nrow, int ncol, double *__restrict__ Yi,
                                 long long ocol, double *Lw, int LDP, int lane, int g, int j) {
  __asm__ volatile("" ::: "memory");
#pragma unroll
  for (int u = 0; u < NT; ++u)
#pragma unroll
    for (int r = 0; r < 4; ++r) Lw[(u * 16 + A::row(g, r)) + LDP * j] = (double)yc[u][r];
  // one wave owns Lw and its LDS operations complete in order
  __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  const int nc = min(16, ncol - c * 16);
  // element e = lane + 64 m of the tile is (row e % nrow, column e / nrow):
  // one division up front, then steps of 64 = q nrow + rem
  const int q = 64 / nrow, rem = 64 - q * nrow;
  int rr = lane % nrow, jj = lane / nrow;
  for (int e = lane; e < nrow * nc; e += 64) {
    Yi[rr + ocol * (c * 16 + jj)] = Lw[rr + LDP * jj];
    rr += rem;
    jj += q;
    if (rr >= nrow) {
      rr -= nrow;
      ++jj;
    }
  }
  __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}


// ---------------------------------------------------------------------------
// Gram with a right factor: G (a x a) = sum_i (M_i Q)(M_i Q)^T, M_i = X(:, i, :)
// (a x b), Q (b x q).  The left Gram of the horizontal unfolding of X x_3 Q^T
// (orthonormalization sweep, §2.3 / Alg. 1).  NT = 16-tiles per dimension,
// KS = k-steps over b (ceil(b/4)).  A = F64, or F32 for the mixed-precision
// first pass (slices and Q rounded to FP32, FP32 accumulation per wave).
// ---------------------------------------------------------------------------
template <int NT, int KS, class A, bool GD = false>
__device__ __forceinline__ void gram_right_factor_body(const int wg, const double *__restrict__ X, int a, int b, long long I,
                                                                const double *__restrict__ Q, int q, long long sQr,
                                                                long long sQc, int tri, long long spw,
                                                                double *__restrict__ partials,
                                                                const double *__restrict__ fscale = nullptr) {
  using T = typename A::T;
  using V = typename A::V;
  // FP32 (fscale given): slices and Q are multiplied by powers of two before
  // they are rounded to FP32 and the Gram is scaled back (exactly) at the end
  const double sM = (sizeof(T) == 4 && fscale) ? fscale[0] : 1.0;
  const double sF = (sizeof(T) == 4 && fscale) ? fscale[1] : 1.0;
  const double post = (sizeof(T) == 4 && fscale) ? fscale[2] : 1.0;
  __shared__ T frag[NT * KS * 64];
  __shared__ double Gs[NT * 16 * NT * 16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  // GD: the dimensions are known only at run time (batched launches); skip
  // k-steps and 16-tiles past them
  const int ksr = (b + 3) / 4, ntq = (q + 15) / 16, nta = (a + 15) / 16;
  // A operand: Q^T (q x b), Q^T(c, beta) = Q(beta, c)
  build_afrag<T>(frag, Q, q, b, sQc, sQr, NT, KS, sF);
  __syncthreads();
  V G[NT][NT];
#pragma unroll
  for (int u = 0; u < NT; ++u)
#pragma unroll
    for (int v = 0; v < NT; ++v) G[u][v] = V{0, 0, 0, 0};
  const long long beg = (long long)wg * spw;
  const long long end = std::min(beg + spw, I);
  const long long col = (long long)a * I;
  // register prefetch of the next slice for FP32 and NT <= 2.  FP64 at NT = 3
  // runs two waves per SIMD without it (measured faster than one wave with
  // it: the other wave's products cover the load latency).  The prefetch holds
  // the raw FP64 loads; FP32 rounding happens when the slice becomes current,
  // so the loads stay in flight across the products.
  constexpr bool PF = (NT <= 2) || sizeof(T) == 4;
  T cur[KS][NT];
  double nxt[KS][NT];  // used only with PF
  long long i = beg + wave;
  if constexpr (PF)
    if (i < end) {
      load_slice<NT, KS, true>(X + (long long)a * i, col, a, b, g, j, nxt);
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int t = 0; t < NT; ++t) cur[ks][t] = (sizeof(T) == 4) ? (T)(nxt[ks][t] * sM) : (T)nxt[ks][t];
    }
  for (; i < end; i += kWaves) {
    // NT = 4: keep the operand fragments in LDS rather than hoisted into
    // registers, which is what lets two waves share a SIMD
    if constexpr (NT == 4) __asm__ volatile("" ::: "memory");
    if constexpr (PF) {
      if (i + kWaves < end) load_slice<NT, KS, true>(X + (long long)a * (i + kWaves), col, a, b, g, j, nxt);
    } else {
      load_slice<NT, KS, true, T>(X + (long long)a * i, col, a, b, g, j, cur);
    }
    // one 16-row band of Wt at a time: its Gram contribution is complete on
    // its own, so only NT accumulator tiles of Wt are live (this keeps the
    // FP64 kernel at two waves per SIMD)
#pragma unroll
    for (int cb = 0; cb < NT; ++cb) {
      if (GD && cb >= ntq) continue;
      V wt[NT];  // Wt(c, alpha), c in band cb, one tile per alpha-tile
#pragma unroll
      for (int t = 0; t < NT; ++t) wt[t] = V{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        // lower-triangular Q: Q^T(c, beta) = 0 for beta < c, so k-steps below 4 cb vanish
        if ((tri && ks < 4 * cb) || (GD && ks >= ksr)) continue;
        const T qa = frag[(cb * KS + ks) * 64 + lane];
#pragma unroll
        for (int t = 0; t < NT; ++t)
          if (!GD || t < nta) wt[t] = A::mma(qa, cur[ks][t], wt[t]);
      }
      // G(alpha, alpha') += sum_c Wt(c, alpha) Wt(c, alpha'); register r holds
      // rows c = cb*16 + row(g, r); rows past q are zero padding
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (cb * 16 + A::row(0, r) >= q) continue;
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
          for (int v = 0; v <= u; ++v)
            if (!GD || u < nta) G[u][v] = A::mma(wt[u][r], wt[v][r], G[u][v]);
      }
    }
    if constexpr (PF) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int t = 0; t < NT; ++t) cur[ks][t] = (sizeof(T) == 4) ? (T)(nxt[ks][t] * sM) : (T)nxt[ks][t];
    }
  }
  reduce_gram<NT, A>(G, NT, a, Gs, partials + (long long)wg * a * a, post);
}

template <int NT, int KS, class A>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(NT <= 3 || (KS <= 13 && sizeof(typename A::T) == 8) ? 2 : 1, NT <= 3 || (KS <= 13 && sizeof(typename A::T) == 8) ? 2 : 1))) void k_gram_right_factor(const double *__restrict__ X, int a, int b, long long I,
                                                                const double *__restrict__ Q, int q, long long sQr,
                                                                long long sQc, int tri, long long spw,
                                                                double *__restrict__ partials,
                                                                const double *__restrict__ fscale) {
  gram_right_factor_body<NT, KS, A>(blockIdx.x, X, a, b, I, Q, q, sQr, sQc, tri, spw, partials, fscale);
}

// ---------------------------------------------------------------------------
// Gram with a left factor: G0 (b x b) = sum_i (P M_i)^T (P M_i), P (p x a).
// The Gram of the vertical unfolding of P x_1 X (truncation sweep, §2.4).
// KS = k-steps over a (ceil(a/4)).
// ---------------------------------------------------------------------------
template <int NT, int KS, class A, bool GD = false>
__device__ __forceinline__ void gram_left_factor_body(const int wg, const double *__restrict__ X, int a, int b, long long I,
                                                               const double *__restrict__ P, int p, long long sPr,
                                                               long long sPa, int tri, long long spw,
                                                               double *__restrict__ partials,
                                                               const double *__restrict__ fscale = nullptr) {
  using T = typename A::T;
  using V = typename A::V;
  // FP32 (fscale given): slices and P scaled by powers of two before the
  // rounding to FP32, the Gram scaled back at the end
  const double sM = (sizeof(T) == 4 && fscale) ? fscale[0] : 1.0;
  const double sF = (sizeof(T) == 4 && fscale) ? fscale[1] : 1.0;
  const double post = (sizeof(T) == 4 && fscale) ? fscale[2] : 1.0;
  // The product contracts over alpha, the fast index of a slice: its k-steps
  // run in pair order, so the slices are read with 16-byte loads straight
  // into the operand layout.
  constexpr int KP = (KS + 1) & ~1;   // k-steps over alpha (pair order covers 8 alpha per two steps)
  __shared__ T frag[NT * KP * 64];
  __shared__ double Gs[NT * 16 * NT * 16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  const int kpr = 2 * ((a + 7) / 8), ntp = (p + 15) / 16, ntb = (b + 15) / 16;  // GD: run-time extents
  const bool v2 = ((a & 1) == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
  build_afrag_pairs<T>(frag, P, p, a, sPr, sPa, NT, KP, sF);
  __syncthreads();
  V G[NT][NT];
#pragma unroll
  for (int u = 0; u < NT; ++u)
#pragma unroll
    for (int v = 0; v < NT; ++v) G[u][v] = V{0, 0, 0, 0};
  const long long beg = (long long)wg * spw;
  const long long end = std::min(beg + spw, I);
  const long long col = (long long)a * I;
  // register prefetch of the next slice (raw FP64 loads, rounded when the
  // slice becomes current) for FP32 and NT <= 2; FP64 at NT = 3 runs two waves
  // per SIMD instead
  constexpr bool PF = (NT <= 2) || sizeof(T) == 4;
  T cur[KP][NT];
  double nxt[PF ? KP : 1][NT];
  long long i = beg + wave;
  if constexpr (PF) {
    if (i < end) {
      if (v2) load_slice_pairs<NT, KP, true>(X + (long long)a * i, col, a, b, g, j, nxt);
      else load_slice_pairs<NT, KP, false>(X + (long long)a * i, col, a, b, g, j, nxt);
#pragma unroll
      for (int ks = 0; ks < KP; ++ks)
#pragma unroll
        for (int t = 0; t < NT; ++t) cur[ks][t] = (sizeof(T) == 4) ? (T)(nxt[ks][t] * sM) : (T)nxt[ks][t];
    }
  }
  for (; i < end; i += kWaves) {
    // NT = 4: keep the operand fragments in LDS rather than hoisted into
    // registers, which is what lets two waves share a SIMD
    if constexpr (NT == 4) __asm__ volatile("" ::: "memory");
    if constexpr (PF) {
      if (i + kWaves < end) {
        const double *Xn = X + (long long)a * (i + kWaves);
        if (v2) load_slice_pairs<NT, KP, true>(Xn, col, a, b, g, j, nxt);
        else load_slice_pairs<NT, KP, false>(Xn, col, a, b, g, j, nxt);
      }
    } else {
      if (v2) load_slice_pairs<NT, KP, true, T>(X + (long long)a * i, col, a, b, g, j, cur);
      else load_slice_pairs<NT, KP, false, T>(X + (long long)a * i, col, a, b, g, j, cur);
    }
    // one 16-row band of Y = P M at a time: its Gram contribution is
    // complete on its own, so only NT accumulator tiles of Y are live
#pragma unroll
    for (int rb = 0; rb < NT; ++rb) {
      if (GD && rb >= ntp) continue;
      V y[NT];  // Y(rho, beta), rho in band rb, one tile per beta-tile
#pragma unroll
      for (int t = 0; t < NT; ++t) y[t] = V{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < KP; ++ks) {
        // upper-triangular P: P(rho, alpha) = 0 for alpha < rho
        if ((tri && ks < 4 * rb) || (GD && ks >= kpr)) continue;
        const T pa = frag[(rb * KP + ks) * 64 + lane];
#pragma unroll
        for (int t = 0; t < NT; ++t)
          if (!GD || t < ntb) y[t] = A::mma(pa, cur[ks][t], y[t]);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (rb * 16 + A::row(0, r) >= p) continue;
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
          for (int v = 0; v <= u; ++v)
            if (!GD || u < ntb) G[u][v] = A::mma(y[u][r], y[v][r], G[u][v]);
      }
    }
    if constexpr (PF) {
#pragma unroll
      for (int ks = 0; ks < KP; ++ks)
#pragma unroll
        for (int t = 0; t < NT; ++t) cur[ks][t] = (sizeof(T) == 4) ? (T)(nxt[ks][t] * sM) : (T)nxt[ks][t];
    }
  }
  reduce_gram<NT, A>(G, NT, b, Gs, partials + (long long)wg * b * b, post);
}

template <int NT, int KS, class A>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(NT <= 3 || KS <= 14 ? 2 : 1, NT <= 3 || KS <= 14 ? 2 : 1))) void k_gram_left_factor(const double *__restrict__ X, int a, int b, long long I,
                                                               const double *__restrict__ P, int p, long long sPr,
                                                               long long sPa, int tri, long long spw,
                                                               double *__restrict__ partials,
                                                               const double *__restrict__ fscale) {
  gram_left_factor_body<NT, KS, A>(blockIdx.x, X, a, b, I, P, p, sPr, sPa, tri, spw, partials, fscale);
}

// ---------------------------------------------------------------------------
// One step of the inner-product recursion (§3.2.3, eq. (4)):
//   W_n (e x b) = sum_i Y_i^T (W_{n-1} X_i),
// X_i the a x b slices of X_n, Y_i the c x e slices of Y_n, W_{n-1} (c x a).
// Per slice and 16-row band of Z_i = W_{n-1} X_i (rows = c): the band's result
// registers are the B-operand fragments of the k-steps of Y_i^T Z_i over that
// band, and Y_i is read straight into the matching A-operand layout, so the two
// contractions chain with no LDS round trip.  KS = k-steps over a.
// ---------------------------------------------------------------------------
template <int NT>
__device__ void reduce_full(const d4 (&G)[NT][NT], int rows, int cols, double *Gs, double *out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  for (int e = threadIdx.x; e < rows * cols; e += blockDim.x) Gs[e] = 0.0;
  __syncthreads();
  for (int w = 0; w < kWaves; ++w) {
    if (wave == w) {
#pragma unroll
      for (int u = 0; u < NT; ++u)
#pragma unroll
        for (int v = 0; v < NT; ++v)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = u * 16 + F64::row(g, r), col = v * 16 + j;
            if (row < rows && col < cols) Gs[row + rows * col] += G[u][v][r];
          }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < rows * cols; e += blockDim.x) out[e] = Gs[e];
}

template <int NT, int KS>
__global__ __launch_bounds__(kThreads) void k_dot_mfma(const double *__restrict__ X, int a, int b,
                                                       const double *__restrict__ Y, int c, int e, long long I,
                                                       const double *__restrict__ W, long long spw,
                                                       double *__restrict__ partials) {
  constexpr int KP = (KS + 1) & ~1;  // k-steps over a in pair order
  __shared__ double frag[NT * KP * 64];
  __shared__ double Gs[NT * 16 * NT * 16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  const int ntb = (b + 15) / 16, nte = (e + 15) / 16, ntc = (c + 15) / 16;
  const bool v2 = ((a & 1) == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
  build_afrag_pairs<double>(frag, W, c, a, 1, c, NT, KP);
  __syncthreads();
  d4 acc[NT][NT];  // [e-tile][b-tile]
#pragma unroll
  for (int u = 0; u < NT; ++u)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[u][t] = d4{0, 0, 0, 0};
  const long long beg = (long long)blockIdx.x * spw;
  const long long end = std::min(beg + spw, I);
  const long long xcol = (long long)a * I, ycol = (long long)c * I;
  for (long long i = beg + wave; i < end; i += kWaves) {
    double xs[KP][NT];
    if (v2) load_slice_pairs<NT, KP, true>(X + (long long)a * i, xcol, a, b, g, j, xs);
    else load_slice_pairs<NT, KP, false>(X + (long long)a * i, xcol, a, b, g, j, xs);
    const double *Yi = Y + (long long)c * i;
#pragma unroll
    for (int rb = 0; rb < NT; ++rb) {
      if (rb >= ntc) continue;
      // the band's rows of Y_i, issued before the band's first product:
      // yb[r][u] = Y_i(16 rb + 4 r + g, 16 u + j)
      double yb[4][NT];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          const int cr = 16 * rb + 4 * r + g, ce = 16 * u + j;
          yb[r][u] = (cr < c && ce < e) ? Yi[cr + ycol * ce] : 0.0;
        }
      d4 z[NT];  // Z_i(16 rb + row(g, r), 16 t + j)
#pragma unroll
      for (int t = 0; t < NT; ++t) z[t] = d4{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < KP; ++ks) {
        if (8 * (ks >> 1) >= a) continue;
        const double wa = frag[(rb * KP + ks) * 64 + lane];
#pragma unroll
        for (int t = 0; t < NT; ++t)
          if (t < ntb) z[t] = mfma(wa, xs[ks][t], z[t]);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (rb * 16 + 4 * r >= c) continue;
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
          for (int t = 0; t < NT; ++t)
            if (u < nte && t < ntb) acc[u][t] = mfma(yb[r][u], z[t][r], acc[u][t]);
      }
    }
  }
  reduce_full<NT>(acc, e, b, Gs, partials + (long long)blockIdx.x * e * b);
}

// ---------------------------------------------------------------------------
// Output pass: Y_i = P M_i Q (p x q) written as a p x I x q core.  P == nullptr
// means the identity (p = a); Q == nullptr means the identity (q = b).
// KS = k-steps over b.  Two waves share each SIMD (NT <= 3, and NT = 4 at
// KS = 13), so one wave's loads and stores overlap the other's matrix-core
// work.
// ---------------------------------------------------------------------------
// Writes the tiles yt[u] of column band c of the transpose of an nrow x ncol
// block of one output slice: register r of yt[u] in lane (g, j) holds
// Y(16u + j, 16c + 4r + g).  The sixteen lanes of a lane group hold sixteen
// consecutive rows of one column, so every store leaves as 128-byte runs,
// with no staging.
template <int NT>
__device__ inline void store_t_band(const d4 (&yt)[NT], int c, int nrow, int ncol, double *__restrict__ Yi,
                                    long long ocol, int g, int j) {
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    const int row = 16 * u + j;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int cc = 16 * c + 4 * r + g;
      if (row < nrow && cc < ncol) Yi[row + ocol * cc] = yt[u][r];
    }
  }
}

// The output products are formed transposed, Y^T = (M Q)^T P^T (or Q^T M^T
// without P): swapping the operands of the last product turns the result
// registers into column runs (store_t_band).
template <int NT, int KS, bool GD = false>
__device__ __forceinline__ void apply_mfma_body(const int wg, const double *__restrict__ X, int a, int b, long long I, const double *__restrict__ P, int p,
                  long long sPr, long long sPa, const double *__restrict__ Q, int q, long long sQr, long long sQc,
                  int tri, long long spw, double *__restrict__ Y) {
  constexpr int KA = NT * 4;  // k-steps over alpha (whole tiles)
  __shared__ double fragQ[NT * KS * 64];
  __shared__ double fragP[NT * KA * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  const int ksr = (b + 3) / 4, nta = (a + 15) / 16, ntp = (p + 15) / 16;  // GD
  const bool hasP = (P != nullptr);
  const bool triQ = (tri & 1) != 0, triP = (tri & 2) != 0;
  build_bfrag(fragQ, Q, b, q, sQr, sQc, NT, KS);
  if (hasP) build_afrag(fragP, P, p, a, sPr, sPa, NT, KA);
  __syncthreads();
  const long long beg = (long long)wg * spw;
  const long long end = std::min(beg + spw, I);
  const long long col = (long long)a * I;
  const long long ocol = (long long)p * I;
  // register prefetch of the next slice where it fits without spilling (the
  // batched form keeps its registers for the run-time extents)
  constexpr bool PF = (NT <= 2 || (NT == 3 && KS <= 11)) && !GD;
  double cur[KS][NT];
  double nxt[PF ? KS : 1][NT];
  long long i = beg + wave;
  if constexpr (PF)
    if (i < end) load_slice<NT, KS, true>(X + (long long)a * i, col, a, b, g, j, cur);
  for (; i < end; i += kWaves) {
    if constexpr (PF) {
      if (i + kWaves < end) load_slice<NT, KS, true>(X + (long long)a * (i + kWaves), col, a, b, g, j, nxt);
    } else {
      load_slice<NT, KS, true>(X + (long long)a * i, col, a, b, g, j, cur);
    }
    double *Yi = Y + (long long)p * i;
    // one 16-column band of the output at a time: Y(:, band) = P M Q(:, band)
    // needs only that band of W = M Q, so few accumulator tiles are live and
    // the next slice's prefetch fits beside them
#pragma unroll
    for (int cb = 0; cb < NT; ++cb) {
      if (cb * 16 >= q) break;
      if (hasP) {
        d4 w[NT];  // W(alpha, c), c in band cb, one tile per alpha-tile
#pragma unroll
        for (int t = 0; t < NT; ++t) w[t] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          // lower-triangular Q: Q(beta, c) = 0 for beta < c, so k-steps below 4 cb vanish
          if ((triQ && ks < 4 * cb) || (GD && ks >= ksr)) continue;
          const double qb = fragQ[(cb * KS + ks) * 64 + lane];
#pragma unroll
          for (int t = 0; t < NT; ++t)
            if (!GD || t < nta) w[t] = mfma(cur[ks][t], qb, w[t]);
        }
        d4 yt[NT];  // Y^T tiles (c-band cb, rho-tile)
#pragma unroll
        for (int u = 0; u < NT; ++u) yt[u] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if (t * 16 + 4 * r >= a) continue;  // rows of W past a are padding
#pragma unroll
            for (int rb = 0; rb < NT; ++rb) {
              // upper-triangular P: P(rho, alpha) = 0 for alpha < rho
              if ((GD && rb >= ntp) || (triP && t < rb)) continue;
              const double pa = fragP[(rb * KA + t * 4 + r) * 64 + lane];
              yt[rb] = mfma(w[t][r], pa, yt[rb]);
            }
          }
        store_t_band<NT>(yt, cb, p, q, Yi, ocol, g, j);
      } else {
        d4 wt[NT];  // W^T tiles (c-band cb, alpha-tile)
#pragma unroll
        for (int t = 0; t < NT; ++t) wt[t] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          if ((triQ && ks < 4 * cb) || (GD && ks >= ksr)) continue;
          const double qb = fragQ[(cb * KS + ks) * 64 + lane];
#pragma unroll
          for (int t = 0; t < NT; ++t)
            if (!GD || t < nta) wt[t] = mfma(qb, cur[ks][t], wt[t]);
        }
        store_t_band<NT>(wt, cb, p, q, Yi, ocol, g, j);
      }
    }
    if constexpr (PF) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int t = 0; t < NT; ++t) cur[ks][t] = nxt[ks][t];
    }
  }
}

template <int NT, int KS>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(NT <= 3 || KS <= 13 ? 2 : 1, NT <= 3 || KS <= 13 ? 2 : 1))) void k_apply_mfma(const double *__restrict__ X, int a, int b, long long I, const double *__restrict__ P, int p,
                  long long sPr, long long sPa, const double *__restrict__ Q, int q, long long sQr, long long sQc,
                  int tri, long long spw, double *__restrict__ Y) {
  apply_mfma_body<NT, KS>(blockIdx.x, X, a, b, I, P, p, sPr, sPa, Q, q, sQr, sQc, tri, spw, Y);
}

// ---------------------------------------------------------------------------
// Refinement passes on a materialized core (truncation sweep, §2.4, when the
// first Gram pass could not settle the factorization).  The slice seen is
// S_i = M_i (TR = false, a x b) or M_i^T (TR = true, b x a); sa x sb below.
//
// k_gram_fac: G (q x q) = sum_i (S_i Q)^T (S_i Q), Q (sb x q).
// k_apply_fac2: Y_i = S_i Q1 Q2 (sa x q2), written as an sa x I x q2 core
//   (TR = false) or as its transpose q2 x I x sa (TR = true).
// The first product is W = S Q1 in k_gram_fac and W^T = Q1^T S^T in
// k_apply_fac2: the same operands with A and B exchanged, which the matrix
// cores round identically, so the output pass applies exactly the stage whose
// orthonormality the Gram pass measured.
// ---------------------------------------------------------------------------
template <int NT, int KS, bool TR, bool GD = false>
__device__ __forceinline__ void gram_fac_body(const int wg, const double *__restrict__ X, int a, int b, long long I,
                                                       const double *__restrict__ Q, int q, long long sQr,
                                                       long long sQc, int tri, long long spw,
                                                       double *__restrict__ partials) {
  // two waves per SIMD without a register prefetch (NT >= 3), as the Gram
  // kernels of the first passes; at NT = 4 only one 16-row band of the slice
  // is held at a time (BL), which is what fits two waves
  constexpr bool PF = (NT <= 2);
  constexpr bool BL = (NT >= 4);
  __shared__ double frag[NT * KS * 64];
  __shared__ double Gs[NT * 16 * NT * 16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  const int ksr = ((TR ? a : b) + 3) / 4, ntq = (q + 15) / 16;  // GD
  const int sa = TR ? b : a, sb = TR ? a : b;
  build_bfrag(frag, Q, sb, q, sQr, sQc, NT, KS);
  __syncthreads();
  d4 G[NT][NT];
#pragma unroll
  for (int u = 0; u < NT; ++u)
#pragma unroll
    for (int v = 0; v < NT; ++v) G[u][v] = d4{0.0, 0.0, 0.0, 0.0};
  const long long beg = (long long)wg * spw;
  const long long end = std::min(beg + spw, I);
  const long long col = (long long)a * I;
  // cur[ks][t] = S(16t + j, 4ks + g)
  double cur[BL ? 1 : KS][BL ? 1 : NT], nxt[PF ? KS : 1][NT];
  long long i = beg + wave;
  if constexpr (PF)
    if (i < end) load_slice<NT, KS, !TR>(X + (long long)a * i, col, a, b, g, j, cur);
  for (; i < end; i += kWaves) {
    if constexpr (PF) {
      if (i + kWaves < end)
        load_slice<NT, KS, !TR>(X + (long long)a * (i + kWaves), col, a, b, g, j, nxt);
    } else if constexpr (!BL) {
      load_slice<NT, KS, !TR>(X + (long long)a * i, col, a, b, g, j, cur);
    }
    // one 16-row band of W = S Q at a time: its Gram contribution is complete
    // on its own
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (t * 16 >= sa) break;
      double sv[KS];  // band t of the slice
      if constexpr (BL) {
        load_band<KS, !TR>(X + (long long)a * i, col, a, b, g, j, t, sv);
      } else {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) sv[ks] = cur[ks][t];
      }
      d4 w[NT];  // W(s, c), s in band t, one tile per c-tile
#pragma unroll
      for (int cb = 0; cb < NT; ++cb) w[cb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int cb = 0; cb < NT; ++cb) {
          if ((tri && ks < 4 * cb) || (GD && (ks >= ksr || cb >= ntq))) continue;  // lower-triangular Q
          w[cb] = mfma(sv[ks], frag[(cb * KS + ks) * 64 + lane], w[cb]);
        }
      // G(c, c') += sum_s W(s, c) W(s, c'); register r holds rows s = 16t + 4r + g;
      // rows past sa are padding
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (t * 16 + 4 * r >= sa) continue;
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
          for (int v = 0; v <= u; ++v)
            if (!GD || u < ntq) G[u][v] = mfma(w[u][r], w[v][r], G[u][v]);
      }
    }
    if constexpr (PF) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int t = 0; t < NT; ++t) cur[ks][t] = nxt[ks][t];
    }
  }
  reduce_gram<NT, F64>(G, NT, q, Gs, partials + (long long)wg * q * q);
}

template <int NT, int KS, bool TR>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(NT <= 3 || TR || KS <= 14 ? 2 : 1, NT <= 3 || TR || KS <= 14 ? 2 : 1))) void k_gram_fac(const double *__restrict__ X, int a, int b, long long I,
                                                       const double *__restrict__ Q, int q, long long sQr,
                                                       long long sQc, int tri, long long spw,
                                                       double *__restrict__ partials) {
  gram_fac_body<NT, KS, TR>(blockIdx.x, X, a, b, I, Q, q, sQr, sQc, tri, spw, partials);
}

template <int NT, int KS, bool TR, bool GD = false>
__device__ __forceinline__ void apply_fac2_body(const int wg, const double *__restrict__ X, int a, int b, long long I,
                                                         const double *__restrict__ Q1, int q1, long long s1r,
                                                         long long s1c, int tri, const double *__restrict__ Q2,
                                                         int q2, long long s2r, long long s2c, long long spw,
                                                         double *__restrict__ Y) {
  // register prefetch of the next slice where it fits without spilling; at
  // NT = 4 one 16-row band of the slice is held at a time (BL)
  constexpr bool PF = (NT <= 2 || (NT == 3 && (TR || KS <= 10))) && !GD;
  constexpr bool BL = (NT >= 4);
  constexpr int KC = NT * 4;  // k-steps over the columns of Q1 (whole tiles)
  __shared__ double frag1[NT * KS * 64];
  __shared__ double frag2[NT * KC * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  const int ksr = ((TR ? a : b) + 3) / 4, ntq1 = (q1 + 15) / 16, ntq2 = (q2 + 15) / 16;  // GD
  const int sa = TR ? b : a, sb = TR ? a : b;
  // A operands: Q1^T (q1 x sb) and Q2^T (q2 x q1)
  build_afrag(frag1, Q1, q1, sb, s1c, s1r, NT, KS);
  build_afrag(frag2, Q2, q2, q1, s2c, s2r, NT, KC);
  __syncthreads();
  const long long beg = (long long)wg * spw;
  const long long end = std::min(beg + spw, I);
  const long long col = (long long)a * I;
  // output addressing: element (s, c2) of slice i
  const long long ostep_s = TR ? (long long)q2 * I : 1;
  const long long ostep_c = TR ? 1 : (long long)sa * I;
  const long long oslice = TR ? q2 : sa;
  double cur[BL ? 1 : KS][BL ? 1 : NT], nxt[PF ? KS : 1][NT];
  long long i = beg + wave;
  if constexpr (PF)
    if (i < end) load_slice<NT, KS, !TR>(X + (long long)a * i, col, a, b, g, j, cur);
  for (; i < end; i += kWaves) {
    if constexpr (PF) {
      if (i + kWaves < end)
        load_slice<NT, KS, !TR>(X + (long long)a * (i + kWaves), col, a, b, g, j, nxt);
    } else if constexpr (!BL) {
      load_slice<NT, KS, !TR>(X + (long long)a * i, col, a, b, g, j, cur);
    }
    double *Yi = Y + oslice * i;
    // one 16-row band of S at a time (rows s of the output): few accumulator
    // tiles are live
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (t * 16 >= sa) break;
      double sv[KS];  // band t of the slice
      if constexpr (BL) {
        load_band<KS, !TR>(X + (long long)a * i, col, a, b, g, j, t, sv);
      } else {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) sv[ks] = cur[ks][t];
      }
      d4 wt[NT];  // W^T = Q1^T S^T tiles (c-tile, s-band t)
#pragma unroll
      for (int u = 0; u < NT; ++u) wt[u] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int cb = 0; cb < NT; ++cb) {
          if ((tri && ks < 4 * cb) || (GD && (ks >= ksr || cb >= ntq1))) continue;
          wt[cb] = mfma(frag1[(cb * KS + ks) * 64 + lane], sv[ks], wt[cb]);
        }
      d4 yt[NT];  // Y^T = Q2^T W^T tiles (c2-tile, s-band t)
#pragma unroll
      for (int u = 0; u < NT; ++u) yt[u] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int cb = 0; cb < NT; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (cb * 16 + 4 * r >= q1) continue;
#pragma unroll
          for (int u = 0; u < NT; ++u) {
            if (GD && u >= ntq2) continue;
            yt[u] = mfma(frag2[(u * KC + cb * 4 + r) * 64 + lane], wt[cb][r], yt[u]);
          }
        }
      const int sidx = t * 16 + j;
#pragma unroll
      for (int u = 0; u < NT; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int c2 = u * 16 + 4 * r + g;
          if (sidx < sa && c2 < q2) Yi[ostep_s * sidx + ostep_c * c2] = yt[u][r];
        }
    }
    if constexpr (PF) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int t = 0; t < NT; ++t) cur[ks][t] = nxt[ks][t];
    }
  }
}

template <int NT, int KS, bool TR>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_apply_fac2(const double *__restrict__ X, int a, int b, long long I,
                                                         const double *__restrict__ Q1, int q1, long long s1r,
                                                         long long s1c, int tri, const double *__restrict__ Q2,
                                                         int q2, long long s2r, long long s2c, long long spw,
                                                         double *__restrict__ Y) {
  apply_fac2_body<NT, KS, TR>(blockIdx.x, X, a, b, I, Q1, q1, s1r, s1c, tri, Q2, q2, s2r, s2c, spw, Y);
}

// ---------------------------------------------------------------------------
// Batched forms: the same bodies over a list of (TT, workgroup) items, with
// each TT's operands in a device descriptor.  KS = 4 NT covers every
// contracted dimension of the tile class (padding k-steps are zero).
// ---------------------------------------------------------------------------
#define TTR_ITEMS_LOOP(BODY)                                                   \
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {                    \
    const WGItem w = items[it];                                                \
    const BDesc &e = d[w.tt];                                                  \
    if (e.active && w.wg < e.nwg) { BODY; }                                    \
    __syncthreads();                                                           \
  }

template <int NT, class A>
__global__ __launch_bounds__(kThreads) void kb_gram_right_factor(const BDesc *__restrict__ d,
                                                                 const WGItem *__restrict__ items, int nitems) {
  TTR_ITEMS_LOOP((gram_right_factor_body<NT, 4 * NT, A, true>(w.wg, e.X, e.a, e.b, e.I, e.Q, e.q, e.sQr, e.sQc, e.tri,
                                                        e.spw, e.out)))
}
template <int NT, class A>
__global__ __launch_bounds__(kThreads) void kb_gram_left_factor(const BDesc *__restrict__ d,
                                                                const WGItem *__restrict__ items, int nitems) {
  TTR_ITEMS_LOOP((gram_left_factor_body<NT, 4 * NT, A, true>(w.wg, e.X, e.a, e.b, e.I, e.P, e.p, e.sPr, e.sPa, e.tri,
                                                       e.spw, e.out)))
}
template <int NT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(NT <= 3 ? 2 : 1, NT <= 3 ? 2 : 1)))
void kb_apply_mfma(const BDesc *__restrict__ d, const WGItem *__restrict__ items, int nitems) {
  TTR_ITEMS_LOOP((apply_mfma_body<NT, 4 * NT, true>(w.wg, e.X, e.a, e.b, e.I, e.P, e.p, e.sPr, e.sPa, e.Q, e.q, e.sQr,
                                              e.sQc, 0, e.spw, e.out)))
}
template <int NT, bool TR>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void kb_gram_fac(const BDesc *__restrict__ d, const WGItem *__restrict__ items,
                                                        int nitems) {
  TTR_ITEMS_LOOP((gram_fac_body<NT, 4 * NT, TR, true>(w.wg, e.X, e.a, e.b, e.I, e.Q, e.q, e.sQr, e.sQc, e.tri, e.spw,
                                                e.out)))
}
template <int NT, bool TR>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void kb_apply_fac2(const BDesc *__restrict__ d,
                                                          const WGItem *__restrict__ items, int nitems) {
  TTR_ITEMS_LOOP((apply_fac2_body<NT, 4 * NT, TR, true>(w.wg, e.X, e.a, e.b, e.I, e.Q, e.q, e.sQr, e.sQc, e.tri, e.Q2,
                                                  e.q2, e.s2r, e.s2c, e.spw, e.out)))
}

struct Grid {
  int nwg;
  long long spw;
};

// FP64 kernels run two workgroups per CU: 512 workgroups cover the 256 CUs
// once, and the fixed-order reduction that follows a Gram pass then reads half
// the partial Grams of TTR_MAXWG (measured faster for FP64; the FP32 Gram
// kernels keep TTR_MAXWG).
constexpr long long kWgF64 = 512;

Grid grid_of(long long I, long long cap = kWgF64) {
  // about 16 slices per wave at least, at most `cap` workgroups
  long long nwg = (I + 16 * kWaves - 1) / (16 * kWaves);
  nwg = std::max(1LL, std::min(nwg, std::min(cap, (long long)TTR_MAXWG)));
  long long spw = (I + nwg - 1) / nwg;
  Grid g;
  g.spw = std::max(1LL, spw);
  g.nwg = (int)((I + g.spw - 1) / g.spw);
  return g;
}

int tiles_for(int m) { return (m + 15) / 16; }

}  // namespace

// (NT, KS) dispatch: NT = 16-tiles covering every dimension, KS = k-steps of the
// contracted slice dimension, KS in {4NT-3, ..., 4NT}.  `f` receives both as
// std::integral_constant values.
template <int NTV, class F>
void ks_cases(int ks, F &&f) {
  switch (ks - (4 * NTV - 3)) {
    case 0: f(std::integral_constant<int, NTV>{}, std::integral_constant<int, 4 * NTV - 3>{}); break;
    case 1: f(std::integral_constant<int, NTV>{}, std::integral_constant<int, 4 * NTV - 2>{}); break;
    case 2: f(std::integral_constant<int, NTV>{}, std::integral_constant<int, 4 * NTV - 1>{}); break;
    default: f(std::integral_constant<int, NTV>{}, std::integral_constant<int, 4 * NTV>{}); break;
  }
}
template <class F>
void nt_ks(int nt, int ks, F &&f) {
  switch (nt) {
    case 1: ks_cases<1>(ks, f); break;
    case 2: ks_cases<2>(ks, f); break;
    case 3: ks_cases<3>(ks, f); break;
    default: ks_cases<4>(ks, f); break;
  }
}
#define TTR_LAUNCH(...) hipLaunchKernelGGL((__VA_ARGS__), dim3(gr.nwg), dim3(kThreads), 0, s,

namespace {
// Scales of an FP32 Gram pass, powers of two: out[0] = 2^-e for the largest
// finite |x| over up to 4096 evenly spaced samples of the n doubles at X
// (2^e <= max < 2^(e+1)), out[1] = 2^-f likewise for every entry of the small
// factor F (rows x cols <= 4096 entries, F(r, c) = F[r sr + c sc]; 1 when F
// is absent), and out[2] = 2^(2(e + f)), which undoes both in the Gram.  A
// zero maximum gives the scale 1.  Only the exponent matters (FP32's range
// leaves decades of room either side), so a sample suffices; each thread
// issues its 16 loads at once.
__global__ __launch_bounds__(256) void k_f32_scale(const double *__restrict__ X, long long n,
                                                   const double *__restrict__ F, int rows, int cols, long long sr,
                                                   long long sc, double *__restrict__ out) {
  __shared__ double red[2][256];
  constexpr int kPer = 16;
  const long long ns = std::min(n, 256LL * kPer);
  const long long stride = std::max(1LL, n / std::max(ns, 1LL));
  double mx = 0.0, mf = 0.0;
  double v[kPer], f[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const long long j = threadIdx.x + 256LL * q;
    v[q] = (j < ns) ? fabs(X[j * stride]) : 0.0;
    const int e = threadIdx.x + 256 * q;
    f[q] = (F && e < rows * cols) ? fabs(F[(long long)(e % rows) * sr + (long long)(e / rows) * sc]) : 0.0;
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    if (v[q] <= 1.7976931348623157e308) mx = fmax(mx, v[q]);
    if (f[q] <= 1.7976931348623157e308) mf = fmax(mf, f[q]);
  }
  red[0][threadIdx.x] = mx;
  red[1][threadIdx.x] = mf;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + off]);
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int e = (red[0][0] > 0.0) ? ilogb(red[0][0]) : 0;
    const int f = (red[1][0] > 0.0) ? ilogb(red[1][0]) : 0;
    out[0] = ldexp(1.0, -e);
    out[1] = ldexp(1.0, -f);
    out[2] = ldexp(1.0, 2 * (e + f));
  }
}
}  // namespace

int launch_gram_right_factor(hipStream_t s, const double *X, int a, int b, long long I, const double *Q, int q,
                             long long sQr, long long sQc, int tri, int f32, double *partials, double *fscale) {
  const Grid gr = grid_of(I, f32 ? TTR_MAXWG : kWgF64);
  if (f32 && fscale)
    hipLaunchKernelGGL(k_f32_scale, dim3(1), dim3(256), 0, s, X, (long long)a * I * b, Q, Q ? b : 0, Q ? q : 0, sQr,
                       sQc, fscale);
  else
    fscale = nullptr;
  const int nt = std::max({tiles_for(a), tiles_for(b), tiles_for(q)});
  const int ks = std::max((b + 3) / 4, 4 * nt - 3);
  nt_ks(nt, ks, [&](auto NTc, auto KSc) {
    constexpr int NTV = decltype(NTc)::value, KSV = decltype(KSc)::value;
    if (f32)
      TTR_LAUNCH(k_gram_right_factor<NTV, KSV, F32>) X, a, b, I, Q, q, sQr, sQc, tri, gr.spw, partials, fscale);
    else
      TTR_LAUNCH(k_gram_right_factor<NTV, KSV, F64>) X, a, b, I, Q, q, sQr, sQc, tri, gr.spw, partials, nullptr);
  });
  return gr.nwg;
}

int launch_gram_left_factor(hipStream_t s, const double *X, int a, int b, long long I, const double *P, int p,
                            long long sPr, long long sPa, int tri, int f32, double *partials, double *fscale) {
  const Grid gr = grid_of(I, f32 ? TTR_MAXWG : kWgF64);
  if (f32 && fscale)
    hipLaunchKernelGGL(k_f32_scale, dim3(1), dim3(256), 0, s, X, (long long)a * I * b, P, P ? p : 0, P ? a : 0, sPr,
                       sPa, fscale);
  else
    fscale = nullptr;
  const int nt = std::max({tiles_for(a), tiles_for(b), tiles_for(p)});
  const int ks = std::max((a + 3) / 4, 4 * nt - 3);
  nt_ks(nt, ks, [&](auto NTc, auto KSc) {
    constexpr int NTV = decltype(NTc)::value, KSV = decltype(KSc)::value;
    if (f32)
      TTR_LAUNCH(k_gram_left_factor<NTV, KSV, F32>) X, a, b, I, P, p, sPr, sPa, tri, gr.spw, partials, fscale);
    else
      TTR_LAUNCH(k_gram_left_factor<NTV, KSV, F64>) X, a, b, I, P, p, sPr, sPa, tri, gr.spw, partials, nullptr);
  });
  return gr.nwg;
}

int dot_mfma_workgroups(long long I) { return grid_of(I).nwg; }

int launch_dot_mfma(hipStream_t s, const double *X, int a, int b, const double *Y, int c, int e, long long I,
                    const double *W, double *partials) {
  const Grid gr = grid_of(I);
  const int nt = std::max({tiles_for(a), tiles_for(b), tiles_for(c), tiles_for(e)});
  const int ks = std::max((a + 3) / 4, 4 * nt - 3);
  nt_ks(nt, ks, [&](auto NTc, auto KSc) {
    constexpr int NTV = decltype(NTc)::value, KSV = decltype(KSc)::value;
    TTR_LAUNCH(k_dot_mfma<NTV, KSV>) X, a, b, Y, c, e, I, W, gr.spw, partials);
  });
  return gr.nwg;
}

void launch_apply_mfma(hipStream_t s, const double *X, int a, int b, long long I, const double *P, int p,
                       long long sPr, long long sPa, const double *Q, int q, long long sQr, long long sQc, int tri,
                       double *Y) {
  const Grid gr = grid_of(I);
  const int nt = std::max({tiles_for(a), tiles_for(b), tiles_for(p), tiles_for(q)});
  const int ks = std::max((b + 3) / 4, 4 * nt - 3);
  nt_ks(nt, ks, [&](auto NTc, auto KSc) {
    constexpr int NTV = decltype(NTc)::value, KSV = decltype(KSc)::value;
    TTR_LAUNCH(k_apply_mfma<NTV, KSV>) X, a, b, I, P, p, sPr, sPa, Q, q, sQr, sQc, tri, gr.spw, Y);
  });
}

int launch_gram_fac(hipStream_t s, const double *X, int a, int b, long long I, int trans, const double *Q, int q,
                    long long sQr, long long sQc, int tri, double *partials) {
  const Grid gr = grid_of(I);
  const int sb = trans ? a : b;
  const int nt = std::max({tiles_for(a), tiles_for(b), tiles_for(q)});
  const int ks = std::max((sb + 3) / 4, 4 * nt - 3);
  nt_ks(nt, ks, [&](auto NTc, auto KSc) {
    constexpr int NTV = decltype(NTc)::value, KSV = decltype(KSc)::value;
    if (trans)
      TTR_LAUNCH(k_gram_fac<NTV, KSV, true>) X, a, b, I, Q, q, sQr, sQc, tri, gr.spw, partials);
    else
      TTR_LAUNCH(k_gram_fac<NTV, KSV, false>) X, a, b, I, Q, q, sQr, sQc, tri, gr.spw, partials);
  });
  return gr.nwg;
}

void launch_apply_fac2(hipStream_t s, const double *X, int a, int b, long long I, int trans, const double *Q1,
                       int q1, long long s1r, long long s1c, int tri, const double *Q2, int q2, long long s2r,
                       long long s2c, double *Y) {
  const Grid gr = grid_of(I);
  const int sb = trans ? a : b;
  const int nt = std::max({tiles_for(a), tiles_for(b), tiles_for(q1), tiles_for(q2)});
  const int ks = std::max((sb + 3) / 4, 4 * nt - 3);
  nt_ks(nt, ks, [&](auto NTc, auto KSc) {
    constexpr int NTV = decltype(NTc)::value, KSV = decltype(KSc)::value;
    if (trans)
      TTR_LAUNCH(k_apply_fac2<NTV, KSV, true>) X, a, b, I, Q1, q1, s1r, s1c, tri, Q2, q2, s2r, s2c, gr.spw, Y);
    else
      TTR_LAUNCH(k_apply_fac2<NTV, KSV, false>) X, a, b, I, Q1, q1, s1r, s1c, tri, Q2, q2, s2r, s2c, gr.spw, Y);
  });
}

// --- batched launchers ------------------------------------------------------
template <class F>
void nt_only(int nt, F &&f) {
  switch (nt) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    default: f(std::integral_constant<int, 4>{}); break;
  }
}
#define TTR_BLAUNCH(...) hipLaunchKernelGGL((__VA_ARGS__), dim3(grid), dim3(kThreads), 0, s, d, items, nitems)

void launch_gram_right_factor_batched(hipStream_t s, int nt, int f32, const BDesc *d, const WGItem *items, int nitems,
                                      int grid) {
  if (nitems <= 0) return;
  nt_only(nt, [&](auto NTc) {
    constexpr int NTV = decltype(NTc)::value;
    if (f32) TTR_BLAUNCH(kb_gram_right_factor<NTV, F32>);
    else TTR_BLAUNCH(kb_gram_right_factor<NTV, F64>);
  });
}
void launch_gram_left_factor_batched(hipStream_t s, int nt, int f32, const BDesc *d, const WGItem *items, int nitems,
                                     int grid) {
  if (nitems <= 0) return;
  nt_only(nt, [&](auto NTc) {
    constexpr int NTV = decltype(NTc)::value;
    if (f32) TTR_BLAUNCH(kb_gram_left_factor<NTV, F32>);
    else TTR_BLAUNCH(kb_gram_left_factor<NTV, F64>);
  });
}
void launch_apply_mfma_batched(hipStream_t s, int nt, const BDesc *d, const WGItem *items, int nitems, int grid) {
  if (nitems <= 0) return;
  nt_only(nt, [&](auto NTc) {
    constexpr int NTV = decltype(NTc)::value;
    TTR_BLAUNCH(kb_apply_mfma<NTV>);
  });
}
void launch_gram_fac_batched(hipStream_t s, int nt, int trans, const BDesc *d, const WGItem *items, int nitems,
                             int grid) {
  if (nitems <= 0) return;
  nt_only(nt, [&](auto NTc) {
    constexpr int NTV = decltype(NTc)::value;
    if (trans) TTR_BLAUNCH(kb_gram_fac<NTV, true>);
    else TTR_BLAUNCH(kb_gram_fac<NTV, false>);
  });
}
void launch_apply_fac2_batched(hipStream_t s, int nt, int trans, const BDesc *d, const WGItem *items, int nitems,
                               int grid) {
  if (nitems <= 0) return;
  nt_only(nt, [&](auto NTc) {
    constexpr int NTV = decltype(NTc)::value;
    if (trans) TTR_BLAUNCH(kb_apply_fac2<NTV, true>);
    else TTR_BLAUNCH(kb_apply_fac2<NTV, false>);
  });
}
