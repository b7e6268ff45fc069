// FP64 matrix-core (MFMA) streaming kernels for the first Gram pass of each
// QR-by-Gram factorization and for the output pass, on cores stored in the
// paper's layout (§3.1): entry (a, i, b) of an R0 x I x R1 core at
// a + R0*(i + I*b).
//
// v_mfma_f64_16x16x4f64 on gfx950: lane l supplies A[l%16][k0 + l/16] and
// B[k0 + l/16][l%16]; the 16x16 result sits in four registers per lane with
// register r of lane l holding D[4r + l/16][l%16].  Register r of a result tile
// is therefore exactly the operand fragment of k-step 4r..4r+3 for a product
// that contracts over the tile's row index, so the chains below
//   Gram, right factor:  Wt = Q^T M^T,  G  += Wt^T Wt   (contract over c)
//   Gram, left factor:   Y  = P M,      G0 += Y^T Y     (contract over rho)
//   output:              W  = M Q,      Y   = P W       (contract over alpha)
// feed one product's accumulators straight into the next, without LDS.
// The small factors (<= 64 x 64) sit in LDS pre-arranged as per-lane
// fragments; slices are read from HBM once, 16 consecutive rows per lane
// group where the layout allows.
//
// Each workgroup (4 waves) owns a contiguous range of slices; the waves take
// slices round-robin, keep their own partial Gram in registers, and combine
// them in LDS in a fixed order, so results are reproducible run to run.
#include "ttr_internal.h"

#include <algorithm>

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kWaves = 4;

__device__ inline d4 mfma(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// A-operand fragments of S (rows x cols): frag[(t*KS + ks)*64 + l] = S(t*16 + l%16, ks*4 + l/16).
// S(r, c) = S[r*sr + c*sc]; S == nullptr means the identity.  Zero outside.
__device__ void build_afrag(double *frag, const double *S, int rows, int cols, long long sr, long long sc, int nt,
                            int KS) {
  const int total = nt * KS * 64;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int l = e & 63;
    const int ks = (e >> 6) % KS;
    const int t = (e >> 6) / KS;
    const int r = t * 16 + (l & 15);
    const int c = ks * 4 + (l >> 4);
    double v = 0.0;
    if (r < rows && c < cols) v = S ? S[r * sr + c * sc] : (r == c ? 1.0 : 0.0);
    frag[e] = v;
  }
}

// B-operand fragments of S (rows x cols): frag[(t*KS + ks)*64 + l] = S(ks*4 + l/16, t*16 + l%16).
__device__ void build_bfrag(double *frag, const double *S, int rows, int cols, long long sr, long long sc, int nt,
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
    frag[e] = v;
  }
}

// Adds this wave's Gram tiles (lower block triangle, tile (u, v) with u >= v)
// into the workgroup's dense gd x gd matrix in LDS, waves in a fixed order.
template <int NT>
__device__ void reduce_gram(const d4 (&G)[NT][NT], int nt, int gd, double *Gs, double *out) {
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
              const int row = u * 16 + g + 4 * r;
              const int col = v * 16 + j;
              if (row < gd && col < gd && row >= col) Gs[row + gd * col] += G[u][v][r];
            }
          }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < gd * gd; e += blockDim.x) {
    const int row = e % gd, col = e / gd;
    out[e] = (row >= col) ? Gs[row + gd * col] : Gs[col + gd * row];
  }
}

// Loads the operand fragments of one slice: buf[ks][t] = M(t*16 + l%16, ks*4 + l/16)
// (ROWS16 = true) or M(ks*4 + l/16, t*16 + l%16) (ROWS16 = false), zero outside
// the a x b slice.  M(alpha, beta) = Xi[alpha + col*beta].
template <int NT, int KS, bool ROWS16>
__device__ inline void load_slice(const double *__restrict__ Xi, long long col, int a, int b, int g, int j,
                                  double (&buf)[KS][NT]) {
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int r = ROWS16 ? t * 16 + j : ks * 4 + g;   // alpha
      const int c = ROWS16 ? ks * 4 + g : t * 16 + j;   // beta
      double v = 0.0;
      if (r < a && c < b) v = Xi[r + col * c];
      buf[ks][t] = v;
    }
}

// ---------------------------------------------------------------------------
// Gram with a right factor: G (a x a) = sum_i (M_i Q)(M_i Q)^T, M_i = X(:, i, :)
// (a x b), Q (b x q).  The left Gram of the horizontal unfolding of X x_3 Q^T
// (orthonormalization sweep, §2.3 / Alg. 1).  NT = 16-tiles per dimension,
// KS = k-steps over b (ceil(b/4)).
// ---------------------------------------------------------------------------
template <int NT, int KS>
__global__ __launch_bounds__(kThreads) void k_gram_right_factor(const double *__restrict__ X, int a, int b, long long I,
                                                                const double *__restrict__ Q, int q, long long sQr,
                                                                long long sQc, int tri, long long spw,
                                                                double *__restrict__ partials) {
  __shared__ double frag[NT * KS * 64];
  __shared__ double Gs[NT * 16 * NT * 16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  // A operand: Q^T (q x b), Q^T(c, beta) = Q(beta, c)
  build_afrag(frag, Q, q, b, sQc, sQr, NT, KS);
  __syncthreads();
  d4 G[NT][NT];
#pragma unroll
  for (int u = 0; u < NT; ++u)
#pragma unroll
    for (int v = 0; v < NT; ++v) G[u][v] = d4{0.0, 0.0, 0.0, 0.0};
  const long long beg = (long long)blockIdx.x * spw;
  const long long end = std::min(beg + spw, I);
  const long long col = (long long)a * I;
  double cur[KS][NT], nxt[KS][NT];
  long long i = beg + wave;
  if (i < end) load_slice<NT, KS, true>(X + (long long)a * i, col, a, b, g, j, cur);
  for (; i < end; i += kWaves) {
    if (i + kWaves < end) load_slice<NT, KS, true>(X + (long long)a * (i + kWaves), col, a, b, g, j, nxt);
    d4 wt[NT][NT];  // [c-tile][alpha-tile]
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
      for (int v = 0; v < NT; ++v) wt[u][v] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int cb = 0; cb < NT; ++cb) {
        // lower-triangular Q: Q^T(c, beta) = 0 for beta < c, so k-steps below 4 cb vanish
        if (tri && ks < 4 * cb) continue;
        const double qa = frag[(cb * KS + ks) * 64 + lane];
#pragma unroll
        for (int t = 0; t < NT; ++t) wt[cb][t] = mfma(qa, cur[ks][t], wt[cb][t]);
      }
    // G(alpha, alpha') += sum_c Wt(c, alpha) Wt(c, alpha'); consecutive MFMAs
    // go to different G tiles; k-steps past q are zero padding
#pragma unroll
    for (int cb = 0; cb < NT; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (cb * 16 + 4 * r >= q) continue;
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
          for (int v = 0; v <= u; ++v) G[u][v] = mfma(wt[cb][u][r], wt[cb][v][r], G[u][v]);
      }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int t = 0; t < NT; ++t) cur[ks][t] = nxt[ks][t];
  }
  reduce_gram<NT>(G, NT, a, Gs, partials + (long long)blockIdx.x * a * a);
}

// ---------------------------------------------------------------------------
// Gram with a left factor: G0 (b x b) = sum_i (P M_i)^T (P M_i), P (p x a).
// The Gram of the vertical unfolding of P x_1 X (truncation sweep, §2.4).
// KS = k-steps over a (ceil(a/4)).
// ---------------------------------------------------------------------------
template <int NT, int KS>
__global__ __launch_bounds__(kThreads) void k_gram_left_factor(const double *__restrict__ X, int a, int b, long long I,
                                                               const double *__restrict__ P, int p, long long sPr,
                                                               long long sPa, int tri, long long spw,
                                                               double *__restrict__ partials) {
  __shared__ double frag[NT * KS * 64];
  __shared__ double Gs[NT * 16 * NT * 16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  build_afrag(frag, P, p, a, sPr, sPa, NT, KS);
  __syncthreads();
  d4 G[NT][NT];
#pragma unroll
  for (int u = 0; u < NT; ++u)
#pragma unroll
    for (int v = 0; v < NT; ++v) G[u][v] = d4{0.0, 0.0, 0.0, 0.0};
  const long long beg = (long long)blockIdx.x * spw;
  const long long end = std::min(beg + spw, I);
  const long long col = (long long)a * I;
  double cur[KS][NT], nxt[KS][NT];
  long long i = beg + wave;
  if (i < end) load_slice<NT, KS, false>(X + (long long)a * i, col, a, b, g, j, cur);
  for (; i < end; i += kWaves) {
    if (i + kWaves < end) load_slice<NT, KS, false>(X + (long long)a * (i + kWaves), col, a, b, g, j, nxt);
    d4 y[NT][NT];  // [rho-tile][beta-tile]
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
      for (int v = 0; v < NT; ++v) y[u][v] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int rb = 0; rb < NT; ++rb) {
        // upper-triangular P: P(rho, alpha) = 0 for alpha < rho
        if (tri && ks < 4 * rb) continue;
        const double pa = frag[(rb * KS + ks) * 64 + lane];
#pragma unroll
        for (int t = 0; t < NT; ++t) y[rb][t] = mfma(pa, cur[ks][t], y[rb][t]);
      }
    // G0(beta, beta') += sum_rho Y(rho, beta) Y(rho, beta'); rows past p are padding
#pragma unroll
    for (int rb = 0; rb < NT; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (rb * 16 + 4 * r >= p) continue;
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
          for (int v = 0; v <= u; ++v) G[u][v] = mfma(y[rb][u][r], y[rb][v][r], G[u][v]);
      }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int t = 0; t < NT; ++t) cur[ks][t] = nxt[ks][t];
  }
  reduce_gram<NT>(G, NT, b, Gs, partials + (long long)blockIdx.x * b * b);
}

// ---------------------------------------------------------------------------
// Output pass: Y_i = P M_i Q (p x q) written as a p x I x q core.  P == nullptr
// means the identity (p = a); Q == nullptr means the identity (q = b).
// KS = k-steps over b.
// ---------------------------------------------------------------------------
template <int NT, int KS>
__global__ __launch_bounds__(kThreads) void k_apply_mfma(const double *__restrict__ X, int a, int b, long long I,
                                                         const double *__restrict__ P, int p, long long sPr,
                                                         long long sPa, const double *__restrict__ Q, int q,
                                                         long long sQr, long long sQc, long long spw,
                                                         double *__restrict__ Y) {
  constexpr int KA = NT * 4;  // k-steps over alpha (whole tiles)
  // per-wave staging of one output slice (NT <= 3): the tile registers are
  // written to LDS and each output column leaves as one contiguous run
  constexpr bool kStage = (NT <= 3);
  constexpr int LD = NT * 16 + 1;
  __shared__ double fragQ[NT * KS * 64];
  __shared__ double fragP[NT * KA * 64];
  __shared__ double Ys[kStage ? kWaves * LD * NT * 16 : 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double *Yw = Ys + (kStage ? wave * LD * NT * 16 : 0);
  const int g = lane >> 4, j = lane & 15;
  const bool hasP = (P != nullptr);
  build_bfrag(fragQ, Q, b, q, sQr, sQc, NT, KS);
  if (hasP) build_afrag(fragP, P, p, a, sPr, sPa, NT, KA);
  __syncthreads();
  const long long beg = (long long)blockIdx.x * spw;
  const long long end = std::min(beg + spw, I);
  const long long col = (long long)a * I;
  const long long ocol = (long long)p * I;
  double cur[KS][NT], nxt[KS][NT];
  long long i = beg + wave;
  if (i < end) load_slice<NT, KS, true>(X + (long long)a * i, col, a, b, g, j, cur);
  for (; i < end; i += kWaves) {
    if (i + kWaves < end) load_slice<NT, KS, true>(X + (long long)a * (i + kWaves), col, a, b, g, j, nxt);
    d4 w[NT][NT];  // [alpha-tile][c-tile]
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
      for (int v = 0; v < NT; ++v) w[u][v] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int cb = 0; cb < NT; ++cb) {
        const double qb = fragQ[(cb * KS + ks) * 64 + lane];
#pragma unroll
        for (int t = 0; t < NT; ++t) w[t][cb] = mfma(cur[ks][t], qb, w[t][cb]);
      }
    double *Yi = Y + (long long)p * i;
    if (hasP) {
      d4 y[NT][NT];  // [rho-tile][c-tile]
#pragma unroll
      for (int u = 0; u < NT; ++u)
#pragma unroll
        for (int v = 0; v < NT; ++v) y[u][v] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (t * 16 + 4 * r >= a) continue;  // rows of W past a are padding
#pragma unroll
          for (int rb = 0; rb < NT; ++rb) {
            const double pa = fragP[(rb * KA + t * 4 + r) * 64 + lane];
#pragma unroll
            for (int cb = 0; cb < NT; ++cb) y[rb][cb] = mfma(pa, w[t][cb][r], y[rb][cb]);
          }
        }
      if (kStage) {
#pragma unroll
        for (int rb = 0; rb < NT; ++rb)
#pragma unroll
          for (int cb = 0; cb < NT; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) Yw[(rb * 16 + g + 4 * r) + LD * (cb * 16 + j)] = y[rb][cb][r];
      } else {
#pragma unroll
        for (int rb = 0; rb < NT; ++rb)
#pragma unroll
          for (int cb = 0; cb < NT; ++cb) {
            const int c = cb * 16 + j;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int rho = rb * 16 + g + 4 * r;
              if (rho < p && c < q) Yi[rho + ocol * c] = y[rb][cb][r];
            }
          }
      }
    } else {
      if (kStage) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int cb = 0; cb < NT; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) Yw[(t * 16 + g + 4 * r) + LD * (cb * 16 + j)] = w[t][cb][r];
      } else {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int cb = 0; cb < NT; ++cb) {
            const int c = cb * 16 + j;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int alpha = t * 16 + g + 4 * r;
              if (alpha < p && c < q) Yi[alpha + ocol * c] = w[t][cb][r];
            }
          }
      }
    }
    if (kStage) {
      // the wave's LDS writes complete before its reads (same wave, in order)
      __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      int rho = lane, c = 0;
      while (rho >= p) {
        rho -= p;
        ++c;
      }
      for (; c < q;) {
        Yi[rho + ocol * c] = Yw[rho + LD * c];
        rho += 64;
        while (rho >= p) {
          rho -= p;
          ++c;
        }
      }
      __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int t = 0; t < NT; ++t) cur[ks][t] = nxt[ks][t];
  }
}

struct Grid {
  int nwg;
  long long spw;
};

Grid grid_of(long long I) {
  // about 16 slices per wave at least, at most TTR_MAXWG workgroups
  long long nwg = (I + 16 * kWaves - 1) / (16 * kWaves);
  nwg = std::max(1LL, std::min(nwg, (long long)TTR_MAXWG));
  long long spw = (I + nwg - 1) / nwg;
  Grid g;
  g.spw = std::max(1LL, spw);
  g.nwg = (int)((I + g.spw - 1) / g.spw);
  return g;
}

int tiles_for(int m) { return (m + 15) / 16; }

}  // namespace

// (NT, KS) dispatch: NT = 16-tiles covering every dimension, KS = k-steps of the
// contracted slice dimension, KS in {4NT-3, ..., 4NT}.
#define TTR_KS_CASES(KERNEL, NTV, ...)                                                                  \
  switch (ks - (4 * NTV - 3)) {                                                                        \
    case 0: hipLaunchKernelGGL((KERNEL<NTV, 4 * NTV - 3>), dim3(gr.nwg), dim3(kThreads), 0, s, __VA_ARGS__); break; \
    case 1: hipLaunchKernelGGL((KERNEL<NTV, 4 * NTV - 2>), dim3(gr.nwg), dim3(kThreads), 0, s, __VA_ARGS__); break; \
    case 2: hipLaunchKernelGGL((KERNEL<NTV, 4 * NTV - 1>), dim3(gr.nwg), dim3(kThreads), 0, s, __VA_ARGS__); break; \
    default: hipLaunchKernelGGL((KERNEL<NTV, 4 * NTV>), dim3(gr.nwg), dim3(kThreads), 0, s, __VA_ARGS__); break;    \
  }
#define TTR_NT_CASES(KERNEL, ...)                       \
  switch (nt) {                                          \
    case 1: TTR_KS_CASES(KERNEL, 1, __VA_ARGS__) break;  \
    case 2: TTR_KS_CASES(KERNEL, 2, __VA_ARGS__) break;  \
    case 3: TTR_KS_CASES(KERNEL, 3, __VA_ARGS__) break;  \
    default: TTR_KS_CASES(KERNEL, 4, __VA_ARGS__) break; \
  }

int launch_gram_right_factor(hipStream_t s, const double *X, int a, int b, long long I, const double *Q, int q,
                             long long sQr, long long sQc, int tri, double *partials) {
  const Grid gr = grid_of(I);
  const int nt = std::max({tiles_for(a), tiles_for(b), tiles_for(q)});
  const int ks = std::max((b + 3) / 4, 4 * nt - 3);
  TTR_NT_CASES(k_gram_right_factor, X, a, b, I, Q, q, sQr, sQc, tri, gr.spw, partials)
  return gr.nwg;
}

int launch_gram_left_factor(hipStream_t s, const double *X, int a, int b, long long I, const double *P, int p,
                            long long sPr, long long sPa, int tri, double *partials) {
  const Grid gr = grid_of(I);
  const int nt = std::max({tiles_for(a), tiles_for(b), tiles_for(p)});
  const int ks = std::max((a + 3) / 4, 4 * nt - 3);
  TTR_NT_CASES(k_gram_left_factor, X, a, b, I, P, p, sPr, sPa, tri, gr.spw, partials)
  return gr.nwg;
}

void launch_apply_mfma(hipStream_t s, const double *X, int a, int b, long long I, const double *P, int p,
                       long long sPr, long long sPa, const double *Q, int q, long long sQr, long long sQc,
                       double *Y) {
  const Grid gr = grid_of(I);
  const int nt = std::max({tiles_for(a), tiles_for(b), tiles_for(p), tiles_for(q)});
  const int ks = std::max((b + 3) / 4, 4 * nt - 3);
  TTR_NT_CASES(k_apply_mfma, X, a, b, I, P, p, sPr, sPa, Q, q, sQr, sQc, gr.spw, Y)
}
