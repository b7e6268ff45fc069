// Streaming kernels over TT cores: sum (§3.2.1), Hadamard product (§3.2.2),
// Gram passes of the tall-skinny unfoldings used by orthonormalization and
// rounding (§2.3, §2.4, §3.4, §3.5), core x small-matrix application, and the
// inner-product recursion (§3.2.3, eq. (4)).
//
// Core layout (§3.1): entry (a, i, b) of an R0 x I x R1 core at a + R0*(i + I*b).
// For a fixed b the slices i0..i0+T-1 occupy R0*T contiguous doubles, so a chunk
// of T slices is read as R1 coalesced panels and staged in LDS.
#include "ttr_internal.h"

#include <cstdint>

#include <algorithm>

namespace {

constexpr int kThreads = 256;
constexpr size_t kLdsBudget = 60 * 1024;  // bytes of dynamic LDS per workgroup

// ---------------------------------------------------------------------------
// Sum: output column b of core n (blockIdx.y) is zr0*I contiguous doubles;
// thread e of the column holds entry (a, i) = (e mod zr0, e div zr0).  The X
// block comes first (§3.2.1); off-diagonal blocks are explicit zeros.
// ---------------------------------------------------------------------------
__global__ void k_add(int n, int N, double alpha, double beta, const double *__restrict__ X, int rx0, int rx1,
                      const double *__restrict__ Y, int ry0, int ry1, int I, double *__restrict__ Z) {
#pragma clang fp contract(off)
  int zr0;
  if (N == 1 || n == 0) zr0 = 1;
  else zr0 = rx0 + ry0;
  const int b = blockIdx.y;
  const int colsz = zr0 * I;
  const long long zoff = (long long)colsz * b;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < colsz; e += gridDim.x * blockDim.x) {
    const int i = e / zr0;
    const int a = e - i * zr0;
    double v;
    if (N == 1) {
      // each product rounded on its own, as in the plain definition (no FMA)
      const double ax = alpha * X[i];
      const double by = beta * Y[i];
      v = ax + by;
    } else if (n == 0) {
      v = (b < rx1) ? alpha * X[i + (long long)I * b] : beta * Y[i + (long long)I * (b - rx1)];
    } else if (n == N - 1) {
      v = (a < rx0) ? X[a + rx0 * (long long)i] : Y[(a - rx0) + ry0 * (long long)i];
    } else if (a < rx0 && b < rx1) {
      v = X[a + (long long)rx0 * (i + (long long)I * b)];
    } else if (a >= rx0 && b >= rx1) {
      v = Y[(a - rx0) + (long long)ry0 * (i + (long long)I * (b - rx1))];
    } else {
      v = 0.0;
    }
    Z[zoff + e] = v;
  }
}

// The same sum for even ranks (and even I on the first core) and 16-byte
// aligned cores, two consecutive rows at a time with 16-byte loads and
// stores.  A pair never
// straddles the X / Y / zero blocks because the block sizes are even.  The
// row/slice split of the pair index uses a float reciprocal with an exact
// integer correction (pair counts per column stay below 2^24).
__global__ void k_add_pairs(int n, int N, double alpha, double beta, const double *__restrict__ X, int rx0, int rx1,
                            const double *__restrict__ Y, int ry0, int ry1, int I, double *__restrict__ Z) {
#pragma clang fp contract(off)
  typedef double d2 __attribute__((ext_vector_type(2)));
  const int zr0 = (n == 0) ? 1 : rx0 + ry0;
  const int b = blockIdx.y;
  const int npair = (zr0 * I) / 2;
  const int hr = zr0 / 2;  // pairs per slice column (0 on the first core: pairs run along i)
  const float inv = (n == 0) ? 0.f : 1.0f / (float)hr;
  d2 *Zb = reinterpret_cast<d2 *>(Z + (long long)zr0 * I * b);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < npair; e += gridDim.x * blockDim.x) {
    d2 v;
    if (n == 0) {
      // first core (1 x I x (rx1 + ry1)): column b is alpha X(0, :, b) or beta Y(0, :, b - rx1)
      const int i = 2 * e;
      if (b < rx1) {
        const d2 x = *reinterpret_cast<const d2 *>(X + i + (long long)I * b);
        v = d2{alpha * x.x, alpha * x.y};
      } else {
        const d2 y = *reinterpret_cast<const d2 *>(Y + i + (long long)I * (b - rx1));
        v = d2{beta * y.x, beta * y.y};
      }
    } else {
      int i = (int)((float)e * inv);
      int a2 = e - i * hr;
      while (a2 < 0) {
        --i;
        a2 += hr;
      }
      while (a2 >= hr) {
        ++i;
        a2 -= hr;
      }
      const int a = 2 * a2;
      if (n == N - 1) {
        v = (a < rx0) ? *reinterpret_cast<const d2 *>(X + a + (long long)rx0 * i)
                      : *reinterpret_cast<const d2 *>(Y + (a - rx0) + (long long)ry0 * i);
      } else if (a < rx0 && b < rx1) {
        v = *reinterpret_cast<const d2 *>(X + a + (long long)rx0 * (i + (long long)I * b));
      } else if (a >= rx0 && b >= rx1) {
        v = *reinterpret_cast<const d2 *>(Y + (a - rx0) + (long long)ry0 * (i + (long long)I * (b - rx1)));
      } else {
        v = d2{0.0, 0.0};
      }
    }
    // written once and read by a later pass: stream past the caches
    __builtin_nontemporal_store(v, &Zb[e]);
  }
}

// Device copy of n doubles (a core written back from scratch): 16-byte loads
// and streaming stores over the pairs, the odd last element by one thread.
// Both pointers are 16-byte aligned (checked by the launcher).
__global__ __launch_bounds__(kThreads) void k_copy_pairs(const double *__restrict__ X, long long n,
                                                         double *__restrict__ Y) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  const d2 *X2 = reinterpret_cast<const d2 *>(X);
  d2 *Y2 = reinterpret_cast<d2 *>(Y);
  const long long np = n / 2;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < np; e += stride)
    __builtin_nontemporal_store(X2[e], &Y2[e]);
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) Y[n - 1] = X[n - 1];
}

// ---------------------------------------------------------------------------
// Hadamard: Z(ax*ry0 + ay, i, bx*ry1 + by) = X(ax, i, bx) * Y(ay, i, by);
// output column b = bx*ry1 + by per blockIdx.y.
// ---------------------------------------------------------------------------
__global__ void k_hadamard(const double *__restrict__ X, int rx0, int rx1, const double *__restrict__ Y, int ry0,
                           int ry1, int I, double *__restrict__ Z) {
  const int zr0 = rx0 * ry0;
  const int b = blockIdx.y;
  const int bx = b / ry1, by = b - bx * ry1;
  const int colsz = zr0 * I;
  const long long zoff = (long long)colsz * b;
  const double *Xb = X + (long long)rx0 * I * bx;
  const double *Yb = Y + (long long)ry0 * I * by;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < colsz; e += gridDim.x * blockDim.x) {
    const int i = e / zr0;
    const int a = e - i * zr0;
    const int ax = a / ry0, ay = a - ax * ry0;
    Z[zoff + e] = Xb[ax + rx0 * (long long)i] * Yb[ay + ry0 * (long long)i];
  }
}

// The same product for even R^Y (ry0) with aligned buffers: output column b =
// (bx, by) of Z is I runs of zr0 = rx0 ry0 doubles, run i being the
// Kronecker product X(:, i, bx) (x) Y(:, i, by).  A thread takes a pair
// (ax, 2 ayp), (ax, 2 ayp + 1) of a run: one 16-byte load of Y, one reused
// X entry, one 16-byte streaming store.  Workgroup (x, b) covers runs
// [x iper, (x+1) iper) of column b; the (run, ax, ayp) position of a thread
// advances by fixed increments with carries (no divisions in the loop).
__global__ __launch_bounds__(256) void k_hadamard_pairs(const double *__restrict__ X, int rx0, int rx1,
                                                        const double *__restrict__ Y, int ry0, int ry1, int I,
                                                        int iper, double *__restrict__ Z) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  const int hp = ry0 / 2;       // pairs per X entry
  const int P = rx0 * hp;       // pairs per run
  const int zr0 = rx0 * ry0;
  const int b = blockIdx.y;
  const int bx = b / ry1, by = b - bx * ry1;
  const int i0 = blockIdx.x * iper;
  const int i1 = min(I, i0 + iper);
  const double *Xb = X + (long long)rx0 * I * bx;
  const double *Yb = Y + (long long)ry0 * I * by;
  double *Zb = Z + (long long)zr0 * I * b;
  // starting position of this thread and the increments of a 256-pair step
  int il = threadIdx.x / P, q = threadIdx.x - il * P;
  int ax = q / hp, ayp = q - ax * hp;
  const int di = 256 / P, dq = 256 - di * P;
  const int dax = dq / hp, dayp = dq - dax * hp;
  for (int i = i0 + il; i < i1;) {
    const double x = Xb[ax + (long long)rx0 * i];
    const d2 y = *reinterpret_cast<const d2 *>(Yb + 2 * ayp + (long long)ry0 * i);
    const d2 z = {x * y.x, x * y.y};
    // written once and read by a later pass: stream past the caches
    __builtin_nontemporal_store(z, reinterpret_cast<d2 *>(Zb + (long long)zr0 * i + ax * ry0 + 2 * ayp));
    i += di;
    ax += dax;
    ayp += dayp;
    if (ayp >= hp) {
      ayp -= hp;
      ++ax;
    }
    if (ax >= rx0) {
      ax -= rx0;
      ++i;
    }
  }
}

// ---------------------------------------------------------------------------
// Mode-2 product with a banded matrix (one core of the Kronecker-operator
// matrix-vector product, §3.2.5): Y(a, i, b) = sum_j A(i, j) X(a, j, b) over
// max(0, i - kl) <= j <= min(I - 1, i + ku), A in band storage
// A(i, j) = AB[(ku + i - j) + (kl + ku + 1) j].  For fixed b the runs
// X(:, j, b) are contiguous, so workgroup (x, b) produces the TI runs
// i0 .. i0 + TI - 1 of column b (TI r0 <= 4096 outputs, 16 per thread) from
// the runs its band reaches, staged in LDS JC at a time with contiguous loads;
// each output sums its band in increasing j.
// ---------------------------------------------------------------------------
constexpr int kKronOut = 16;  // outputs per thread
__global__ __launch_bounds__(256) void k_kron_apply(const double *__restrict__ X, int r0, long long I,
                                                    const double *__restrict__ AB, int kl, int ku, int TI, int JC,
                                                    double *__restrict__ Y) {
  HIP_DYNAMIC_SHARED(double, Xs);
  const int b = blockIdx.y;
  const long long i0 = (long long)blockIdx.x * TI;
  const int ti = (int)std::min<long long>(TI, I - i0);
  const int nout = ti * r0;
  const long long ld = (long long)kl + ku + 1;
  const double *Xb = X + (long long)r0 * I * b;
  double *Yb = Y + (long long)r0 * I * b;
  int oi[kKronOut], oa[kKronOut];
  double acc[kKronOut];
#pragma unroll
  for (int k = 0; k < kKronOut; ++k) {
    const int e = threadIdx.x + 256 * k;
    oi[k] = e / r0;
    oa[k] = e - oi[k] * r0;
    acc[k] = 0.0;
  }
  const long long jlo = std::max(0LL, i0 - kl), jhi = std::min(I, i0 + ti + ku);
  for (long long j0 = jlo; j0 < jhi; j0 += JC) {
    const int jc = (int)std::min<long long>(JC, jhi - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < jc * r0; e += 256) Xs[e] = Xb[(long long)r0 * j0 + e];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kKronOut; ++k) {
      if (threadIdx.x + 256 * k >= nout) break;
      const long long i = i0 + oi[k];
      const long long ja = std::max(j0, i - kl), jb = std::min(j0 + jc, i + ku + 1);
      double s = acc[k];
      for (long long j = ja; j < jb; ++j) s += AB[(ku + i - j) + ld * j] * Xs[(j - j0) * r0 + oa[k]];
      acc[k] = s;
    }
  }
#pragma unroll
  for (int k = 0; k < kKronOut; ++k) {
    const int e = threadIdx.x + 256 * k;
    if (e < nout) Yb[(long long)r0 * i0 + e] = acc[k];
  }
}

// ---------------------------------------------------------------------------
// Chunk staging and the small transforms, shared by the Gram and apply passes.
// ---------------------------------------------------------------------------
struct Chunk {
  const double *Z;  // per-slice matrices, slice t at Z + t*stride, column-major zr x zc
  int zr, zc;
  int stride;
};

__device__ inline void stage_chunk(const CoreView &cv, long long i0, int nt, int T, double *Ms) {
  const int pa = cv.pa, pb = cv.pb, ea = cv.ea();
  const long long panel = (long long)pa * nt;
  const long long total = panel * pb;
  for (long long e = threadIdx.x; e < total; e += blockDim.x) {
    const int b = (int)(e / panel);
    const int rem = (int)(e - (long long)b * panel);
    const int t = rem / pa;
    const int a = rem - t * pa;
    const double v = cv.X[a + (long long)pa * (i0 + t) + (long long)pa * cv.I * b];
    const int r = cv.trans ? b : a;
    const int c = cv.trans ? a : b;
    Ms[(long long)t * pa * pb + r + ea * c] = v;
  }
  (void)T;
}

// Applies the stage list to the nt staged slices: left stages first, then
// right stages, ping-ponging between two LDS buffers of `buf` doubles per slice.
__device__ inline Chunk transform_chunk(const CoreView &cv, const Stages &st, int nt, double *Ms, double *B0,
                                        double *B1, int buf) {
  const double *cur = Ms;
  int cr = cv.ea(), cc = cv.eb();
  int curstride = cv.pa * cv.pb;
  double *bufs[2] = {B0, B1};
  int which = 0;
  for (int j = 0; j < st.nl; ++j) {
    const Stage S = st.L[j];
    const int p = S.rows;
    double *out = bufs[which];
    const int total = nt * p * cc;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
      const int t = e / (p * cc);
      const int rem = e - t * p * cc;
      const int c = rem / p;
      const int r = rem - c * p;
      const double *m = cur + (long long)t * curstride + (long long)cr * c;
      double s = 0.0;
      for (int k = 0; k < cr; ++k) s += S.S[r * S.sr + k * S.sc] * m[k];
      out[(long long)t * buf + r + p * c] = s;
    }
    __syncthreads();
    cur = out;
    curstride = buf;
    cr = p;
    which ^= 1;
  }
  for (int j = 0; j < st.nr; ++j) {
    const Stage S = st.R[j];
    const int q = S.cols;
    double *out = bufs[which];
    const int total = nt * cr * q;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
      const int t = e / (cr * q);
      const int rem = e - t * cr * q;
      const int c = rem / cr;
      const int r = rem - c * cr;
      const double *m = cur + (long long)t * curstride + r;
      double s = 0.0;
      for (int k = 0; k < cc; ++k) s += m[(long long)cr * k] * S.S[k * S.sr + c * S.sc];
      out[(long long)t * buf + r + cr * c] = s;
    }
    __syncthreads();
    cur = out;
    curstride = buf;
    cc = q;
    which ^= 1;
  }
  Chunk ch;
  ch.Z = cur;
  ch.zr = cr;
  ch.zc = cc;
  ch.stride = curstride;
  return ch;
}


// Largest per-slice intermediate of the stage chain (doubles).
inline int stage_buf(const CoreView &cv, const Stages &st) {
  int cr = cv.ea(), cc = cv.eb(), mx = 0;
  for (int j = 0; j < st.nl; ++j) {
    cr = st.L[j].rows;
    mx = std::max(mx, cr * cc);
  }
  for (int j = 0; j < st.nr; ++j) {
    cc = st.R[j].cols;
    mx = std::max(mx, cr * cc);
  }
  return mx;
}

inline long long per_slice(const CoreView &cv, const Stages &st) {
  const int nb = (st.nl + st.nr) >= 2 ? 2 : (st.nl + st.nr);
  return (long long)cv.pa * cv.pb + (long long)nb * stage_buf(cv, st);
}

inline int chunk_slices(const CoreView &cv, const Stages &st, long long I) {
  long long T = (long long)(kLdsBudget / sizeof(double)) / std::max(per_slice(cv, st), 1LL);
  T = std::max(1LL, std::min(T, 64LL));
  T = std::min(T, std::max(I, 1LL));
  return (int)T;
}

inline size_t chunk_lds(const CoreView &cv, const Stages &st, int T) {
  return (size_t)(per_slice(cv, st) * T) * sizeof(double);
}

// ---------------------------------------------------------------------------
// Gram pass: per-workgroup partial G over a contiguous range of slices.
// Each thread owns up to kMaxOwn entries of the lower triangle.
// ---------------------------------------------------------------------------
constexpr int kMaxOwn = (TTR_RMAX * (TTR_RMAX + 1) / 2 + kThreads - 1) / kThreads;

__global__ __launch_bounds__(kThreads) void k_gram(CoreView cv, Stages st, int mode, int T, long long spw, int buf,
                                                  double *__restrict__ partials) {
  HIP_DYNAMIC_SHARED(double, smem);
  const int zr = st.nl ? st.L[st.nl - 1].rows : cv.ea();
  const int zc = st.nr ? st.R[st.nr - 1].cols : cv.eb();
  const int gd = (mode == GRAM_LEFT) ? zr : zc;
  double *Ms = smem;
  double *B0 = Ms + (long long)T * cv.pa * cv.pb;
  double *B1 = B0 + (long long)T * buf;

  const int nent = gd * (gd + 1) / 2;
  int ou[kMaxOwn], ov[kMaxOwn];
  double acc[kMaxOwn];
#pragma unroll
  for (int j = 0; j < kMaxOwn; ++j) {
    const int e = threadIdx.x + j * kThreads;
    int u = 0, v = 0;
    if (e < nent) {
      u = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
      while (u * (u + 1) / 2 > e) --u;
      while ((u + 1) * (u + 2) / 2 <= e) ++u;
      v = e - u * (u + 1) / 2;
    }
    ou[j] = u;
    ov[j] = v;
    acc[j] = 0.0;
  }

  const long long beg = (long long)blockIdx.x * spw;
  const long long end = std::min(beg + spw, cv.I);
  for (long long i0 = beg; i0 < end; i0 += T) {
    const int nt = (int)std::min((long long)T, end - i0);
    stage_chunk(cv, i0, nt, T, Ms);
    __syncthreads();
    const Chunk ch = transform_chunk(cv, st, nt, Ms, B0, B1, buf);
#pragma unroll
    for (int j = 0; j < kMaxOwn; ++j) {
      const int e = threadIdx.x + j * kThreads;
      if (e < nent) {
        const int u = ou[j], v = ov[j];
        double s = acc[j];
        for (int t = 0; t < nt; ++t) {
          const double *z = ch.Z + (long long)t * ch.stride;
          if (mode == GRAM_LEFT) {
            for (int c = 0; c < ch.zc; ++c) s += z[u + ch.zr * c] * z[v + ch.zr * c];
          } else {
            const double *zu = z + (long long)ch.zr * u;
            const double *zv = z + (long long)ch.zr * v;
            for (int r = 0; r < ch.zr; ++r) s += zu[r] * zv[r];
          }
        }
        acc[j] = s;
      }
    }
    __syncthreads();
  }
  double *out = partials + (long long)blockIdx.x * gd * gd;
#pragma unroll
  for (int j = 0; j < kMaxOwn; ++j) {
    const int e = threadIdx.x + j * kThreads;
    if (e < nent) {
      out[ou[j] + gd * ov[j]] = acc[j];
      out[ov[j] + gd * ou[j]] = acc[j];
    }
  }
}

// Fixed-order sum of the per-workgroup partials: G[e] = sum_w partials[w][e].
// A block handles 16 entries; its 16 x 16 threads each sum one contiguous
// segment of the partials, and the 16 segment sums are added in order.
constexpr int kRedEnt = 16, kRedSeg = 16;
__global__ __launch_bounds__(kRedEnt *kRedSeg) void k_reduce(const double *__restrict__ partials, int nwg, int ne,
                                                             double *__restrict__ G) {
  __shared__ double part[kRedSeg][kRedEnt];
  const int le = threadIdx.x % kRedEnt, seg = threadIdx.x / kRedEnt;
  const int e = blockIdx.x * kRedEnt + le;
  const int per = (nwg + kRedSeg - 1) / kRedSeg;
  const int w0 = seg * per, w1 = min(nwg, w0 + per);
  double s = 0.0;
  if (e < ne)
    for (int w = w0; w < w1; ++w) s += partials[(long long)w * ne + e];
  part[seg][le] = s;
  __syncthreads();
  if (seg == 0 && e < ne) {
    double t = 0.0;
    for (int k = 0; k < kRedSeg; ++k) t += part[k][le];
    G[e] = t;
  }
}

// ---------------------------------------------------------------------------
// Apply pass: Y(i) = P M(i) Q written as a new core.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_apply(CoreView cv, Stages st, int T, long long spw, int buf,
                                                   double *__restrict__ Y, int trans_out) {
  HIP_DYNAMIC_SHARED(double, smem);
  double *Ms = smem;
  double *B0 = Ms + (long long)T * cv.pa * cv.pb;
  double *B1 = B0 + (long long)T * buf;
  const long long beg = (long long)blockIdx.x * spw;
  const long long end = std::min(beg + spw, cv.I);
  const long long I = cv.I;
  for (long long i0 = beg; i0 < end; i0 += T) {
    const int nt = (int)std::min((long long)T, end - i0);
    stage_chunk(cv, i0, nt, T, Ms);
    __syncthreads();
    const Chunk ch = transform_chunk(cv, st, nt, Ms, B0, B1, buf);
    const int p = ch.zr, q = ch.zc;
    const long long total = (long long)p * nt * q;
    if (!trans_out) {
      // output p x I x q: for each column c the chunk is p*nt contiguous doubles
      const long long panel = (long long)p * nt;
      for (long long e = threadIdx.x; e < total; e += blockDim.x) {
        const int c = (int)(e / panel);
        const int rem = (int)(e - (long long)c * panel);
        const int t = rem / p;
        const int r = rem - t * p;
        Y[r + (long long)p * (i0 + t) + (long long)p * I * c] = ch.Z[(long long)t * ch.stride + r + p * c];
      }
    } else {
      // output q x I x p (transposed slices)
      const long long panel = (long long)q * nt;
      for (long long e = threadIdx.x; e < total; e += blockDim.x) {
        const int r = (int)(e / panel);
        const int rem = (int)(e - (long long)r * panel);
        const int t = rem / q;
        const int c = rem - t * q;
        Y[c + (long long)q * (i0 + t) + (long long)q * I * r] = ch.Z[(long long)t * ch.stride + r + p * c];
      }
    }
    __syncthreads();
  }
}


int grid_for(long long I, int T) {
  const long long chunks = (I + T - 1) / T;
  return (int)std::max(1LL, std::min(chunks, (long long)TTR_MAXWG));
}

long long slices_per_wg(long long I, int T, int nwg) {
  long long spw = (I + nwg - 1) / nwg;
  spw = ((spw + T - 1) / T) * T;
  return std::max(spw, 1LL);
}

}  // namespace

void launch_add(hipStream_t s, int n, int N, double alpha, double beta, const double *X, int rx0, int rx1,
                const double *Y, int ry0, int ry1, long long I, double *Z) {
  int zr0, zr1;
  if (N == 1) zr0 = zr1 = 1;
  else if (n == 0) { zr0 = 1; zr1 = rx1 + ry1; }
  else if (n == N - 1) { zr0 = rx0 + ry0; zr1 = 1; }
  else { zr0 = rx0 + ry0; zr1 = rx1 + ry1; }
  const long long colsz = (long long)zr0 * I;
  // 16-byte accesses: even extents and 16-byte aligned cores
  const bool aligned = (((uintptr_t)X | (uintptr_t)Y | (uintptr_t)Z) % 16) == 0;
  const bool pairs = N > 1 && aligned && (n == 0 ? (I % 2 == 0) : (rx0 % 2 == 0 && ry0 % 2 == 0)) &&
                     colsz / 2 < (1LL << 24);
  if (pairs) {
    const long long bx = std::min((colsz / 2 + kThreads - 1) / kThreads, 4096LL);
    hipLaunchKernelGGL(k_add_pairs, dim3((unsigned)std::max(bx, 1LL), (unsigned)zr1), dim3(kThreads), 0, s, n, N,
                       alpha, beta, X, rx0, rx1, Y, ry0, ry1, (int)I, Z);
    return;
  }
  const long long bx = std::min((colsz + kThreads - 1) / kThreads, 4096LL);
  hipLaunchKernelGGL(k_add, dim3((unsigned)std::max(bx, 1LL), (unsigned)zr1), dim3(kThreads), 0, s, n, N, alpha, beta,
                     X, rx0, rx1, Y, ry0, ry1, (int)I, Z);
}

void launch_copy(hipStream_t s, const double *X, long long n, double *Y) {
  if (n <= 0) return;
  if ((uintptr_t)X % 16 != 0 || (uintptr_t)Y % 16 != 0) {
    (void)hipMemcpyAsync(Y, X, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s);
    return;
  }
  // about eight pairs per thread, at most 8192 workgroups
  const long long bx = std::min((n / 2 + 8LL * kThreads - 1) / (8LL * kThreads), 8192LL);
  hipLaunchKernelGGL(k_copy_pairs, dim3((unsigned)std::max(bx, 1LL)), dim3(kThreads), 0, s, X, n, Y);
}

void launch_kron_apply(hipStream_t s, const double *X, int r0, int r1, long long I, const double *AB, int kl, int ku,
                       double *Y) {
  const int TI = (int)std::max(1LL, std::min<long long>(I, (256LL * kKronOut) / r0));
  const int JC = std::max(1, 8192 / r0);
  const long long gx = (I + TI - 1) / TI;
  hipLaunchKernelGGL(k_kron_apply, dim3((unsigned)gx, (unsigned)r1), dim3(256), (size_t)JC * r0 * sizeof(double), s, X,
                     r0, I, AB, kl, ku, TI, JC, Y);
}

void launch_hadamard(hipStream_t s, const double *X, int rx0, int rx1, const double *Y, int ry0, int ry1, long long I,
                     double *Z) {
  const long long colsz = (long long)rx0 * ry0 * I;
  const bool aligned = ((uintptr_t)Y % 16 == 0) && ((uintptr_t)Z % 16 == 0);
  if (ry0 % 2 == 0 && aligned && I < (1LL << 31)) {
    // runs per workgroup: about 64 K pairs of a column per workgroup
    const long long P = (long long)rx0 * (ry0 / 2);
    const long long iper = std::max(1LL, std::min(I, (65536 + P - 1) / P));
    const long long gx = (I + iper - 1) / iper;
    hipLaunchKernelGGL(k_hadamard_pairs, dim3((unsigned)gx, (unsigned)(rx1 * ry1)), dim3(256), 0, s, X, rx0, rx1, Y,
                       ry0, ry1, (int)I, (int)iper, Z);
    return;
  }
  const long long bx = std::min((colsz + kThreads - 1) / kThreads, 4096LL);
  hipLaunchKernelGGL(k_hadamard, dim3((unsigned)std::max(bx, 1LL), (unsigned)(rx1 * ry1)), dim3(kThreads), 0, s, X,
                     rx0, rx1, Y, ry0, ry1, (int)I, Z);
}

int launch_gram(hipStream_t s, const CoreView &cv, const Stages &st, int mode, double *partials, double *G,
                int mixed) {
  (void)mixed;
  const int T = chunk_slices(cv, st, cv.I);
  const int nwg = grid_for(cv.I, T);
  const long long spw = slices_per_wg(cv.I, T, nwg);
  const int nwg_used = (int)((cv.I + spw - 1) / spw);
  const size_t lds = chunk_lds(cv, st, T);
  const int buf = stage_buf(cv, st);
  hipLaunchKernelGGL(k_gram, dim3(nwg_used), dim3(kThreads), lds, s, cv, st, mode, T, spw, buf, partials);
  (void)G;
  return nwg_used;
}

void launch_reduce(hipStream_t s, const double *partials, int nwg, int ne, double *G) {
  hipLaunchKernelGGL(k_reduce, dim3((ne + kRedEnt - 1) / kRedEnt), dim3(kRedEnt * kRedSeg), 0, s, partials, nwg, ne,
                     G);
}

void launch_apply(hipStream_t s, const CoreView &cv, const Stages &st, double *Y, int trans_out) {
  const int T = chunk_slices(cv, st, cv.I);
  const int nwg = grid_for(cv.I, T);
  const long long spw = slices_per_wg(cv.I, T, nwg);
  const int nwg_used = (int)((cv.I + spw - 1) / spw);
  const size_t lds = chunk_lds(cv, st, T);
  const int buf = stage_buf(cv, st);
  hipLaunchKernelGGL(k_apply, dim3(nwg_used), dim3(kThreads), lds, s, cv, st, T, spw, buf, Y, trans_out);
}

