// Host side of libttr: argument checking, workspace, and the sweeps of TT
// orthonormalization (§2.3 Alg. 1, §3.4 Alg. 5) and TT rounding (§2.4 Alg. 2,
// §3.5 Alg. 6).  All arithmetic runs in the kernels of ttr_stream.hip and
// ttr_small.hip; this file only plans launches and reads back the small
// integer decisions (ranks, pass counts) that size the next launch.
#include "ttr_host.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

// Scratch of ttr_dot_noalloc: the partial inner-product matrices of one step
// (at most 512 workgroups x 64 x 64 doubles) and the two W matrices of the
// recursion.  One copy per device, held until the process ends.  Host code
// never uses this name as an address: it uses the pointer that
// hipGetSymbolAddress returned on the device (noalloc_scratch_of).
constexpr size_t kNoAllocPartials = (size_t)512 * TTR_RMAX * TTR_RMAX;
constexpr size_t kNoAllocDoubles = kNoAllocPartials + 2 * (size_t)TTR_RMAX * TTR_RMAX;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

__global__ void k_set_one(double *p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = 1.0;
}

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

}  // namespace

int ttr_fail(int code, const std::string &msg) { return fail(code, msg); }

namespace {

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(TTR_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

const double kTau1 = 1e-3;   // pass-1 eigenvalue ratio above which one Gram pass is enough
const double kTau2 = 1e-12;  // preconditioned eigenvalues below this are rounding noise

int check_tt(const ttr_tt *X, const char *name, int max_rank) {
  if (!X) return fail(TTR_ERR_INVALID_ARG, std::string(name) + " is NULL");
  if (X->N < 1) return fail(TTR_ERR_INVALID_ARG, std::string(name) + ": N must be >= 1");
  if (!X->I || !X->R || !X->core) return fail(TTR_ERR_INVALID_ARG, std::string(name) + ": NULL array");
  if (X->R[0] != 1 || X->R[X->N] != 1)
    return fail(TTR_ERR_INVALID_ARG, std::string(name) + ": boundary ranks must be 1");
  for (int n = 0; n < X->N; ++n) {
    if (X->I[n] <= 0) return fail(TTR_ERR_INVALID_ARG, std::string(name) + ": mode size must be > 0");
    if (X->R[n + 1] <= 0) return fail(TTR_ERR_INVALID_ARG, std::string(name) + ": rank must be > 0");
    if (!X->core[n]) return fail(TTR_ERR_INVALID_ARG, std::string(name) + ": NULL core pointer");
    if (max_rank > 0 && (X->R[n] > max_rank || X->R[n + 1] > max_rank))
      return fail(TTR_ERR_UNSUPPORTED, std::string(name) + ": rank above TTR_MAX_RANK");
  }
  return TTR_OK;
}

int check_out(const ttr_tt *Z, const char *name, int N, const int64_t *I) {
  if (!Z) return fail(TTR_ERR_INVALID_ARG, std::string(name) + " is NULL");
  if (Z->N != N) return fail(TTR_ERR_SHAPE, std::string(name) + ": N differs");
  if (!Z->I || !Z->R || !Z->core || !Z->cap) return fail(TTR_ERR_INVALID_ARG, std::string(name) + ": NULL array");
  for (int n = 0; n < N; ++n) {
    if (Z->I[n] != I[n]) return fail(TTR_ERR_SHAPE, std::string(name) + ": mode sizes differ");
    if (!Z->core[n]) return fail(TTR_ERR_INVALID_ARG, std::string(name) + ": NULL core pointer");
  }
  return TTR_OK;
}

int ensure_ws(ttr_handle *h, size_t bytes) {
  if (bytes <= h->ws_bytes) return TTR_OK;
  if (h->ws) {
    HIPCHK(hipStreamSynchronize(h->stream));
    ttr_dev_free(h, h->ws);
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  void *p = nullptr;
  int rc;
  if ((rc = ttr_dev_alloc(h, &p, bytes))) return rc;
  h->ws = static_cast<double *>(p);
  h->ws_bytes = bytes;
  return TTR_OK;
}

// Workspace carve-up (in doubles).  Every small matrix slot holds RMAX^2.
constexpr size_t kSlot = (size_t)TTR_RMAX * TTR_RMAX;
constexpr int kStagesPerCore = 3;
constexpr int kScalF32 = 16;  // w.scal[16..18]: the scales of an FP32 Gram pass
struct WS {
  double *partials, *G, *Ra, *Rb, *Gst[3], *Pa, *Pb, *GU, *Wa, *Wb, *Fp, *scal, *sigma, *tails, *Tn, *Bst, *tmp, *matA,
      *matB;
  int *dec;
  double *T(int n) const { return Tn + (size_t)n * kSlot; }
  double *B(int n, int j) const { return Bst + ((size_t)n * kStagesPerCore + j) * kSlot; }
};
// tmp: staging for an explicit output core; mat: each of the two buffers that
// hold materialized cores of ill-conditioned factorizations
// every segment of the workspace starts on a 256-byte boundary: the sizes
// that are not multiples of 32 doubles are rounded up
size_t r32(size_t n) { return (n + 31) / 32 * 32; }
size_t ws_doubles(int N, size_t tmp, size_t mat = 0) {
  return (size_t)TTR_MAXWG * kSlot + 12 * kSlot + 64 + (size_t)(N + 1) * TTR_RMAX + r32(N + 1) +
         (size_t)(N + 2) * (1 + kStagesPerCore) * kSlot + r32(tmp) + 2 * r32(mat) + 64;
}
WS carve(ttr_handle *h, int N, size_t tmp, size_t mat = 0) {
  WS w;
  double *p = h->ws;
  w.partials = p; p += (size_t)TTR_MAXWG * kSlot;
  w.G = p; p += kSlot;
  w.Ra = p; p += kSlot;
  w.Rb = p; p += kSlot;
  for (int j = 0; j < 3; ++j) { w.Gst[j] = p; p += kSlot; }
  w.Pa = p; p += kSlot;
  w.Pb = p; p += kSlot;
  w.GU = p; p += kSlot;
  w.Wa = p; p += kSlot;
  w.Wb = p; p += kSlot;
  w.Fp = p; p += kSlot;
  w.scal = p; p += 64;
  w.sigma = p; p += (size_t)(N + 1) * TTR_RMAX;
  w.tails = p; p += r32(N + 1);
  w.Tn = p; p += (size_t)(N + 2) * kSlot;
  w.Bst = p; p += (size_t)(N + 2) * kStagesPerCore * kSlot;
  w.tmp = p; p += r32(tmp);
  w.matA = mat ? p : nullptr; p += r32(mat);
  w.matB = mat ? p : nullptr; p += r32(mat);
  w.dec = h->dec_dev;
  return w;
}

// --- opt-in kernel timing ------------------------------------------------
enum {
  P_GRAM_R = 0, P_GRAM_L = 1, P_GRAM_G = 2, P_APPLY = 3, P_APPLY_G = 4, P_ADD = 5, P_HAD = 6, P_DOT = 7, P_SMALL = 8,
  P_GRAM_FAC = 9, P_APPLY_FAC2 = 10, P_GRAM_R32 = 11, P_GRAM_L32 = 12, P_KRON = 13
};

hipEvent_t take_event(ttr_handle *h) {
  if (!h->evpool.empty()) {
    hipEvent_t e = h->evpool.back();
    h->evpool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct ProfScope {
  ttr_handle *h;
  hipEvent_t a = nullptr;
  int cls;
  double bytes, flops;
  ProfScope(ttr_handle *h_, int cls_, double bytes_, double flops_) : h(h_), cls(cls_), bytes(bytes_), flops(flops_) {
    if (h->profiling) {
      a = take_event(h);
      if (a) (void)hipEventRecord(a, h->stream);
    }
  }
  ~ProfScope() {
    if (!h->profiling || !a) return;
    hipEvent_t b = take_event(h);
    if (!b) return;
    (void)hipEventRecord(b, h->stream);
    h->pending.push_back({a, b, cls, bytes, flops});
  }
};

void prof_resolve(ttr_handle *h) {
  if (h->pending.empty()) return;
  (void)hipStreamSynchronize(h->stream);
  for (auto &p : h->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      h->prof.count[p.cls] += 1;
      h->prof.ms[p.cls] += ms;
      h->prof.bytes[p.cls] += p.bytes;
      h->prof.flops[p.cls] += p.flops;
    }
    h->evpool.push_back(p.a);
    h->evpool.push_back(p.b);
  }
  h->pending.clear();
}

// per-slice flops of a stage chain and the chain's output shape
double chain_flops(const CoreView &cv, const Stages &st, int *zr, int *zc) {
  double f = 0.0;
  int cr = cv.ea(), cc = cv.eb();
  for (int j = 0; j < st.nl; ++j) {
    f += 2.0 * st.L[j].rows * cr * cc;
    cr = st.L[j].rows;
  }
  for (int j = 0; j < st.nr; ++j) {
    f += 2.0 * cr * cc * st.R[j].cols;
    cc = st.R[j].cols;
  }
  *zr = cr;
  *zc = cc;
  return f;
}

// A stage on the physical core: transposed views swap roles (Z^T = R^T X L^T).
// transposes swap lower <-> upper: "lower" 1 = lower, 2 = upper
Stage st_transpose(const Stage &a) {
  Stage t;
  t.S = a.S;
  t.rows = a.cols;
  t.cols = a.rows;
  t.sr = a.sc;
  t.sc = a.sr;
  t.lower = (a.lower == 1) ? 2 : (a.lower == 2 ? 1 : 0);
  return t;
}

// Streaming Gram of the chain Z(i) = lefts M(i) rights.  The one-factor forms
// (the first pass of every factorization, the common case) run on the matrix
// cores, in FP32 when `f32` asks for it (*ran_f32 reports whether it did);
// the one-right-factor RIGHT form of a materialized core (refinement passes)
// runs on the FP64 matrix cores; longer chains run on the staged generic
// kernel.
// Returns the number of workgroups (partial Grams) the pass used.
int gram(ttr_handle *h, double *partials, double *G, const CoreView &cv, const Stages &st, int mode, int f32 = 0,
         bool *ran_f32 = nullptr, double *fscale = nullptr) {
  int zr, zc;
  const double cf = chain_flops(cv, st, &zr, &zc);
  const double gf = (mode == GRAM_LEFT) ? (double)zr * (zr + 1) * zc : (double)zc * (zc + 1) * zr;
  const int gd = (mode == GRAM_LEFT) ? zr : zc;
  const double bytes = 8.0 * cv.pa * cv.pb * (double)cv.I, flops = (cf + gf) * (double)cv.I;
  // physical form: trans views transpose the chain and swap the Gram side
  const bool tr = cv.trans != 0;
  const int pmode = tr ? (mode == GRAM_LEFT ? GRAM_RIGHT : GRAM_LEFT) : mode;
  const int pnl = tr ? st.nr : st.nl;
  const int pnr = tr ? st.nl : st.nr;
  const double *X = cv.X;
  int nwg = 0;
  bool done = false;
  if (ran_f32) *ran_f32 = false;
  {
    if (pmode == GRAM_LEFT && pnl == 0 && pnr <= 1) {
      // sum (X Q)(X Q)^T
      const Stage *q = pnr ? (tr ? &st.L[0] : &st.R[0]) : nullptr;
      Stage qq;
      if (q) qq = tr ? st_transpose(*q) : *q;
      ProfScope ps(h, f32 ? P_GRAM_R32 : P_GRAM_R, bytes, flops);
      nwg = launch_gram_right_factor(h->stream, X, cv.pa, cv.pb, cv.I, q ? qq.S : nullptr, q ? qq.cols : cv.pb,
                                     q ? qq.sr : 1, q ? qq.sc : cv.pb, (q && qq.lower == 1) ? 1 : 0, f32, partials,
                                     fscale);
      done = true;
      if (ran_f32) *ran_f32 = f32 != 0;
    } else if (pmode == GRAM_RIGHT && pnl <= 1 && pnr == 0) {
      // sum (P X)^T (P X)
      const Stage *pp = pnl ? (tr ? &st.R[0] : &st.L[0]) : nullptr;
      Stage ps_;
      if (pp) ps_ = tr ? st_transpose(*pp) : *pp;
      ProfScope ps(h, f32 ? P_GRAM_L32 : P_GRAM_L, bytes, flops);
      nwg = launch_gram_left_factor(h->stream, X, cv.pa, cv.pb, cv.I, pp ? ps_.S : nullptr, pp ? ps_.rows : cv.pa,
                                    pp ? ps_.sr : 1, pp ? ps_.sc : cv.pa, (pp && ps_.lower == 2) ? 1 : 0, f32,
                                    partials, fscale);
      done = true;
      if (ran_f32) *ran_f32 = f32 != 0;
    } else if (mode == GRAM_RIGHT && st.nl == 0 && st.nr == 1) {
      // logical sum (M Q)^T (M Q), M the (possibly transposed) slice
      const Stage &q = st.R[0];
      ProfScope ps(h, P_GRAM_FAC, bytes, flops);
      nwg = launch_gram_fac(h->stream, X, cv.pa, cv.pb, cv.I, cv.trans, q.S, q.cols, q.sr, q.sc, q.lower == 1 ? 1 : 0,
                            partials);
      done = true;
    } else if (mode == GRAM_LEFT && st.nl == 1 && st.nr == 0) {
      // logical sum (L M)(L M)^T = sum (M^T L^T)^T (M^T L^T): the same kernel on
      // the transposed slice with Q = L^T
      const Stage &l = st.L[0];
      ProfScope ps(h, P_GRAM_FAC, bytes, flops);
      nwg = launch_gram_fac(h->stream, X, cv.pa, cv.pb, cv.I, !cv.trans, l.S, l.rows, l.sc, l.sr, l.lower == 2 ? 1 : 0,
                            partials);
      done = true;
    }
  }
  if (!done) {
    ProfScope ps(h, P_GRAM_G, bytes, flops);
    nwg = launch_gram(h->stream, cv, st, mode, partials, G, 0);
  }
  launch_reduce(h->stream, partials, nwg, gd * gd, G);
  return nwg;
}

// Output pass Y(i) = lefts M(i) rights, on the matrix cores when the chain has
// at most one factor on each side, or is two right factors on a materialized
// core.
void apply(ttr_handle *h, const CoreView &cv, const Stages &st, double *Y, int trans_out) {
  int zr, zc;
  const double cf = chain_flops(cv, st, &zr, &zc);
  const double abytes = 8.0 * ((double)cv.pa * cv.pb + (double)zr * zc) * (double)cv.I;
  const bool tr = cv.trans != 0;
  if (st.nl <= 1 && st.nr <= 1 && trans_out == cv.trans) {
    ProfScope ps(h, P_APPLY, abytes, cf * (double)cv.I);
    // physical: Y_phys = Pp X Qp; trans views: (L M' R)^T = R^T X L^T
    const Stage *L = st.nl ? &st.L[0] : nullptr;
    const Stage *R = st.nr ? &st.R[0] : nullptr;
    const Stage *pl = tr ? R : L;
    const Stage *pr = tr ? L : R;
    Stage P, Q;
    if (pl) P = tr ? st_transpose(*pl) : *pl;
    if (pr) Q = tr ? st_transpose(*pr) : *pr;
    const int tri = ((pr && Q.lower == 1) ? 1 : 0) | ((pl && P.lower == 2) ? 2 : 0);
    launch_apply_mfma(h->stream, cv.X, cv.pa, cv.pb, cv.I, pl ? P.S : nullptr, pl ? P.rows : cv.pa, pl ? P.sr : 1,
                      pl ? P.sc : cv.pa, pr ? Q.S : nullptr, pr ? Q.cols : cv.pb, pr ? Q.sr : 1,
                      pr ? Q.sc : cv.pb, tri, Y);
    return;
  }
  if (st.nl == 0 && st.nr == 2 && trans_out == cv.trans) {
    ProfScope ps(h, P_APPLY_FAC2, abytes, cf * (double)cv.I);
    const Stage &q1 = st.R[0], &q2 = st.R[1];
    launch_apply_fac2(h->stream, cv.X, cv.pa, cv.pb, cv.I, cv.trans, q1.S, q1.cols, q1.sr, q1.sc,
                      q1.lower == 1 ? 1 : 0, q2.S, q2.cols, q2.sr, q2.sc, Y);
    return;
  }
  if (st.nl == 2 && st.nr == 0 && trans_out == cv.trans) {
    // L2 L1 M = (M^T L1^T L2^T)^T: the transposed slice with Q1 = L1^T, Q2 = L2^T,
    // written transposed back
    ProfScope ps(h, P_APPLY_FAC2, abytes, cf * (double)cv.I);
    const Stage &l1 = st.L[0], &l2 = st.L[1];
    launch_apply_fac2(h->stream, cv.X, cv.pa, cv.pb, cv.I, !cv.trans, l1.S, l1.rows, l1.sc, l1.sr,
                      l1.lower == 2 ? 1 : 0, l2.S, l2.rows, l2.sc, l2.sr, Y);
    return;
  }
  ProfScope ps(h, P_APPLY_G, abytes, cf * (double)cv.I);
  launch_apply(h->stream, cv, st, Y, trans_out);
}

int sync_dec(ttr_handle *h) {
  HIPCHK(hipMemcpyAsync(h->dec_host, h->dec_dev, 16 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(h->decf_host, h->decf_dev, 8 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipGetLastError());
  if (h->dec_host[2] != 0) return fail(TTR_ERR_NUMERICAL, "non-finite data or a small factorization did not converge");
  return TTR_OK;
}

int reset_dec(ttr_handle *h) {
  for (int i = 0; i < 16; ++i) h->dec_host[i] = 0;
  HIPCHK(hipMemcpyAsync(h->dec_dev, h->dec_host, 16 * sizeof(int), hipMemcpyHostToDevice, h->stream));
  return TTR_OK;
}

// Logical sequence of cores: RLR / right side uses the cores as stored; LRL /
// left side uses the reversed train with transposed slices (the mirror image).
struct Seq {
  const ttr_tt *X;
  int rev;
  int N() const { return X->N; }
  int phys(int n) const { return rev ? X->N - 1 - n : n; }
  CoreView view(int n) const {
    const int p = phys(n);
    CoreView cv;
    cv.X = X->core[p];
    cv.I = X->I[p];
    cv.pa = (int)X->R[p];
    cv.pb = (int)X->R[p + 1];
    cv.trans = rev;
    return cv;
  }
  // logical rank at logical link l (between logical cores l-1 and l), l = 0..N
  int64_t rank(int l) const { return rev ? X->R[X->N - l] : X->R[l]; }
};

// Stage constructors (column-major small matrices)
Stage st_plain(const double *M, int rows, int cols, int lower = 0) {  // M (rows x cols, ld rows)
  Stage s;
  s.lower = lower;
  s.S = M;
  s.rows = rows;
  s.cols = cols;
  s.sr = 1;
  s.sc = rows;
  return s;
}
Stage st_trans(const double *M, int rows, int cols) {  // M^T where M is (cols x rows, ld cols)
  Stage s;
  s.lower = 0;
  s.S = M;
  s.rows = rows;
  s.cols = cols;
  s.sr = cols;
  s.sc = 1;
  return s;
}
Stages no_stages() {
  Stages s;
  s.nl = 0;
  s.nr = 0;
  return s;
}

// The orthonormal factor of one core's orthonormalization QR, kept as stages
// F_1 ... F_j (F_i is dim[i] x dim[i+1]); dim[0] = left rank of the core.
struct Factor {
  int nst = 0;
  int dim[4] = {0, 0, 0, 0};
  int tri = 0;    // one-pass Cholesky route: T = L lower triangular, F = L^{-T}
  int mat = 0;    // stages apply to the materialized core M(i) T_{n+1}, not to M(i)
  int rorth = 0;  // one-pass eigen route: the rows of R are mutually orthogonal
};

// One QR-by-Gram factorization of a tall-skinny unfolding of a logical core,
// through up to three streaming Gram passes.
//   LEFT  (orthonormalization sweep): A = H(C)^T with C(i) = base(M(i)); the
//         stages F_j^T are appended as LEFT stages, pass Gram sum Z Z^T.
//   RIGHT (truncation sweep): A = V(C'), C'(i) = base(M(i)); the stages F_j are
//         appended as RIGHT stages, pass Gram sum Z^T Z.
// `slot(j)` gives the device slot for stage j.  On return: the collapsed R
// (k x b) in *Rout, the stages recorded in *f.
//   tcond: kappa(T)^2 of a single right stage T of `base` in RIGHT mode.  When
//   finite, the first pass forms G0 without T on the matrix cores and the step
//   kernel applies G = T^T G0 T; a tightened acceptance test accounts for T.
// Truncation-sweep context for the step kernel's "no truncation possible" test.
struct TruncCtx {
  int check = 0;
  const double *delta_dev = nullptr;
  int first = 0;
  double tol2_nm1 = 0.0;
  int notrunc = 0;  // out: proved at the accepted one-pass step
};

// Precision plan of one factorization.
//   FP64 (TTR_FP64): every Gram pass in FP64; a pass settles when the Gram's
//     condition number is at most 1/kTau1 (orthonormality to ~1e-13).
//   Mixed (TTR_MIXED): the first pass forms the Gram on the FP32 matrix cores
//     (FP32 products and accumulation); refinement passes are FP64.  A pass
//     settles when u * kappa(G) <= kTauMix for the unit roundoff u of the
//     arithmetic that formed G, i.e. the factor is orthonormal to ~kTauMix.
//     The tensor itself is not affected by this choice: every factor R is the
//     exact inverse of the basis change applied to the core, in FP64.
struct Prec {
  int mixed = 0;
};
const double kU64 = 1.1102230246251565e-16;  // 2^-53
const double kU32 = 5.9604644775390625e-08;  // 2^-24
const double kTauMix = 1e-5;

// Bound on the rounding error of a streamed Gram, relative to its trace:
// sequential accumulations per entry (slices per wave times the contracted
// length), the fixed-order cross-wave/workgroup sums and the products.  `nwg`
// is the number of workgroups the pass ran with (each takes a contiguous run
// of ceil(I / nwg) slices, split over its four waves).
double gram_err(const CoreView &cv, int contracted, double u, long long nwg) {
  nwg = std::max<long long>(1, nwg);
  const long long spw = (cv.I + nwg - 1) / nwg;
  const double nacc = (double)((spw + 3) / 4) * contracted + 4.0 + (double)nwg + 2.0;
  return 2.0 * nacc * u;
}

template <class SlotFn>
int qr_by_gram(ttr_handle *h, WS &w, const CoreView &cv, int mode, const Stages &base, int b, SlotFn slot,
               double *Tdst, Factor *f, double **Rout, int *kout, int *passes, double tcond = -1.0,
               double *ratio = nullptr, TruncCtx *tc = nullptr, Prec pr = Prec(), double *mat = nullptr,
               CoreView *cv_out = nullptr, int *materialized = nullptr, const Stage *gram_left = nullptr) {
  double *R[2] = {w.Ra, w.Rb};
  const double *Rc = nullptr;
  int d = b;
  f->nst = 0;
  f->dim[0] = b;
  Stages st = base;
  CoreView cvp = cv;  // the core the current stages apply to
  if (cv_out) *cv_out = cv;
  if (materialized) *materialized = 0;
  for (int pass = 1; pass <= 3; ++pass) {
    QrStepArgs qa;
    qa.Tpost = nullptr;
    qa.tpr = qa.tpc = 0;
    qa.tsr = qa.tsc = 0;
    qa.cond_scale = 1.0;
    qa.ratio_out = (pass == 1) ? h->decf_dev : nullptr;
    const bool post = (pass == 1 && mode == GRAM_RIGHT && tcond > 0.0 && base.nr == 1 && base.nl <= 1);
    bool f32 = false;
    int zr, zc;
    int gnwg = 1;
    if (post) {
      Stages s1 = base;
      s1.nr = 0;
      // a triangular F with F^T F = P^T P in place of the left factor P: the
      // same Gram, with the zero half of F skipped
      if (gram_left && s1.nl == 1) s1.L[0] = *gram_left;
      gnwg = gram(h, w.partials, w.G, cvp, s1, mode, pr.mixed, &f32, w.scal + kScalF32);
      qa.Tpost = base.R[0].S;
      qa.tpr = base.R[0].rows;
      qa.tpc = base.R[0].cols;
      qa.tsr = base.R[0].sr;
      qa.tsc = base.R[0].sc;
      qa.cond_scale = tcond;
      chain_flops(cvp, s1, &zr, &zc);
    } else {
      gnwg = gram(h, w.partials, w.G, cvp, st, mode, (pass == 1) ? pr.mixed : 0, &f32, w.scal + kScalF32);
      chain_flops(cvp, st, &zr, &zc);
    }
    ++*passes;
    const double u = f32 ? kU32 : kU64;
    qa.G = w.G;
    qa.d = d;
    qa.pass = pass;
    qa.b = b;
    qa.Rc = Rc;
    qa.Fstep = slot(pass - 1);
    qa.Rnext = R[(pass - 1) & 1];
    qa.Tdst = Tdst;
    qa.dec = w.dec;
    qa.tau1 = pr.mixed ? u / kTauMix : kTau1;
    qa.tau2 = kTau2;
    qa.ugram = u;
    qa.gerr = gram_err(cvp, mode == GRAM_LEFT ? zc : zr, u, gnwg);
    qa.try_chol = 1;
    qa.shift_pass = pr.mixed ? 2 : 1;
    qa.notrunc_check = (tc && tc->check) ? 1 : 0;
    qa.delta_dev = tc ? tc->delta_dev : nullptr;
    qa.first = tc ? tc->first : 0;
    qa.tol2_nm1 = tc ? tc->tol2_nm1 : 0.0;
    {
      ProfScope ps(h, P_SMALL, 0.0, 0.0);
      launch_qr_step(h->stream, qa);
    }
    h->stats.small_launches++;
    int rc = sync_dec(h);
    if (rc) return rc;
    const int k = h->dec_host[0];
    const int done = h->dec_host[1];
    if (pass == 1 && ratio) *ratio = h->decf_host[0];
    if (tc) tc->notrunc = (pass == 1 && done) ? h->dec_host[5] : 0;
    f->tri = (pass == 1 && done) ? h->dec_host[4] : 0;
    f->rorth = (pass == 1 && done) ? h->dec_host[6] : 0;
    f->nst = pass;
    f->dim[pass] = k;
    const bool can_mat = (mode == GRAM_RIGHT) ? (base.nl <= 1 && base.nr <= 1) : (base.nl == 0 && base.nr <= 1);
    if (!done && pass == 1 && mat && base.nl + base.nr > 0 && can_mat) {
      // The first pass did not settle: materialize the base chain once, so
      // that the refinement Gram passes and the output pass read one core
      // and apply the refinement stages to bitwise the same data.
      Stages sb = base;
      apply(h, cv, sb, mat, cv.trans);
      int mr, mc;
      chain_flops(cv, base, &mr, &mc);
      cvp.X = mat;
      cvp.I = cv.I;
      cvp.trans = cv.trans;
      cvp.pa = cv.trans ? mc : mr;
      cvp.pb = cv.trans ? mr : mc;
      st = no_stages();
      if (cv_out) *cv_out = cvp;
      if (materialized) *materialized = 1;
    }
    if (mode == GRAM_LEFT) st.L[st.nl++] = st_trans(qa.Fstep, k, d);
    else st.R[st.nr++] = st_plain(qa.Fstep, d, k);
    Rc = qa.Rnext;
    d = k;
    if (done) {
      *Rout = qa.Rnext;
      *kout = k;
      return TTR_OK;
    }
  }
  return fail(TTR_ERR_NUMERICAL, "QR-by-Gram did not settle in three passes");
}

// Orthonormalization sweep over logical cores N-1..1 (Alg. 1 order), implicit
// factors as in Alg. 6: for each core the stages of B_n and T_n = R_n^T are
// kept in the workspace, k[n] is the rank at logical link n.  When `Out` is
// given, each orthonormal core B_n^T M_n(i) T_{n+1} is written to it (Alg. 5).
int orth_sweep(ttr_handle *h, WS &w, const Seq &S, std::vector<int> &k, std::vector<Factor> &fac, ttr_tt *Out,
               int *passes, std::vector<double> *kappa2 = nullptr, Prec pr = Prec()) {
  const int N = S.N();
  k.assign(N + 1, 1);
  fac.assign(N + 1, Factor());
  if (kappa2) kappa2->assign(N + 1, -1.0);
  for (int n = 0; n <= N; ++n) k[n] = (int)S.rank(n);
  for (int n = N - 1; n >= 1; --n) {
    const CoreView cv = S.view(n);
    const int b = cv.ea();
    Stages base = no_stages();
    if (n < N - 1) base.R[base.nr++] = st_plain(w.T(n + 1), cv.eb(), k[n + 1], fac[n + 1].tri ? 1 : 0);
    double *Rout;
    int kn;
    auto slot = [&](int j) { return w.B(n, j); };
    double ratio = -1.0;
    CoreView cvm;
    int materialized = 0;
    int rc = qr_by_gram(h, w, cv, GRAM_LEFT, base, b, slot, w.T(n), &fac[n], &Rout, &kn, passes, -1.0, &ratio,
                        nullptr, pr, w.matA, &cvm, &materialized);
    if (rc) return rc;
    fac[n].mat = materialized;
    k[n] = kn;
    if (kappa2 && fac[n].nst == 1) (*kappa2)[n] = ratio;
    if (Out) {
      Stages st = no_stages();
      for (int j = 0; j < fac[n].nst; ++j) st.L[st.nl++] = st_trans(w.B(n, j), fac[n].dim[j + 1], fac[n].dim[j]);
      if (n < N - 1 && !materialized) st.R[st.nr++] = st_plain(w.T(n + 1), cv.eb(), k[n + 1]);
      // in place (Out is the source) through scratch, else straight into Out
      const int pn = S.phys(n);
      const bool direct = Out->core[pn] != cv.X;
      apply(h, materialized ? cvm : cv, st, direct ? Out->core[pn] : w.tmp, S.rev);
      if (!direct) launch_copy(h->stream, w.tmp, (long long)kn * cv.I * k[n + 1], Out->core[pn]);
    }
  }
  return TTR_OK;
}

int handle_ok(ttr_handle *h) {
  if (!h) return fail(TTR_ERR_INVALID_ARG, "handle is NULL");
  HIPCHK(hipSetDevice(h->device));
  return TTR_OK;
}

size_t max_core(const ttr_tt *X) {
  size_t m = 0;
  for (int n = 0; n < X->N; ++n) {
    const size_t c = (size_t)X->R[n] * X->I[n] * X->R[n + 1];
    if (c > m) m = c;
  }
  return m;
}

}  // namespace

// The device address of `scratch` on `device` (the current device), looked
// up once per device.
int noalloc_scratch_of(int device, double **out) {
  static std::mutex mu;
  static std::vector<double *> addr;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= device) addr.resize(device + 1, nullptr);
  if (!addr[device]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(TTR_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    addr[device] = static_cast<double *>(p);
  }
  *out = addr[device];
  return TTR_OK;
}

int ttr_dev_alloc(ttr_handle *h, void **p, size_t bytes) {
  *p = nullptr;
  if (h->alloc_fn) {
    *p = h->alloc_fn(bytes, h->alloc_ctx);
  } else if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
  }
  if (!*p) return fail(TTR_ERR_ALLOC, "workspace allocation of " + std::to_string(bytes) + " bytes failed");
  return TTR_OK;
}

void ttr_dev_free(ttr_handle *h, void *p) {
  if (!p) return;
  if (h->free_fn) h->free_fn(p, h->alloc_ctx);
  else (void)hipFree(p);
}

extern "C" {

int ttr_create(ttr_handle **h, int device, void *stream) {
  if (!h) return fail(TTR_ERR_INVALID_ARG, "h is NULL");
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(TTR_ERR_INVALID_ARG, "no such device");
  HIPCHK(hipSetDevice(device));
  ttr_handle *p = new ttr_handle();
  p->device = device;
  p->stream = (hipStream_t)stream;
  std::memset(&p->stats, 0, sizeof(p->stats));
  std::memset(&p->prof, 0, sizeof(p->prof));
  if (hipHostMalloc((void **)&p->dec_host, 16 * sizeof(int)) != hipSuccess ||
      hipHostMalloc((void **)&p->scal_host, 16 * sizeof(double)) != hipSuccess ||
      hipMalloc((void **)&p->dec_dev, 16 * sizeof(int)) != hipSuccess ||
      hipHostMalloc((void **)&p->decf_host, 8 * sizeof(double)) != hipSuccess ||
      hipMalloc((void **)&p->decf_dev, 8 * sizeof(double)) != hipSuccess) {
    delete p;
    return fail(TTR_ERR_ALLOC, "handle allocation failed");
  }
  int rc = noalloc_scratch_of(device, &p->noalloc_scratch);
  if (rc) {
    (void)hipFree(p->dec_dev);
    (void)hipFree(p->decf_dev);
    (void)hipHostFree(p->decf_host);
    (void)hipHostFree(p->dec_host);
    (void)hipHostFree(p->scal_host);
    delete p;
    return rc;
  }
  *h = p;
  return TTR_OK;
}

int ttr_destroy(ttr_handle *h) {
  if (!h) return TTR_OK;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  if (h->ws) ttr_dev_free(h, h->ws);
  if (h->dec_dev) (void)hipFree(h->dec_dev);
  if (h->decf_dev) (void)hipFree(h->decf_dev);
  if (h->decf_host) (void)hipHostFree(h->decf_host);
  if (h->dec_host) (void)hipHostFree(h->dec_host);
  if (h->scal_host) (void)hipHostFree(h->scal_host);
  ttr_batch_release(h);
  ttr_large_release(h);
  for (auto &p : h->pending) {
    h->evpool.push_back(p.a);
    h->evpool.push_back(p.b);
  }
  for (hipEvent_t e : h->evpool) (void)hipEventDestroy(e);
  delete h;
  return TTR_OK;
}

int ttr_set_stream(ttr_handle *h, void *stream) {
  if (!h) return fail(TTR_ERR_INVALID_ARG, "handle is NULL");
  h->stream = (hipStream_t)stream;
  return TTR_OK;
}

int ttr_set_allocator(ttr_handle *h, void *(*alloc)(size_t bytes, void *ctx), void (*dealloc)(void *ptr, void *ctx),
                      void *ctx) {
  if (!h) return fail(TTR_ERR_INVALID_ARG, "handle is NULL");
  if ((alloc == nullptr) != (dealloc == nullptr))
    return fail(TTR_ERR_INVALID_ARG, "alloc and free must both be given or both be NULL");
  HIPCHK(hipSetDevice(h->device));
  HIPCHK(hipStreamSynchronize(h->stream));
  // every workspace goes back to the allocator it came from
  if (h->ws) ttr_dev_free(h, h->ws);
  h->ws = nullptr;
  h->ws_bytes = 0;
  ttr_batch_release(h);
  ttr_large_release(h);
  h->alloc_fn = alloc;
  h->free_fn = dealloc;
  h->alloc_ctx = ctx;
  return TTR_OK;
}

int ttr_add(ttr_handle *h, double alpha, const ttr_tt *X, double beta, const ttr_tt *Y, ttr_tt *Z) {
  int rc;
  if ((rc = handle_ok(h))) return rc;
  if ((rc = check_tt(X, "X", 0))) return rc;
  if ((rc = check_tt(Y, "Y", 0))) return rc;
  if (X->N != Y->N) return fail(TTR_ERR_SHAPE, "X and Y differ in N");
  for (int n = 0; n < X->N; ++n)
    if (X->I[n] != Y->I[n]) return fail(TTR_ERR_SHAPE, "X and Y differ in mode sizes");
  if ((rc = check_out(Z, "Z", X->N, X->I))) return rc;
  const int N = X->N;
  std::vector<int64_t> R(N + 1, 1);
  for (int n = 1; n < N; ++n) R[n] = X->R[n] + Y->R[n];
  for (int n = 0; n < N; ++n) {
    if (Z->core[n] == X->core[n] || Z->core[n] == Y->core[n]) return fail(TTR_ERR_INVALID_ARG, "Z aliases an input");
    if (Z->cap[n] < R[n] * X->I[n] * R[n + 1]) return fail(TTR_ERR_CAPACITY, "Z core capacity too small");
    if (R[n] * X->I[n] >= (int64_t)1 << 31 || R[n + 1] >= 65536)
      return fail(TTR_ERR_UNSUPPORTED, "Z core column above 2^31 entries or rank above 65535");
  }
  for (int n = 0; n < N; ++n) {
    const double bytes = 8.0 * X->I[n] * ((double)X->R[n] * X->R[n + 1] + (double)Y->R[n] * Y->R[n + 1] +
                                         (double)R[n] * R[n + 1]);
    ProfScope ps(h, P_ADD, bytes, 0.0);
    launch_add(h->stream, n, N, alpha, beta, X->core[n], (int)X->R[n], (int)X->R[n + 1], Y->core[n], (int)Y->R[n],
               (int)Y->R[n + 1], X->I[n], Z->core[n]);
  }
  HIPCHK(hipGetLastError());
  for (int n = 0; n <= N; ++n) Z->R[n] = R[n];
  return TTR_OK;
}

int ttr_hadamard(ttr_handle *h, const ttr_tt *X, const ttr_tt *Y, ttr_tt *Z) {
  int rc;
  if ((rc = handle_ok(h))) return rc;
  if ((rc = check_tt(X, "X", 0))) return rc;
  if ((rc = check_tt(Y, "Y", 0))) return rc;
  if (X->N != Y->N) return fail(TTR_ERR_SHAPE, "X and Y differ in N");
  for (int n = 0; n < X->N; ++n)
    if (X->I[n] != Y->I[n]) return fail(TTR_ERR_SHAPE, "X and Y differ in mode sizes");
  if ((rc = check_out(Z, "Z", X->N, X->I))) return rc;
  const int N = X->N;
  std::vector<int64_t> R(N + 1, 1);
  for (int n = 0; n <= N; ++n) R[n] = X->R[n] * Y->R[n];
  for (int n = 0; n < N; ++n) {
    if (Z->core[n] == X->core[n] || Z->core[n] == Y->core[n]) return fail(TTR_ERR_INVALID_ARG, "Z aliases an input");
    if (Z->cap[n] < R[n] * X->I[n] * R[n + 1]) return fail(TTR_ERR_CAPACITY, "Z core capacity too small");
    if (R[n] * X->I[n] >= (int64_t)1 << 31 || R[n + 1] >= 65536)
      return fail(TTR_ERR_UNSUPPORTED, "Z core column above 2^31 entries or rank above 65535");
  }
  for (int n = 0; n < N; ++n) {
    const double zsz = (double)R[n] * R[n + 1] * X->I[n];
    const double bytes = 8.0 * (X->I[n] * ((double)X->R[n] * X->R[n + 1] + (double)Y->R[n] * Y->R[n + 1]) + zsz);
    ProfScope ps(h, P_HAD, bytes, zsz);
    launch_hadamard(h->stream, X->core[n], (int)X->R[n], (int)X->R[n + 1], Y->core[n], (int)Y->R[n],
                    (int)Y->R[n + 1], X->I[n], Z->core[n]);
  }
  HIPCHK(hipGetLastError());
  for (int n = 0; n <= N; ++n) Z->R[n] = R[n];
  return TTR_OK;
}

static bool any_rank_above(const ttr_tt *X, int64_t r) {
  for (int n = 0; n <= X->N; ++n)
    if (X->R[n] > r) return true;
  return false;
}

int ttr_apply_kron(ttr_handle *h, const double *const *A, const int64_t *kl, const int64_t *ku, const ttr_tt *X,
                   ttr_tt *Y) {
  int rc;
  if ((rc = handle_ok(h))) return rc;
  if (!A || !kl || !ku) return fail(TTR_ERR_INVALID_ARG, "A, kl or ku is NULL");
  if ((rc = check_tt(X, "X", 0))) return rc;
  if ((rc = check_out(Y, "Y", X->N, X->I))) return rc;
  const int N = X->N;
  for (int n = 0; n < N; ++n) {
    if (!A[n]) return fail(TTR_ERR_INVALID_ARG, "NULL operator matrix");
    if (kl[n] < 0 || ku[n] < 0 || kl[n] >= X->I[n] || ku[n] >= X->I[n])
      return fail(TTR_ERR_INVALID_ARG, "bandwidths must satisfy 0 <= kl, ku < I_n");
    if (Y->core[n] == X->core[n]) return fail(TTR_ERR_INVALID_ARG, "Y aliases X");
    if (Y->cap[n] < X->R[n] * X->I[n] * X->R[n + 1]) return fail(TTR_ERR_CAPACITY, "Y core capacity too small");
    if (X->R[n] > 4096 || X->R[n + 1] >= 65536 || X->I[n] >= ((int64_t)1 << 40))
      return fail(TTR_ERR_UNSUPPORTED, "rank above 4096 (left) or 65535 (right)");
  }
  for (int n = 0; n < N; ++n) {
    const double elems = (double)X->R[n] * X->I[n] * X->R[n + 1];
    ProfScope ps(h, P_KRON, 16.0 * elems + 8.0 * (double)(kl[n] + ku[n] + 1) * X->I[n],
                 2.0 * elems * (double)(kl[n] + ku[n] + 1));
    launch_kron_apply(h->stream, X->core[n], (int)X->R[n], (int)X->R[n + 1], X->I[n], A[n], (int)kl[n], (int)ku[n],
                      Y->core[n]);
  }
  HIPCHK(hipGetLastError());
  for (int n = 0; n <= N; ++n) Y->R[n] = X->R[n];
  return TTR_OK;
}

int ttr_dot(ttr_handle *h, const ttr_tt *X, const ttr_tt *Y, double *out) {
  int rc;
  if ((rc = handle_ok(h))) return rc;
  if (!out) return fail(TTR_ERR_INVALID_ARG, "out is NULL");
  if ((rc = check_tt(X, "X", TTR_MAX_RANK_LARGE))) return rc;
  if ((rc = check_tt(Y, "Y", TTR_MAX_RANK_LARGE))) return rc;
  if (X->N != Y->N) return fail(TTR_ERR_SHAPE, "X and Y differ in N");
  for (int n = 0; n < X->N; ++n)
    if (X->I[n] != Y->I[n]) return fail(TTR_ERR_SHAPE, "X and Y differ in mode sizes");
  const int N = X->N;
  if (any_rank_above(X, TTR_MAX_RANK) || any_rank_above(Y, TTR_MAX_RANK)) {
    rc = ttr_dot_large(h, X, Y, out);
    prof_resolve(h);
    return rc;
  }
  if ((rc = ensure_ws(h, ws_doubles(N, 0) * sizeof(double)))) return rc;
  WS w = carve(h, N, 0);
  h->scal_host[0] = 1.0;
  HIPCHK(hipMemcpyAsync(w.Wa, h->scal_host, sizeof(double), hipMemcpyHostToDevice, h->stream));
  double *Wp = w.Wa, *Wn = w.Wb;
  for (int n = 0; n < N; ++n) {
    {
      const double rx0 = X->R[n], rx1 = X->R[n + 1], ry0 = Y->R[n], ry1 = Y->R[n + 1];
      ProfScope ps(h, P_DOT, 8.0 * X->I[n] * (rx0 * rx1 + ry0 * ry1),
                   2.0 * X->I[n] * (ry0 * rx0 * rx1 + ry1 * ry0 * rx1));
      const int nwg = launch_dot_mfma(h->stream, X->core[n], (int)X->R[n], (int)X->R[n + 1], Y->core[n],
                                      (int)Y->R[n], (int)Y->R[n + 1], X->I[n], Wp, w.partials);
      launch_reduce(h->stream, w.partials, nwg, (int)(Y->R[n + 1] * X->R[n + 1]), Wn);
    }
    std::swap(Wp, Wn);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(h->scal_host + 1, Wp, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  *out = h->scal_host[1];
  prof_resolve(h);
  return TTR_OK;
}

int ttr_dot_noalloc(ttr_handle *h, const ttr_tt *X, const ttr_tt *Y, double *out_dev) {
  int rc;
  if ((rc = handle_ok(h))) return rc;
  if (!out_dev) return fail(TTR_ERR_INVALID_ARG, "out_dev is NULL");
  if ((rc = check_tt(X, "X", TTR_MAX_RANK))) return rc;
  if ((rc = check_tt(Y, "Y", TTR_MAX_RANK))) return rc;
  if (X->N != Y->N) return fail(TTR_ERR_SHAPE, "X and Y differ in N");
  for (int n = 0; n < X->N; ++n)
    if (X->I[n] != Y->I[n]) return fail(TTR_ERR_SHAPE, "X and Y differ in mode sizes");
  const int N = X->N;
  // every step's partials must fit the fixed scratch (ranks <= 64 always do;
  // checked here so that a change of the launch grid cannot overrun it)
  for (int n = 0; n < N; ++n) {
    const size_t need = (size_t)dot_mfma_workgroups(X->I[n]) * (size_t)(Y->R[n + 1] * X->R[n + 1]);
    if (need > kNoAllocPartials)
      return fail(TTR_ERR_UNSUPPORTED, "ttr_dot_noalloc: partial sums need " + std::to_string(need) +
                                           " doubles, above its fixed scratch of " + std::to_string(kNoAllocPartials));
  }
  double *partials = h->noalloc_scratch;
  double *Wp = partials + kNoAllocPartials, *Wn = Wp + (size_t)TTR_RMAX * TTR_RMAX;
  hipLaunchKernelGGL(k_set_one, dim3(1), dim3(64), 0, h->stream, Wp);
  for (int n = 0; n < N; ++n) {
    const int nwg = launch_dot_mfma(h->stream, X->core[n], (int)X->R[n], (int)X->R[n + 1], Y->core[n], (int)Y->R[n],
                                    (int)Y->R[n + 1], X->I[n], Wp, partials);
    // the last step's 1 x 1 result goes straight to the caller's buffer
    launch_reduce(h->stream, partials, nwg, (int)(Y->R[n + 1] * X->R[n + 1]), n == N - 1 ? out_dev : Wn);
    std::swap(Wp, Wn);
  }
  HIPCHK(hipGetLastError());
  return TTR_OK;
}

int ttr_norm(ttr_handle *h, const ttr_tt *X, int method, double *out) {
  int rc;
  if ((rc = handle_ok(h))) return rc;
  if (!out) return fail(TTR_ERR_INVALID_ARG, "out is NULL");
  if (method == TTR_NORM_GRAM) {
    double v;
    if ((rc = ttr_dot(h, X, X, &v))) return rc;
    *out = v > 0 ? std::sqrt(v) : (v == v ? 0.0 : v);
    return TTR_OK;
  }
  if (method == TTR_NORM_SYM) {
    // W_1 = V(X_1)^T V(X_1); W_n = V(Z_n)^T V(Z_n) with Z_n(i) = F_{n-1} X_n(i)
    // and F_{n-1} upper triangular, F^T F = W_{n-1} (§3.2.4, symmetric form):
    // the streaming Gram kernel skips the zero half of F, the Gram itself is
    // formed on the lower block triangle only
    if ((rc = check_tt(X, "X", TTR_MAX_RANK_LARGE))) return rc;
    if (any_rank_above(X, TTR_MAX_RANK))
      return fail(TTR_ERR_UNSUPPORTED, "TTR_NORM_SYM supports ranks up to TTR_MAX_RANK");
    const int N = X->N;
    if ((rc = ensure_ws(h, ws_doubles(N, 0) * sizeof(double)))) return rc;
    WS w = carve(h, N, 0);
    const Seq S{X, 0};
    double *Fbuf[2] = {w.Pa, w.Pb};
    for (int n = 0; n < N; ++n) {
      const CoreView cv = S.view(n);
      Stages st = no_stages();
      if (n > 0) st.L[st.nl++] = st_plain(Fbuf[(n - 1) & 1], cv.pa, cv.pa, 2);
      gram(h, w.partials, w.G, cv, st, GRAM_RIGHT);
      if (n + 1 < N) launch_sym_factor(h->stream, w.G, cv.pb, Fbuf[n & 1]);
    }
    launch_sqrt_scalar(h->stream, w.G, w.scal);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(h->scal_host, w.scal, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    *out = h->scal_host[0];
    prof_resolve(h);
    return TTR_OK;
  }
  if (method != TTR_NORM_ORTHO) return fail(TTR_ERR_INVALID_ARG, "unknown norm method");
  if ((rc = check_tt(X, "X", TTR_MAX_RANK_LARGE))) return rc;
  const int N = X->N;
  if (any_rank_above(X, TTR_MAX_RANK)) {
    if ((rc = reset_dec(h))) return rc;
    rc = ttr_norm_ortho_large(h, X, out);
    prof_resolve(h);
    return rc;
  }
  const size_t mat = max_core(X);
  if ((rc = ensure_ws(h, ws_doubles(N, 0, mat) * sizeof(double)))) return rc;
  WS w = carve(h, N, 0, mat);
  if ((rc = reset_dec(h))) return rc;
  Seq S{X, 0};
  std::vector<int> k;
  std::vector<Factor> fac;
  int passes = 0;
  if ((rc = orth_sweep(h, w, S, k, fac, nullptr, &passes))) return rc;
  // ||X|| = ||C_1||_F with C_1(i) = X_1(i) T_2 (end of §2.3)
  const CoreView cv = S.view(0);
  Stages st = no_stages();
  if (N > 1) st.R[st.nr++] = st_plain(w.T(1), cv.eb(), k[1]);
  gram(h, w.partials, w.G, cv, st, GRAM_LEFT);
  launch_sqrt_scalar(h->stream, w.G, w.scal);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(h->scal_host, w.scal, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  *out = h->scal_host[0];
  prof_resolve(h);
  return TTR_OK;
}

int ttr_orthogonalize(ttr_handle *h, ttr_tt *X, int side, int prec) {
  int rc;
  if ((rc = handle_ok(h))) return rc;
  if (side != TTR_RIGHT && side != TTR_LEFT) return fail(TTR_ERR_INVALID_ARG, "side must be TTR_RIGHT or TTR_LEFT");
  if (prec != TTR_FP64) return fail(TTR_ERR_INVALID_ARG, "ttr_orthogonalize supports TTR_FP64");
  if ((rc = check_tt(X, "X", TTR_MAX_RANK_LARGE))) return rc;
  const int N = X->N;
  if (N == 1) return TTR_OK;
  if (any_rank_above(X, TTR_MAX_RANK)) {
    if ((rc = reset_dec(h))) return rc;
    rc = ttr_orthogonalize_large(h, X, side);
    prof_resolve(h);
    return rc;
  }
  const size_t tmp = max_core(X);
  if ((rc = ensure_ws(h, ws_doubles(N, tmp, tmp) * sizeof(double)))) return rc;
  WS w = carve(h, N, tmp, tmp);
  if ((rc = reset_dec(h))) return rc;
  Seq S{X, side == TTR_LEFT};
  std::vector<int> k;
  std::vector<Factor> fac;
  int passes = 0;
  if ((rc = orth_sweep(h, w, S, k, fac, X, &passes))) return rc;
  // the first logical core absorbs T_2: C_1(i) = M_1(i) T_2
  const CoreView cv = S.view(0);
  Stages st = no_stages();
  st.R[st.nr++] = st_plain(w.T(1), cv.eb(), k[1]);
  apply(h, cv, st, w.tmp, S.rev);
  launch_copy(h->stream, w.tmp, (long long)cv.I * k[1], X->core[S.phys(0)]);
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipGetLastError());
  for (int l = 0; l <= N; ++l) {
    const int pl = S.rev ? N - l : l;
    X->R[pl] = k[l];
  }
  prof_resolve(h);
  return TTR_OK;
}

}  // extern "C"

namespace {

// Rounding with explicit orthonormal factors (the explicit variant of
// §4.3.2, the orthonormalization of §3.4 Alg. 5): Y <- X, Y is orthonormalized
// in place with its cores written (right for RLR, left for LRL), then the
// truncation sweep of Alg. 2 runs over the written cores, C'_n(i) = P_n Y_n(i)
// with no factor of the first sweep left to apply.  Ranks <= 64.
int round_explicit_small(ttr_handle *h, const ttr_tt *X, double tol, int rev, int prec, ttr_tt *Y, double *norm_out) {
  const int N = X->N;
  int rc;
  for (int n = 0; n < N; ++n) Y->R[n] = X->R[n];
  Y->R[N] = 1;
  const size_t tmp = max_core(X);
  if ((rc = ensure_ws(h, ws_doubles(N, tmp, tmp) * sizeof(double)))) return rc;
  WS w = carve(h, N, tmp, tmp);
  if ((rc = reset_dec(h))) return rc;
  Prec pr;
  pr.mixed = (prec == TTR_MIXED);
  const Seq SX{X, rev};
  const Seq S{Y, rev};
  std::vector<int> k;
  std::vector<Factor> fac;
  int passes = 0, applies = 0;
  // sweep 1: the orthonormal cores of X written into Y (the first core
  // absorbs T_2); X is only read
  if ((rc = orth_sweep(h, w, SX, k, fac, Y, &passes, nullptr, pr))) return rc;
  {
    const CoreView cv = SX.view(0);
    Stages st = no_stages();
    st.R[st.nr++] = st_plain(w.T(1), cv.eb(), k[1]);
    apply(h, cv, st, Y->core[S.phys(0)], S.rev);
    ++applies;
  }
  for (int l = 0; l <= N; ++l) Y->R[rev ? N - l : l] = k[l];
  // sweep 2: truncation over the written cores
  std::vector<int> L(N + 1, 1), sweeps(N, 0);
  double *Pbuf[2] = {w.Pa, w.Pb};
  const double *Pcur = nullptr;
  int Lprev = 1;
  for (int n = 0; n < N - 1; ++n) {
    const CoreView cv = S.view(n);
    const int b = cv.eb();
    Stages base = no_stages();
    if (n > 0) base.L[base.nl++] = st_plain(Pcur, Lprev, cv.ea());
    double *Rq;
    int kq;
    Factor g;
    auto slot = [&](int j) { return w.Gst[j]; };
    TruncCtx tcx;
    tcx.check = 1;
    tcx.delta_dev = w.scal + 1;
    tcx.first = (n == 0);
    tcx.tol2_nm1 = tol * tol / (double)(N - 1);
    CoreView cvm;
    int materialized = 0;
    if ((rc = qr_by_gram(h, w, cv, GRAM_RIGHT, base, b, slot, nullptr, &g, &Rq, &kq, &passes, -1.0, nullptr, &tcx, pr,
                         w.matA, &cvm, &materialized)))
      return rc;
    // the next core's orthonormal factor is written into it: Fn = I (b x b)
    double *Id = w.Wb;
    {
      std::vector<double> id((size_t)b * b, 0.0);
      for (int j = 0; j < b; ++j) id[(size_t)j * b + j] = 1.0;
      HIPCHK(hipMemcpy(Id, id.data(), id.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    TruncArgs ta;
    ta.R = Rq;
    ta.k = kq;
    ta.b = b;
    ta.Glast = w.Gst[g.nst - 1];
    ta.d = g.dim[g.nst - 1];
    ta.Fn = Id;
    ta.dn = b;
    ta.GU = w.GU;
    ta.Pnext = Pbuf[n & 1];
    ta.delta = w.scal + 1;
    ta.norm = w.scal + 2;
    ta.first = (n == 0);
    ta.tol = tol;
    ta.Nm1 = N - 1;
    ta.sigma_out = w.sigma + (size_t)n * TTR_RMAX;
    ta.tail_out = w.tails + n;
    ta.dec = w.dec;
    ta.identity = tcx.notrunc;
    ta.r_orth = (g.nst == 1 && !tcx.notrunc && g.rorth) ? 1 : 0;
    {
      ProfScope ps(h, P_SMALL, 0.0, 0.0);
      launch_trunc_step(h->stream, ta);
    }
    h->stats.small_launches++;
    if ((rc = sync_dec(h))) return rc;
    const int Ln = h->dec_host[3];
    L[n + 1] = Ln;
    sweeps[n] = h->dec_host[9];
    Stages st = materialized ? no_stages() : base;
    for (int j = 0; j + 1 < g.nst; ++j) st.R[st.nr++] = st_plain(w.Gst[j], g.dim[j], g.dim[j + 1]);
    st.R[st.nr++] = st_plain(w.GU, ta.d, Ln);
    apply(h, materialized ? cvm : cv, st, w.tmp, S.rev);
    const int zr = (n > 0) ? Lprev : cv.ea();
    launch_copy(h->stream, w.tmp, (long long)zr * cv.I * Ln, Y->core[S.phys(n)]);
    ++applies;
    Pcur = ta.Pnext;
    Lprev = Ln;
  }
  {
    const int n = N - 1;
    const CoreView cv = S.view(n);
    Stages st = no_stages();
    st.L[st.nl++] = st_plain(Pcur, Lprev, cv.ea());
    apply(h, cv, st, w.tmp, S.rev);
    launch_copy(h->stream, w.tmp, (long long)Lprev * cv.I * cv.eb(), Y->core[S.phys(n)]);
    ++applies;
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(h->scal_host, w.scal, 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  const int nsig = (N - 1) * TTR_RMAX;
  std::vector<double> sig(nsig), tails(N - 1);
  HIPCHK(hipMemcpyAsync(sig.data(), w.sigma, nsig * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(tails.data(), w.tails, (N - 1) * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipGetLastError());
  for (int l = 0; l <= N; ++l) Y->R[rev ? N - l : l] = (l == 0 || l == N) ? 1 : L[l];
  h->stats.gram_passes = passes;
  h->stats.apply_passes = applies;
  h->stats.links = N - 1;
  h->stats.norm = h->scal_host[2];
  h->stats.delta = h->scal_host[1];
  for (int l = 0; l < N - 1; ++l) {
    const int pl = rev ? (N - 1 - l) - 1 : l;
    if (pl >= TTR_STATS_LINKS) continue;
    int cnt = 0;
    for (int j = 0; j < TTR_RMAX; ++j) {
      h->stats.sigma[(size_t)pl * TTR_STATS_SIGMA + j] = sig[(size_t)l * TTR_RMAX + j];
      if (sig[(size_t)l * TTR_RMAX + j] > 0) cnt = j + 1;
    }
    h->stats.nsigma[pl] = cnt;
    h->stats.tail2[pl] = tails[l];
    h->stats.sweeps[pl] = sweeps[l];
  }
  if (norm_out) *norm_out = h->scal_host[2];
  prof_resolve(h);
  return TTR_OK;
}

}  // namespace

extern "C" {

int ttr_round(ttr_handle *h, const ttr_tt *X, double tol, int direction, int prec, ttr_tt *Y, double *norm_out) {
  int rc;
  if ((rc = handle_ok(h))) return rc;
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(TTR_ERR_INVALID_ARG, "tol must be finite and >= 0");
  if (direction != TTR_RLR && direction != TTR_LRL && direction != TTR_RLR_EXPLICIT && direction != TTR_LRL_EXPLICIT)
    return fail(TTR_ERR_INVALID_ARG, "unknown direction");
  const int explicit_f = (direction == TTR_RLR_EXPLICIT || direction == TTR_LRL_EXPLICIT);
  direction = (direction == TTR_LRL || direction == TTR_LRL_EXPLICIT) ? TTR_LRL : TTR_RLR;
  if (prec != TTR_FP64 && prec != TTR_MIXED) return fail(TTR_ERR_INVALID_ARG, "unknown precision");
  if ((rc = check_tt(X, "X", TTR_MAX_RANK_LARGE))) return rc;
  if ((rc = check_out(Y, "Y", X->N, X->I))) return rc;
  const int N = X->N;
  int64_t rmax = 1;
  for (int n = 0; n < N; ++n) {
    if (Y->core[n] == X->core[n]) return fail(TTR_ERR_INVALID_ARG, "Y aliases X");
    if (Y->cap[n] < X->R[n] * X->I[n] * X->R[n + 1]) return fail(TTR_ERR_CAPACITY, "Y core capacity too small");
    rmax = std::max(rmax, X->R[n + 1]);
  }
  std::memset(&h->stats, 0, sizeof(h->stats));
  if (rmax > TTR_MAX_RANK && N > 1) {
    // ranks above the register-tiled kernels' range: the unfolding-based path
    if ((rc = reset_dec(h))) return rc;
    rc = ttr_round_large(h, X, tol, direction, prec, explicit_f, Y, norm_out);
    prof_resolve(h);
    return rc;
  }
  if (explicit_f && N > 1) return round_explicit_small(h, X, tol, direction == TTR_LRL, prec, Y, norm_out);
  if (N == 1) {
    HIPCHK(hipMemcpyAsync(Y->core[0], X->core[0], (size_t)X->I[0] * sizeof(double), hipMemcpyDeviceToDevice,
                          h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    Y->R[0] = Y->R[1] = 1;
    if (norm_out) *norm_out = NAN;
    return TTR_OK;
  }
  // scratch for one materialized core of the truncation sweep (L_{n-1} x I_n x R_n <= R_{n-1} I_n R_n)
  const size_t mat = max_core(X);
  if ((rc = ensure_ws(h, ws_doubles(N, 0, mat) * sizeof(double)))) return rc;
  WS w = carve(h, N, 0, mat);
  if ((rc = reset_dec(h))) return rc;
  const Seq S{X, direction == TTR_LRL};
  Prec pr;
  pr.mixed = (prec == TTR_MIXED);
  std::vector<int> k;
  std::vector<Factor> fac;
  std::vector<double> kappa2;
  int passes = 0;
  // Sweep 1: orthonormalization with implicit factors (Alg. 6, first loop).
  if ((rc = orth_sweep(h, w, S, k, fac, nullptr, &passes, &kappa2, pr))) return rc;
  // Sweep 2: truncation (Alg. 2 loop / Alg. 6 second loop).  The current core
  // n is C'_n(i) = [P_n B_n^T] M_n(i) T_{n+1}; its left stages are the
  // orthonormalization stages of core n with the last one merged into P_n.
  std::vector<int> L(N + 1, 1), sweeps(N, 0);
  double *Pbuf[2] = {w.Pa, w.Pb};
  // F (upper triangular, F^T F = P^T P) for the next link's first Gram pass
  Stage fp_stage{};
  bool have_fp = false;
  const double *Pcur = nullptr;  // merged last left stage (Lprev x dim)
  int Lprev = 1;
  int applies = 0;
  for (int n = 0; n < N - 1; ++n) {
    CoreView cv = S.view(n);
    const int tr = cv.eb();  // rows of T_{n+1}
    const int b = k[n + 1];  // columns of A = V(C'_n)
    Stages base = no_stages();
    if (n > 0) {
      const Factor &f = fac[n];
      for (int j = 0; j + 1 < f.nst; ++j) base.L[base.nl++] = st_trans(w.B(n, j), f.dim[j + 1], f.dim[j]);
      base.L[base.nl++] = st_plain(Pcur, Lprev, f.dim[f.nst - 1]);
    }
    base.R[base.nr++] = st_plain(w.T(n + 1), tr, b);
    // T folded into the chain already: the core was materialized in sweep 1
    bool tfold = false;
    if (fac[n].mat) {
      // sweep 1 refined this core on C_n = M_n T_{n+1}: rebuild C_n bitwise as
      // it was (same kernel, same inputs), then C'_n = lefts C_n, so that this
      // sweep applies the refinement stages to the data they were measured on
      Stages s1 = no_stages();
      s1.R[s1.nr++] = base.R[0];
      apply(h, cv, s1, w.matA, cv.trans);
      CoreView cva = cv;
      cva.X = w.matA;
      if (cv.trans) cva.pa = b; else cva.pb = b;
      Stages s2 = no_stages();
      for (int j = 0; j < base.nl; ++j) s2.L[s2.nl++] = base.L[j];
      apply(h, cva, s2, w.matB, cv.trans);
      int zr, zc;
      chain_flops(cva, s2, &zr, &zc);
      cv.X = w.matB;
      cv.pa = cv.trans ? zc : zr;
      cv.pb = cv.trans ? zr : zc;
      base = no_stages();
      tfold = true;
    }
    double *Rq;
    int kq;
    Factor g;
    auto slot = [&](int j) { return w.Gst[j]; };
    const double tcond = (fac[n + 1].nst == 1 && !tfold) ? kappa2[n + 1] : -1.0;
    TruncCtx tcx;
    tcx.check = 1;
    tcx.delta_dev = w.scal + 1;
    tcx.first = (n == 0);
    tcx.tol2_nm1 = tol * tol / (double)(N - 1);
    CoreView cvm;
    int materialized = 0;
    rc = qr_by_gram(h, w, cv, GRAM_RIGHT, base, b, slot, nullptr, &g, &Rq, &kq, &passes, tcond, nullptr, &tcx, pr,
                    tfold ? nullptr : w.matA, &cvm, &materialized, have_fp ? &fp_stage : nullptr);
    if (rc) return rc;
    const Factor &fn = fac[n + 1];
    TruncArgs ta;
    ta.R = Rq;
    ta.k = kq;
    ta.b = b;
    ta.Glast = w.Gst[g.nst - 1];
    ta.d = g.dim[g.nst - 1];
    ta.Fn = w.B(n + 1, fn.nst - 1);
    ta.dn = fn.dim[fn.nst - 1];
    ta.GU = w.GU;
    ta.Pnext = Pbuf[n & 1];
    ta.delta = w.scal + 1;
    ta.norm = w.scal + 2;
    ta.first = (n == 0);
    ta.tol = tol;
    ta.Nm1 = N - 1;
    ta.sigma_out = w.sigma + (size_t)n * TTR_RMAX;
    ta.tail_out = w.tails + n;
    ta.dec = w.dec;
    ta.identity = tcx.notrunc;              // proved L = k: no SVD needed
    ta.r_orth = (g.nst == 1 && !tcx.notrunc && g.rorth) ? 1 : 0;  // one-pass eigen route: R = t^{1/2} W^T
    {
      ProfScope ps(h, P_SMALL, 0.0, 0.0);
      launch_trunc_step(h->stream, ta);
    }
    h->stats.small_launches++;
    if ((rc = sync_dec(h))) return rc;
    const int Ln = h->dec_host[3];
    L[n + 1] = Ln;
    sweeps[n] = h->dec_host[9];
    // The next link's first Gram pass, sum_i (P M_i)^T (P M_i), is the same
    // with any F of F^T F = P^T P in place of P: the upper-triangular F of
    // the symmetric-norm factorization skips half of the product's k-steps.
    // (FP64 only: the FP32 pass is bound by its loads, not its products.)
    have_fp = false;
    if (!pr.mixed && n + 1 < N - 1 && fac[n + 1].nst == 1 && !fac[n + 1].mat && Ln <= ta.dn) {
      launch_ptp(h->stream, ta.Pnext, Ln, ta.dn, w.G);
      launch_sym_factor(h->stream, w.G, ta.dn, w.Fp);
      fp_stage.S = w.Fp;
      fp_stage.rows = Ln;  // rows past the rank of P are zero
      fp_stage.cols = ta.dn;
      fp_stage.sr = 1;
      fp_stage.sc = ta.dn;
      fp_stage.lower = 2;  // upper triangular
      have_fp = true;
    }
    // output core n: the same staged chain as the Gram passes, the last
    // refinement stage merged with U_R[:, :L]
    Stages st = materialized ? no_stages() : base;
    if (g.nst == 1 && tfold) {
      st.R[st.nr++] = st_plain(w.GU, ta.d, Ln);
    } else if (g.nst == 1) {
      // one-pass factorization: T and U-hat merge into one right factor
      launch_small_gemm(h->stream, w.T(n + 1), w.GU, w.Gst[1], tr, b, Ln);
      st.nr = 0;
      st.R[st.nr++] = st_plain(w.Gst[1], tr, Ln);
    } else {
      for (int j = 0; j + 1 < g.nst; ++j) st.R[st.nr++] = st_plain(w.Gst[j], g.dim[j], g.dim[j + 1]);
      st.R[st.nr++] = st_plain(w.GU, ta.d, Ln);
    }
    apply(h, materialized ? cvm : cv, st, Y->core[S.phys(n)], S.rev);
    ++applies;
    Pcur = ta.Pnext;
    Lprev = Ln;
  }
  {
    const int n = N - 1;
    const CoreView cv = S.view(n);
    const Factor &f = fac[n];
    Stages st = no_stages();
    for (int j = 0; j + 1 < f.nst; ++j) st.L[st.nl++] = st_trans(w.B(n, j), f.dim[j + 1], f.dim[j]);
    st.L[st.nl++] = st_plain(Pcur, Lprev, f.dim[f.nst - 1]);
    apply(h, cv, st, Y->core[S.phys(n)], S.rev);
    ++applies;
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(h->scal_host, w.scal, 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  const int nsig = (N - 1) * TTR_RMAX;
  std::vector<double> sig(nsig);
  HIPCHK(hipMemcpyAsync(sig.data(), w.sigma, nsig * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  std::vector<double> tails(N - 1);
  HIPCHK(hipMemcpyAsync(tails.data(), w.tails, (N - 1) * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipGetLastError());
  for (int l = 0; l <= N; ++l) {
    const int pl = S.rev ? N - l : l;
    Y->R[pl] = (l == 0 || l == N) ? 1 : L[l];
  }
  h->stats.gram_passes = passes;
  h->stats.apply_passes = applies;
  h->stats.links = N - 1;
  h->stats.norm = h->scal_host[2];
  h->stats.delta = h->scal_host[1];
  for (int l = 0; l < N - 1; ++l) {
    // logical link l+1; stats are reported in physical link order, for the
    // first TTR_STATS_LINKS physical links
    const int pl = S.rev ? (N - 1 - l) - 1 : l;
    if (pl >= TTR_STATS_LINKS) continue;
    int cnt = 0;
    for (int j = 0; j < TTR_RMAX; ++j) {
      h->stats.sigma[(size_t)pl * TTR_STATS_SIGMA + j] = sig[(size_t)l * TTR_RMAX + j];
      if (sig[(size_t)l * TTR_RMAX + j] > 0) cnt = j + 1;
    }
    h->stats.nsigma[pl] = cnt;
    h->stats.tail2[pl] = tails[l];
    h->stats.sweeps[pl] = sweeps[l];
  }
  if (norm_out) *norm_out = h->scal_host[2];
  prof_resolve(h);
  return TTR_OK;
}

int ttr_round_hadamard(ttr_handle *h, const ttr_tt *A, const ttr_tt *B, double tol, int direction, int prec,
                       ttr_tt *Y, double *norm_out) {
  int rc;
  if ((rc = handle_ok(h))) return rc;
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(TTR_ERR_INVALID_ARG, "tol must be finite and >= 0");
  if (prec != TTR_FP64 && prec != TTR_MIXED) return fail(TTR_ERR_INVALID_ARG, "unknown precision");
  if (direction != TTR_RLR) return fail(TTR_ERR_UNSUPPORTED, "ttr_round_hadamard supports TTR_RLR");
  if ((rc = check_tt(A, "A", 16))) return rc;
  if ((rc = check_tt(B, "B", 16))) return rc;
  if (A->N != B->N) return fail(TTR_ERR_SHAPE, "A and B differ in N");
  for (int n = 0; n < A->N; ++n)
    if (A->I[n] != B->I[n]) return fail(TTR_ERR_SHAPE, "A and B differ in mode sizes");
  if ((rc = check_out(Y, "Y", A->N, A->I))) return rc;
  const int N = A->N;
  for (int n = 0; n < N; ++n) {
    const int64_t need = A->R[n] * B->R[n] * A->I[n] * A->R[n + 1] * B->R[n + 1];
    if (Y->cap[n] < need) return fail(TTR_ERR_CAPACITY, "Y core capacity too small");
    if (Y->core[n] == A->core[n] || Y->core[n] == B->core[n]) return fail(TTR_ERR_INVALID_ARG, "Y aliases A or B");
  }
  std::memset(&h->stats, 0, sizeof(h->stats));
  if (N == 1) {
    // a single core: the product itself
    launch_hadamard(h->stream, A->core[0], 1, 1, B->core[0], 1, 1, A->I[0], Y->core[0]);
    HIPCHK(hipStreamSynchronize(h->stream));
    HIPCHK(hipGetLastError());
    Y->R[0] = Y->R[1] = 1;
    if (norm_out) *norm_out = NAN;
    return TTR_OK;
  }
  if ((rc = reset_dec(h))) return rc;
  rc = ttr_round_hadamard_large(h, A, B, tol, prec, Y, norm_out);
  prof_resolve(h);
  return rc;
}

const char *ttr_status_string(int status) {
  switch (status) {
    case TTR_OK: return "ok";
    case TTR_ERR_INVALID_ARG: return "invalid argument";
    case TTR_ERR_SHAPE: return "shape mismatch";
    case TTR_ERR_CAPACITY: return "output capacity too small";
    case TTR_ERR_ALLOC: return "allocation failed";
    case TTR_ERR_HIP: return "HIP runtime error";
    case TTR_ERR_NUMERICAL: return "numerical failure";
    case TTR_ERR_UNSUPPORTED: return "unsupported size";
    default: return "unknown status";
  }
}

const char *ttr_last_error(void) { return g_err.c_str(); }

int ttr_set_profiling(ttr_handle *h, int on) {
  if (!h) return fail(TTR_ERR_INVALID_ARG, "handle is NULL");
  prof_resolve(h);
  h->profiling = on ? 1 : 0;
  std::memset(&h->prof, 0, sizeof(h->prof));
  return TTR_OK;
}

int ttr_get_profile(ttr_handle *h, ttr_profile *out) {
  if (!h || !out) return fail(TTR_ERR_INVALID_ARG, "NULL argument");
  prof_resolve(h);
  *out = h->prof;
  return TTR_OK;
}

int ttr_get_round_stats(const ttr_handle *h, ttr_round_stats *out) {
  if (!h || !out) return fail(TTR_ERR_INVALID_ARG, "NULL argument");
  *out = h->stats;
  return TTR_OK;
}

}  // extern "C"
