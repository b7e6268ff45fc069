// Host-side definitions shared by the C ABI (ttr_api.hip) and the batched
// rounding (ttr_batch.hip).
#pragma once

#include "../../include/ttr.h"
#include "ttr_internal.h"

#include <string>
#include <vector>

struct BatchPlan;  // ttr_batch.hip
struct LargeCtx;   // ttr_large.hip

struct ttr_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  double *ws = nullptr;
  size_t ws_bytes = 0;
  int *dec_host = nullptr;  // pinned
  int *dec_dev = nullptr;
  double *decf_host = nullptr;  // pinned: per-step doubles (conditioning ratio)
  double *decf_dev = nullptr;
  double *scal_host = nullptr;  // pinned scalars
  ttr_round_stats stats;
  // opt-in kernel timing
  struct Pending {
    hipEvent_t a, b;
    int cls;
    double bytes, flops;
  };
  int profiling = 0;
  std::vector<hipEvent_t> evpool;
  std::vector<Pending> pending;
  ttr_profile prof;
  // batched rounding: the cached plan (workspace, item lists, captured graph)
  BatchPlan *plan = nullptr;
  // ranks above 64: library handle and workspace of the GEMM-based path
  LargeCtx *large = nullptr;
  // caller-registered device allocator for the workspaces (ttr_set_allocator);
  // nullptr: hipMalloc / hipFree
  void *(*alloc_fn)(size_t, void *) = nullptr;
  void (*free_fn)(void *, void *) = nullptr;
  void *alloc_ctx = nullptr;
  // this device's copy of the fixed scratch array of ttr_dot_noalloc (its
  // address from hipGetSymbolAddress, taken in ttr_create)
  double *noalloc_scratch = nullptr;
};

// Workspace memory through the handle's allocator: TTR_OK, or TTR_ERR_ALLOC
// with the message recorded.
int ttr_dev_alloc(ttr_handle *h, void **p, size_t bytes);
void ttr_dev_free(ttr_handle *h, void *p);

// Records `msg` for ttr_last_error() and returns `code`.
int ttr_fail(int code, const std::string &msg);
// Frees the batched plan of a handle (ttr_destroy).
void ttr_batch_release(ttr_handle *h);
// Frees the large-rank path's resources of a handle (ttr_destroy).
void ttr_large_release(ttr_handle *h);
// Ranks 65..256 (ttr_large.hip): rounding (RLR or LRL, FP64 or mixed),
// in-place orthonormalization, the orthonormalization norm and the inner
// product.  Arguments are checked by the callers.
int ttr_round_large(ttr_handle *h, const ttr_tt *X, double tol, int direction, int prec, int explicit_factors,
                    ttr_tt *Y, double *norm_out);
int ttr_orthogonalize_large(ttr_handle *h, ttr_tt *X, int side);
int ttr_norm_ortho_large(ttr_handle *h, const ttr_tt *X, double *out);
int ttr_dot_large(ttr_handle *h, const ttr_tt *X, const ttr_tt *Y, double *out);
int ttr_round_hadamard_large(ttr_handle *h, const ttr_tt *A, const ttr_tt *B, double tol, int prec, ttr_tt *Y,
                             double *norm_out);

#define TTR_HIPCHK(expr)                                                                              \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess) return ttr_fail(TTR_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)
