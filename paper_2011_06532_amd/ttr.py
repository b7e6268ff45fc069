"""Python binding of libttr (ctypes).  Argument marshalling only: every step of
the TT path runs in the library's HIP kernels; torch provides device memory and
the current HIP stream.

A :class:`TT` holds one torch float64 tensor per core on a CUDA (HIP) device,
each a flat buffer in the paper's core layout (entry (a, i, b) of an
R_{n-1} x I_n x R_n core at a + R_{n-1}(i + I_n b)), plus the host-side mode
sizes and ranks.  Output tensors are allocated here with the capacity the call
needs; the library writes the ranks it produced.
"""

from __future__ import annotations

import ctypes
import math
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libttr.so")

TTR_OK = 0
TTR_RIGHT, TTR_LEFT = 0, 1
TTR_RLR, TTR_LRL = 0, 1
TTR_NORM_ORTHO, TTR_NORM_GRAM, TTR_NORM_SYM = 0, 1, 2
TTR_FP64, TTR_MIXED = 0, 1
TTR_MAX_RANK = 64
TTR_STATS_LINKS, TTR_STATS_SIGMA = 64, 256
TTR_ERR_NUMERICAL = 6

_DIR = {"RLR": TTR_RLR, "LRL": TTR_LRL, "RLR_EXPLICIT": 2, "LRL_EXPLICIT": 3}
_SIDE = {"right": TTR_RIGHT, "left": TTR_LEFT}
_NORM = {"ortho": TTR_NORM_ORTHO, "gram": TTR_NORM_GRAM, "sym": TTR_NORM_SYM}
_PREC = {"fp64": TTR_FP64, "mixed": TTR_MIXED}

# exported symbols the header declares (checked by the CPU test suite)
SYMBOLS = [
    "ttr_create", "ttr_destroy", "ttr_set_stream", "ttr_add", "ttr_hadamard", "ttr_dot", "ttr_norm",
    "ttr_orthogonalize", "ttr_round", "ttr_status_string", "ttr_last_error", "ttr_get_round_stats",
    "ttr_set_profiling", "ttr_get_profile", "ttr_round_batched", "ttr_get_batch_plan", "ttr_set_allocator",
    "ttr_dot_noalloc", "ttr_apply_kron", "ttr_round_hadamard",
]

# ttr_set_allocator callback types: void *alloc(size_t bytes, void *ctx), void free(void *ptr, void *ctx)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

PROF_CLASSES = ["k_gram_right_factor", "k_gram_left_factor", "k_gram", "k_apply_mfma", "k_apply", "k_add",
                "k_hadamard", "k_dot", "small", "k_gram_fac", "k_apply_fac2", "k_gram_right_factor_f32",
                "k_gram_left_factor_f32", "k_kron_apply"]
NPROF = len(PROF_CLASSES)  # TTR_NPROF


class _TTStruct(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int32),
        ("I", ctypes.POINTER(ctypes.c_int64)),
        ("R", ctypes.POINTER(ctypes.c_int64)),
        ("core", ctypes.POINTER(ctypes.c_void_p)),
        ("cap", ctypes.POINTER(ctypes.c_int64)),
    ]


class BatchPlan(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_int32),
        ("spw_target", ctypes.c_int32),
        ("grid_cap", ctypes.c_int32),
        ("graph_nodes", ctypes.c_int32),
        ("workspace_bytes", ctypes.c_int64),
        ("candidates", ctypes.c_int32),
        ("cand_spw", ctypes.c_int32 * 16),
        ("cand_grid", ctypes.c_int32 * 16),
        ("cand_ms", ctypes.c_double * 16),
    ]


class RoundStats(ctypes.Structure):
    _fields_ = [
        ("gram_passes", ctypes.c_int32),
        ("apply_passes", ctypes.c_int32),
        ("small_launches", ctypes.c_int32),
        ("links", ctypes.c_int32),
        ("norm", ctypes.c_double),
        ("delta", ctypes.c_double),
        ("sigma", ctypes.c_double * (TTR_STATS_LINKS * TTR_STATS_SIGMA)),
        ("nsigma", ctypes.c_int32 * TTR_STATS_LINKS),
        ("tail2", ctypes.c_double * TTR_STATS_LINKS),
        ("sweeps", ctypes.c_int32 * TTR_STATS_LINKS),
    ]


class Profile(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_int64 * NPROF),
        ("ms", ctypes.c_double * NPROF),
        ("bytes", ctypes.c_double * NPROF),
        ("flops", ctypes.c_double * NPROF),
    ]


_lib = None


class TTRError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libttr error {code}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    """Loads libttr.so; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not built: run `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    tt = P(_TTStruct)
    lib.ttr_create.argtypes = [P(vp), ctypes.c_int, vp]
    lib.ttr_destroy.argtypes = [vp]
    lib.ttr_set_stream.argtypes = [vp, vp]
    lib.ttr_set_allocator.argtypes = [vp, ALLOC_FN, FREE_FN, vp]
    lib.ttr_add.argtypes = [vp, ctypes.c_double, tt, ctypes.c_double, tt, tt]
    lib.ttr_hadamard.argtypes = [vp, tt, tt, tt]
    lib.ttr_dot.argtypes = [vp, tt, tt, P(ctypes.c_double)]
    lib.ttr_dot_noalloc.argtypes = [vp, tt, tt, vp]
    lib.ttr_apply_kron.argtypes = [vp, P(ctypes.c_void_p), P(ctypes.c_int64), P(ctypes.c_int64), tt, tt]
    lib.ttr_round_hadamard.argtypes = [vp, tt, tt, ctypes.c_double, ctypes.c_int, ctypes.c_int, tt,
                                       P(ctypes.c_double)]
    lib.ttr_norm.argtypes = [vp, tt, ctypes.c_int, P(ctypes.c_double)]
    lib.ttr_orthogonalize.argtypes = [vp, tt, ctypes.c_int, ctypes.c_int]
    lib.ttr_round.argtypes = [vp, tt, ctypes.c_double, ctypes.c_int, ctypes.c_int, tt, P(ctypes.c_double)]
    lib.ttr_status_string.argtypes = [ctypes.c_int]
    lib.ttr_status_string.restype = ctypes.c_char_p
    lib.ttr_last_error.argtypes = []
    lib.ttr_last_error.restype = ctypes.c_char_p
    lib.ttr_get_round_stats.argtypes = [vp, P(RoundStats)]
    lib.ttr_set_profiling.argtypes = [vp, ctypes.c_int]
    lib.ttr_get_profile.argtypes = [vp, P(Profile)]
    lib.ttr_round_batched.argtypes = [vp, ctypes.c_int, tt, P(ctypes.c_double), ctypes.c_int, ctypes.c_int, tt,
                                      vp, ctypes.c_int]
    lib.ttr_get_batch_plan.argtypes = [vp, P(BatchPlan)]
    for name in SYMBOLS:
        if name not in ("ttr_status_string", "ttr_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(code: int):
    if code != TTR_OK:
        raise TTRError(code, _lib.ttr_last_error().decode())


class TT:
    """Device-resident TT tensor (torch float64 flat cores)."""

    def __init__(self, cores, I: Sequence[int], R: Sequence[int]):
        self.cores = list(cores)
        self.I = [int(x) for x in I]
        self.R = [int(x) for x in R]

    @property
    def N(self) -> int:
        return len(self.I)

    def nbytes(self) -> int:
        return sum(8 * self.R[n] * self.I[n] * self.R[n + 1] for n in range(self.N))

    @staticmethod
    def empty(I: Sequence[int], caps: Sequence[int], device="cuda"):
        import torch
        cores = [torch.empty(max(int(c), 1), dtype=torch.float64, device=device) for c in caps]
        return TT(cores, I, [1] * (len(I) + 1))

    @staticmethod
    def from_numpy(cores_np: List[np.ndarray], device="cuda"):
        """Copies host cores (any memory order) into device buffers in the core layout."""
        import torch
        cores, R = [], [1]
        for c in cores_np:
            flat = np.asarray(c, dtype=np.float64).reshape(-1, order="F")
            cores.append(torch.from_numpy(np.ascontiguousarray(flat)).to(device))
            R.append(int(c.shape[2]))
        return TT(cores, [int(c.shape[1]) for c in cores_np], R)

    def to_numpy(self) -> List[np.ndarray]:
        out = []
        for n in range(self.N):
            cnt = self.R[n] * self.I[n] * self.R[n + 1]
            flat = self.cores[n][:cnt].detach().cpu().numpy()
            out.append(np.asfortranarray(flat.reshape(self.R[n], self.I[n], self.R[n + 1], order="F")))
        return out

    def slices(self, n: int, idx) -> np.ndarray:
        """Copies slices X_n(i) for the given indices to the host: (len(idx), R_{n-1}, R_n)."""
        import torch
        r0, I, r1 = self.R[n], self.I[n], self.R[n + 1]
        core = self.cores[n][: r0 * I * r1].view(r1, I, r0)  # C-order view of the F-order core
        sel = core[:, torch.as_tensor(list(idx), device=core.device, dtype=torch.long), :]
        return sel.permute(1, 2, 0).contiguous().cpu().numpy()

    def _struct(self, caps: Optional[Sequence[int]] = None):
        N = self.N
        self._I = (ctypes.c_int64 * N)(*self.I)
        self._R = (ctypes.c_int64 * (N + 1))(*self.R)
        self._P = (ctypes.c_void_p * N)(*[c.data_ptr() for c in self.cores])
        cap = caps if caps is not None else [c.numel() for c in self.cores]
        self._C = (ctypes.c_int64 * N)(*[int(x) for x in cap])
        s = _TTStruct(N, self._I, self._R, self._P, self._C)
        self._s = s
        return s

    def _read_ranks(self):
        self.R = [int(self._R[i]) for i in range(self.N + 1)]


class Handle:
    """A libttr handle bound to a device and to torch's current stream."""

    def __init__(self, device: int = 0):
        import torch
        load()
        self.device = device
        self.h = ctypes.c_void_p()
        stream = torch.cuda.current_stream(device).cuda_stream
        _check(_lib.ttr_create(ctypes.byref(self.h), device, ctypes.c_void_p(stream)))

    def sync_stream(self):
        import torch
        _check(_lib.ttr_set_stream(self.h, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)))

    def set_allocator(self, alloc=None, free=None):
        """Workspaces through alloc(nbytes) -> int pointer (0 on failure) and
        free(pointer); both None restores hipMalloc / hipFree."""
        if (alloc is None) != (free is None):
            raise ValueError("give both alloc and free, or neither")
        if alloc is None:
            a, f = ctypes.cast(None, ALLOC_FN), ctypes.cast(None, FREE_FN)
        else:
            a = ALLOC_FN(lambda n, ctx: alloc(int(n)) or None)
            f = FREE_FN(lambda p, ctx: free(int(p)))
        _check(_lib.ttr_set_allocator(self.h, a, f, None))
        self._alloc_cb = (a, f)  # the library keeps the function pointers

    def use_torch_allocator(self):
        """Workspaces from torch's caching allocator (on the current stream)."""
        import torch
        stream = torch.cuda.current_stream(self.device)
        dev = self.device
        self.set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n, dev, stream),
                           torch.cuda.caching_allocator_delete)

    def close(self):
        if self.h:
            _lib.ttr_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- operations ------------------------------------------------------
    def add(self, alpha: float, X: TT, beta: float, Y: TT, out: Optional[TT] = None) -> TT:
        N = X.N
        R = [1] + [X.R[n] + Y.R[n] for n in range(1, N)] + [1]
        caps = [R[n] * X.I[n] * R[n + 1] for n in range(N)]
        Z = out if out is not None else TT.empty(X.I, caps, X.cores[0].device)
        sx, sy, sz = X._struct(), Y._struct(), Z._struct()
        _check(_lib.ttr_add(self.h, alpha, ctypes.byref(sx), beta, ctypes.byref(sy), ctypes.byref(sz)))
        Z._read_ranks()
        return Z

    def hadamard(self, X: TT, Y: TT, out: Optional[TT] = None) -> TT:
        N = X.N
        R = [X.R[n] * Y.R[n] for n in range(N + 1)]
        caps = [R[n] * X.I[n] * R[n + 1] for n in range(N)]
        Z = out if out is not None else TT.empty(X.I, caps, X.cores[0].device)
        sx, sy, sz = X._struct(), Y._struct(), Z._struct()
        _check(_lib.ttr_hadamard(self.h, ctypes.byref(sx), ctypes.byref(sy), ctypes.byref(sz)))
        Z._read_ranks()
        return Z

    def dot(self, X: TT, Y: TT) -> float:
        out = ctypes.c_double()
        sx, sy = X._struct(), Y._struct()
        _check(_lib.ttr_dot(self.h, ctypes.byref(sx), ctypes.byref(sy), ctypes.byref(out)))
        return out.value

    def dot_noalloc(self, X: TT, Y: TT, out=None):
        """<X, Y> into a one-element float64 device tensor, without any
        allocation in the library (ttr_dot_noalloc); asynchronous on the
        handle's stream."""
        import torch
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=X.cores[0].device)
        sx, sy = X._struct(), Y._struct()
        _check(_lib.ttr_dot_noalloc(self.h, ctypes.byref(sx), ctypes.byref(sy), ctypes.c_void_p(out.data_ptr())))
        return out

    def apply_kron(self, A_band, kl, ku, X: TT, out: Optional[TT] = None) -> TT:
        """Y = (A_1 (x) ... (x) A_N) X (ttr_apply_kron).  A_band: N float64
        device tensors in band storage ((kl + ku + 1) x I_n, column-major, i.e.
        torch shape (I_n, kl + ku + 1) row-major); kl, ku: bandwidths."""
        N = X.N
        caps = [X.R[n] * X.I[n] * X.R[n + 1] for n in range(N)]
        Y = out if out is not None else TT.empty(X.I, caps, X.cores[0].device)
        ptrs = (ctypes.c_void_p * N)(*[a.data_ptr() for a in A_band])
        kla = (ctypes.c_int64 * N)(*[int(v) for v in kl])
        kua = (ctypes.c_int64 * N)(*[int(v) for v in ku])
        sx, sy = X._struct(), Y._struct()
        _check(_lib.ttr_apply_kron(self.h, ptrs, kla, kua, ctypes.byref(sx), ctypes.byref(sy)))
        Y._read_ranks()
        return Y

    def norm(self, X: TT, method: str = "ortho") -> float:
        out = ctypes.c_double()
        sx = X._struct()
        _check(_lib.ttr_norm(self.h, ctypes.byref(sx), _NORM[method], ctypes.byref(out)))
        return out.value

    def orthogonalize(self, X: TT, side: str = "right") -> TT:
        sx = X._struct()
        _check(_lib.ttr_orthogonalize(self.h, ctypes.byref(sx), _SIDE[side], TTR_FP64))
        X._read_ranks()
        return X

    def round(self, X: TT, tol: float, direction: str = "RLR", prec: str = "fp64",
              out: Optional[TT] = None, return_norm: bool = False):
        caps = [X.R[n] * X.I[n] * X.R[n + 1] for n in range(X.N)]
        Y = out if out is not None else TT.empty(X.I, caps, X.cores[0].device)
        nrm = ctypes.c_double()
        sx, sy = X._struct(), Y._struct()
        _check(_lib.ttr_round(self.h, ctypes.byref(sx), float(tol), _DIR[direction], _PREC[prec],
                              ctypes.byref(sy), ctypes.byref(nrm)))
        Y._read_ranks()
        return (Y, nrm.value) if return_norm else Y

    def round_hadamard(self, A: TT, B: TT, tol: float, direction: str = "RLR", prec: str = "fp64",
                       out: Optional[TT] = None, return_norm: bool = False):
        """Rounding of A * B without forming it (ttr_round_hadamard)."""
        R = [A.R[n] * B.R[n] for n in range(A.N + 1)]
        caps = [R[n] * A.I[n] * R[n + 1] for n in range(A.N)]
        Y = out if out is not None else TT.empty(A.I, caps, A.cores[0].device)
        nrm = ctypes.c_double()
        sa, sb, sy = A._struct(), B._struct(), Y._struct()
        _check(_lib.ttr_round_hadamard(self.h, ctypes.byref(sa), ctypes.byref(sb), float(tol), _DIR[direction],
                                       _PREC[prec], ctypes.byref(sy), ctypes.byref(nrm)))
        Y._read_ranks()
        return (Y, nrm.value) if return_norm else Y

    def round_batched(self, Xs: Sequence[TT], tols, prec: str = "fp64", outs: Optional[Sequence[TT]] = None,
                      ranks=None, tune: bool = False):
        """Rounds every X in Xs (same N, RLR) with one replay of a captured
        graph.  Returns (Ys, ranks) where ranks is a device int64 tensor of
        shape (count, N+1); Ys[t].R is filled only by `sync_ranks`."""
        import torch
        count = len(Xs)
        N = Xs[0].N
        if outs is None:
            outs = [TT.empty(X.I, [X.R[n] * X.I[n] * X.R[n + 1] for n in range(N)], X.cores[0].device)
                    for X in Xs]
        if ranks is None:
            ranks = torch.zeros((count, N + 1), dtype=torch.int64, device=Xs[0].cores[0].device)
        if not isinstance(tols, (list, tuple)):
            tols = [float(tols)] * count
        xs = (_TTStruct * count)(*[X._struct() for X in Xs])
        ys = (_TTStruct * count)(*[Y._struct() for Y in outs])
        tl = (ctypes.c_double * count)(*[float(t) for t in tols])
        self._batch_keep = (xs, ys, tl, Xs, outs)  # the arrays must outlive the call
        _check(_lib.ttr_round_batched(self.h, count, xs, tl, _DIR["RLR"], _PREC[prec], ys,
                                      ctypes.c_void_p(ranks.data_ptr()), 1 if tune else 0))
        return outs, ranks

    @staticmethod
    def sync_ranks(Ys: Sequence[TT], ranks):
        """Copies the device ranks of a batched call into the Y objects."""
        r = ranks.cpu().tolist()
        for Y, rr in zip(Ys, r):
            if rr[0] < 0:
                raise TTRError(TTR_ERR_NUMERICAL, "a small factorization of a batch member failed")
            Y.R = [int(x) for x in rr]

    def batch_plan(self) -> dict:
        bp = BatchPlan()
        _check(_lib.ttr_get_batch_plan(self.h, ctypes.byref(bp)))
        return {"count": bp.count, "spw_target": bp.spw_target, "grid_cap": bp.grid_cap,
                "graph_nodes": bp.graph_nodes, "workspace_bytes": bp.workspace_bytes,
                "candidates": [{"spw": bp.cand_spw[i], "grid": bp.cand_grid[i], "ms": bp.cand_ms[i]}
                               for i in range(bp.candidates)]}

    def set_profiling(self, on: bool = True):
        _check(_lib.ttr_set_profiling(self.h, 1 if on else 0))

    def profile(self) -> dict:
        pr = Profile()
        _check(_lib.ttr_get_profile(self.h, ctypes.byref(pr)))
        return {name: {"count": int(pr.count[i]), "ms": pr.ms[i], "bytes": pr.bytes[i], "flops": pr.flops[i]}
                for i, name in enumerate(PROF_CLASSES)}

    def round_stats(self) -> dict:
        st = RoundStats()
        _check(_lib.ttr_get_round_stats(self.h, ctypes.byref(st)))
        nl = min(st.links, TTR_STATS_LINKS)
        sig = [[st.sigma[l * TTR_STATS_SIGMA + j] for j in range(st.nsigma[l])] for l in range(nl)]
        return {"gram_passes": st.gram_passes, "apply_passes": st.apply_passes,
                "small_launches": st.small_launches, "norm": st.norm, "delta": st.delta, "sigmas": sig,
                "tail2": [st.tail2[l] for l in range(nl)], "sweeps": [st.sweeps[l] for l in range(nl)]}
