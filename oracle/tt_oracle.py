"""Plain FP64 CPU oracle for tensor-train (TT) arithmetic.

TEST INFRASTRUCTURE ONLY.  This module is the checker, not the product: only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the HIP library (no
kernels, headers, helpers or constants) and never imports it.

Everything is written from "Parallel Algorithms for Tensor Train Arithmetic"
(Al Daas, Ballard, Benner), in float64, with NumPy/LAPACK routines used only
as single steps (a Householder QR, an SVD, a matrix product).  There is no
blocking, fusion or reordering beyond what the paper states, so that each
function can be checked against the paper by eye.

Representation (paper §2.1, §2.2, §3.1)
---------------------------------------
A TT tensor is a Python list of N numpy arrays; core n has shape
``(R_{n-1}, I_n, R_n)`` with ``R_0 = R_N = 1``.  Slice ``X_n(i)`` is
``core[:, i, :]``.  The paper's memory layout ("natural descending" order,
§3.1) is Fortran order of that shape: entry (a, i, b) sits at offset
``a + R_{n-1} (i + I_n b)``.  With that order both unfoldings of §2.2 are
column-major views of the same buffer:

* horizontal ``H(X_n)`` = ``R_{n-1} x (I_n R_n)`` (mode-1 modal unfolding),
* vertical   ``V(X_n)`` = ``(R_{n-1} I_n) x R_n``.

The helpers ``H``/``V`` below realise exactly those reshapes (order='F').

Readings of points the paper leaves open (repeated where they are used):

* R1  "epsilon-truncated SVD" = smallest rank whose Frobenius tail is <= the
      threshold (the only reading under which Alg. 2's guarantee follows from
      splitting the budget over N-1 links).
* R2  ties (tail == threshold) truncate; the kept rank is at least 1.
* R3  N = 1: rounding returns a copy; tol = 0 keeps every nonzero singular
      value; a zero tensor rounds to a rank-1 zero TT.
* R4  the norm feeding the threshold is the computed ||X_1||_F after the
      orthonormalization sweep.
* R5  Alg. 2 is RLR (right-orthonormalize, truncate left to right); LRL is its
      mirror image.
* R9  sum: X-block first; Hadamard: standard Kronecker index a_x * R^Y + a_y.
* R17 the pivoted Cholesky of the symmetric norm stops at pivots of at most
      d u times the largest diagonal entry (LAPACK's xPSTRF default).
"""

from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np

TT = List[np.ndarray]

__all__ = [
    "H", "V", "from_H", "from_V", "ranks", "dims", "tt_bytes",
    "add", "hadamard", "apply_kron", "dot", "norm_gram", "norm_gram_sym", "pivoted_cholesky", "norm_ortho",
    "orthogonalize", "round_tt", "choose_rank",
    "full", "entry", "tt_svd", "diff_norm", "copy_tt",
]


# ---------------------------------------------------------------------------
# Unfoldings (§2.2) and bookkeeping
# ---------------------------------------------------------------------------

def H(core: np.ndarray) -> np.ndarray:
    """Horizontal unfolding: slices X(i) side by side, R_{n-1} x (I_n R_n) (§2.2)."""
    r0, n, r1 = core.shape
    return core.reshape(r0, n * r1, order="F")


def V(core: np.ndarray) -> np.ndarray:
    """Vertical unfolding: slices X(i) stacked, (R_{n-1} I_n) x R_n (§2.2)."""
    r0, n, r1 = core.shape
    return core.reshape(r0 * n, r1, order="F")


def from_H(mat: np.ndarray, r0: int, n: int, r1: int) -> np.ndarray:
    """Inverse of :func:`H`."""
    return np.asarray(mat).reshape(r0, n, r1, order="F")


def from_V(mat: np.ndarray, r0: int, n: int, r1: int) -> np.ndarray:
    """Inverse of :func:`V`."""
    return np.asarray(mat).reshape(r0, n, r1, order="F")


def ranks(X: TT) -> List[int]:
    """TT ranks (R_0, ..., R_N) with R_0 = R_N = 1 (§2.1)."""
    return [int(X[0].shape[0])] + [int(c.shape[2]) for c in X]


def dims(X: TT) -> List[int]:
    """Mode sizes (I_1, ..., I_N)."""
    return [int(c.shape[1]) for c in X]


def tt_bytes(X: TT) -> int:
    """Bytes of all FP64 cores, sum_n 8 R_{n-1} I_n R_n."""
    return int(sum(8 * c.size for c in X))


def copy_tt(X: TT) -> TT:
    return [np.array(c, dtype=np.float64, order="F", copy=True) for c in X]


def _check(X: TT) -> None:
    if len(X) == 0:
        raise ValueError("a TT tensor needs at least one core")
    if X[0].shape[0] != 1 or X[-1].shape[2] != 1:
        raise ValueError("boundary ranks must be 1 (R_0 = R_N = 1, §2.1)")
    for a, b in zip(X[:-1], X[1:]):
        if a.shape[2] != b.shape[0]:
            raise ValueError("adjacent cores disagree on a rank")


# ---------------------------------------------------------------------------
# Basic operations (§3.2)
# ---------------------------------------------------------------------------

def add(alpha: float, X: TT, beta: float, Y: TT) -> TT:
    """alpha*X + beta*Y in TT form, by the slice-wise formula of §3.2.1.

    First core [alpha X_1, beta Y_1] (the scalars ride on the first cores),
    interior slices blockdiag(X_n(i), Y_n(i)) with the X block first, last core
    [X_N; Y_N].  Ranks add.  With N = 1 the first and last core coincide and
    the single 1 x I x 1 core is alpha X_1 + beta Y_1.
    """
    _check(X)
    _check(Y)
    if dims(X) != dims(Y):
        raise ValueError("mode sizes differ")
    N = len(X)
    if N == 1:
        return [np.asfortranarray(alpha * X[0] + beta * Y[0])]
    Z: TT = []
    for n in range(N):
        x, y = X[n], Y[n]
        rx0, In, rx1 = x.shape
        ry0, _, ry1 = y.shape
        if n == 0:
            z = np.zeros((1, In, rx1 + ry1), order="F")
            z[:, :, :rx1] = alpha * x
            z[:, :, rx1:] = beta * y
        elif n == N - 1:
            z = np.zeros((rx0 + ry0, In, 1), order="F")
            z[:rx0] = x
            z[rx0:] = y
        else:
            z = np.zeros((rx0 + ry0, In, rx1 + ry1), order="F")
            z[:rx0, :, :rx1] = x
            z[rx0:, :, rx1:] = y
        Z.append(z)
    return Z


def hadamard(X: TT, Y: TT) -> TT:
    """Elementwise product in TT form: Z_n(i) = X_n(i) (x) Y_n(i) (§3.2.2).

    The Kronecker product is written out per slice with ``np.kron``; row index
    a_x R^Y + a_y, column index b_x R^Y + b_y.  Ranks multiply.
    """
    _check(X)
    _check(Y)
    if dims(X) != dims(Y):
        raise ValueError("mode sizes differ")
    Z: TT = []
    for x, y in zip(X, Y):
        rx0, In, rx1 = x.shape
        ry0, _, ry1 = y.shape
        z = np.empty((rx0 * ry0, In, rx1 * ry1), order="F")
        for i in range(In):
            z[:, i, :] = np.kron(x[:, i, :], y[:, i, :])
        Z.append(z)
    return Z


def apply_kron(A: Sequence[np.ndarray], X: TT) -> TT:
    """Matrix-vector product with a Kronecker product of matrices (§3.2.5):
    vec(Y) = (A_1 (x) ... (x) A_N) vec(X) in TT form, Y_n = X_n x_2 A_n, i.e.
    Y_n(a, :, b) = A_n X_n(a, :, b) for every a, b; ranks are unchanged.
    A_n is a dense I_n x I_n array."""
    _check(X)
    if len(A) != len(X):
        raise ValueError("one matrix per mode")
    Y: TT = []
    for a_n, x in zip(A, X):
        r0, In, r1 = x.shape
        if a_n.shape != (In, In):
            raise ValueError("A_n must be I_n x I_n")
        y = np.empty((r0, In, r1), order="F")
        for b in range(r1):
            y[:, :, b] = x[:, :, b] @ a_n.T      # rows: (A_n X_n(a, :, b))^T
        Y.append(y)
    return Y


def dot(X: TT, Y: TT) -> float:
    """Inner product <X, Y> by the recursion of eq. (4) (§3.2.3).

    W_0 = 1 and W_n = sum_i Y_n(i)^T W_{n-1} X_n(i), an R^Y_n x R^X_n matrix;
    the result is the final 1 x 1 W_N.  Each slice term is one pair of matrix
    products, summed over i in order.
    """
    _check(X)
    _check(Y)
    if dims(X) != dims(Y):
        raise ValueError("mode sizes differ")
    W = np.ones((1, 1))
    for x, y in zip(X, Y):
        Wn = np.zeros((y.shape[2], x.shape[2]))
        for i in range(x.shape[1]):
            Wn += y[:, i, :].T @ W @ x[:, i, :]
        W = Wn
    return float(W[0, 0])


def norm_gram(X: TT) -> float:
    """||X|| = sqrt(<X, X>) (first approach of §3.2.4).

    Suffers cancellation for small norms of difference tensors; a tiny negative
    rounding residue is clamped to zero.
    """
    v = dot(X, X)
    return math.sqrt(max(v, 0.0))


def pivoted_cholesky(W: np.ndarray, rel_tol: float | None = None):
    """Pivoted Cholesky of a symmetric positive semi-definite W (§3.2.4 names it
    as the triangular factorization of the inner-product matrices).

    Diagonal pivoting: step j moves the largest remaining diagonal entry of the
    Schur complement to position j (first one among ties), takes its square
    root as L(j, j), scales the column below it and subtracts the rank-one
    update.  It stops when that entry is at most ``rel_tol`` times the largest
    diagonal entry of W (LAPACK's xPSTRF default ``d * u`` when None; reading
    R17), or is not positive.  Returns ``(perm, L)`` with L (d x k) lower
    trapezoidal and ``W[perm][:, perm] ~= L L^T``, i.e. W = P L L^T P^T with
    P[perm[j], j] = 1.
    """
    W = np.array(W, dtype=np.float64)
    d = W.shape[0]
    if rel_tol is None:
        rel_tol = d * (np.finfo(np.float64).eps / 2)
    A = W.copy()
    perm = list(range(d))
    dmax0 = max(np.max(np.diag(A)), 0.0) if d else 0.0
    k = d
    for j in range(d):
        p = j + int(np.argmax(np.diag(A)[j:]))
        if not (A[p, p] > rel_tol * dmax0):
            k = j
            break
        if p != j:
            A[[j, p], :] = A[[p, j], :]
            A[:, [j, p]] = A[:, [p, j]]
            perm[j], perm[p] = perm[p], perm[j]
        A[j, j] = math.sqrt(A[j, j])
        A[j + 1:, j] /= A[j, j]
        A[j + 1:, j + 1:] -= np.outer(A[j + 1:, j], A[j + 1:, j])
    L = np.tril(A[:, :k])
    return np.array(perm, dtype=np.int64), L


def norm_gram_sym(X: TT) -> float:
    """||X|| = sqrt(W_N) by the symmetric form of the inner-product recursion
    (first approach of §3.2.4 with its structure exploited).

    W_1 = V(X_1)^T V(X_1).  For n >= 2, W_{n-1} = P L L^T P^T (pivoted
    Cholesky), H(Z_n) = L^T (P^T H(X_n)) and W_n = V(Z_n)^T V(Z_n), which
    equals sum_i X_n(i)^T W_{n-1} X_n(i).  Like ``norm_gram`` it cancels for
    small norms of difference tensors; a negative residue is clamped to zero.
    """
    _check(X)
    W = V(X[0]).T @ V(X[0])
    for n in range(1, len(X)):
        r0, In, r1 = X[n].shape
        perm, L = pivoted_cholesky(W)
        k = L.shape[1]
        Hz = L.T @ H(X[n])[perm, :]          # P^T H(X_n) selects rows perm[0], perm[1], ...
        Z = from_H(Hz, k, In, r1)
        W = V(Z).T @ V(Z)
    return math.sqrt(max(float(W[0, 0]), 0.0))


# ---------------------------------------------------------------------------
# Orthonormalization (§2.3, Alg. 1) and the orthonormal-norm (§2.3, §3.2.4)
# ---------------------------------------------------------------------------

def _right_orth(X: TT) -> TT:
    """Alg. 1: for n = N..2, QR of H(X_n)^T; H(X_n) <- Q^T; V(X_{n-1}) <- V(X_{n-1}) R^T.

    The QR is LAPACK's Householder QR (``numpy.linalg.qr``, reduced), so an
    unfolding with fewer rows than columns yields a thin factor and the rank
    becomes I_n R_n (a shape the configurations never reach).
    """
    Y = copy_tt(X)
    for n in range(len(Y) - 1, 0, -1):
        r0, In, r1 = Y[n].shape
        Q, R = np.linalg.qr(H(Y[n]).T, mode="reduced")
        k = Q.shape[1]
        Y[n] = np.asfortranarray(from_H(Q.T, k, In, r1))
        p0, Ip, _ = Y[n - 1].shape
        Y[n - 1] = np.asfortranarray(from_V(V(Y[n - 1]) @ R.T, p0, Ip, k))
    return Y


def _left_orth(X: TT) -> TT:
    """Mirror of Alg. 1: for n = 1..N-1, QR of V(X_n); V(X_n) <- Q; H(X_{n+1}) <- R H(X_{n+1})."""
    Y = copy_tt(X)
    for n in range(len(Y) - 1):
        r0, In, r1 = Y[n].shape
        Q, R = np.linalg.qr(V(Y[n]), mode="reduced")
        k = Q.shape[1]
        Y[n] = np.asfortranarray(from_V(Q, r0, In, k))
        _, In1, q1 = Y[n + 1].shape
        Y[n + 1] = np.asfortranarray(from_H(R @ H(Y[n + 1]), k, In1, q1))
    return Y


def orthogonalize(X: TT, side: str = "right") -> TT:
    """Right-orthonormal (H(X_n) row-orthonormal for n >= 2) or left-orthonormal
    (V(X_n) column-orthonormal for n <= N-1) equivalent of X (§2.3)."""
    _check(X)
    if side == "right":
        return _right_orth(X)
    if side == "left":
        return _left_orth(X)
    raise ValueError("side must be 'right' or 'left'")


def norm_ortho(X: TT) -> float:
    """||X|| = ||X_1||_F after right-orthonormalization (end of §2.3; second
    approach of §3.2.4, accurate for small norms).

    Alg. 1's sweep, keeping only what reaches the first core: for n = N..2 the
    triangular factor R of H(X_n)^T = QR and V(X_{n-1}) <- V(X_{n-1}) R^T.  The
    orthonormal cores Q^T do not enter ||X_1||_F, so they are not formed (the
    R of LAPACK's Householder QR is the same with or without Q)."""
    _check(X)
    Y = copy_tt(X)
    for n in range(len(Y) - 1, 0, -1):
        R = np.linalg.qr(H(Y[n]).T, mode="r")
        k = R.shape[0]
        p0, Ip, _ = Y[n - 1].shape
        Y[n - 1] = np.asfortranarray(from_V(V(Y[n - 1]) @ R.T, p0, Ip, k))
        Y[n] = None
    return float(np.linalg.norm(Y[0]))


# ---------------------------------------------------------------------------
# Rounding (§2.4, Alg. 2)
# ---------------------------------------------------------------------------

def choose_rank(s: np.ndarray, delta: float) -> int:
    """Truncation rank for singular values ``s`` (descending) and threshold delta.

    Reading R1/R2: the smallest L >= 1 whose Frobenius tail
    sqrt(sum_{j > L} s_j^2) is <= delta.  Tails are summed from the smallest
    value upwards.
    """
    s = np.asarray(s, dtype=np.float64)
    m = s.size
    if m == 0:
        return 1
    tail_sq = np.zeros(m + 1)
    tail_sq[:m] = np.cumsum((s * s)[::-1])[::-1]     # tail_sq[L] = sum_{j >= L} s_j^2 (0-based)
    for L in range(1, m + 1):
        if math.sqrt(tail_sq[L]) <= delta:
            return L
    return m


def round_tt(X: TT, tol: float, direction: str = "RLR", return_info: bool = False):
    """TT rounding, Alg. 2 (§2.4), with Alg. 1 as its first sweep.

    RLR (the paper's listing): right-orthonormalize; ||X|| = ||X_1||_F; threshold
    delta = tol ||X|| / sqrt(N-1); for n = 1..N-1 take the truncated SVD
    V(X_n) ~ U S V^T, set V(X_n) <- U and H(X_{n+1}) <- S V^T H(X_{n+1}).
    LRL is the mirror image: left-orthonormalize, ||X|| = ||X_N||_F, then for
    n = N..2 truncate the SVD of H(X_n)^T and pass V S into core n-1.

    Guarantees ||X - round(X)|| <= tol ||X|| (Alg. 2).  N = 1 returns a copy
    (reading R3).  ``return_info`` adds the norm, threshold and the full list
    of singular values met at every link (gauge-invariant, App. A).
    """
    _check(X)
    if tol < 0 or not np.isfinite(tol):
        raise ValueError("tol must be finite and >= 0")
    N = len(X)
    if N == 1:
        Y = copy_tt(X)
        info = {"norm": float(np.linalg.norm(Y[0])), "delta": 0.0, "sigmas": []}
        return (Y, info) if return_info else Y
    sigmas = []
    if direction == "RLR":
        Y = _right_orth(X)
        nrm = float(np.linalg.norm(Y[0]))
        delta = tol * nrm / math.sqrt(N - 1)
        for n in range(N - 1):
            r0, In, r1 = Y[n].shape
            U, s, Vt = np.linalg.svd(V(Y[n]), full_matrices=False)
            L = choose_rank(s, delta)
            sigmas.append(s.copy())
            Y[n] = np.asfortranarray(from_V(U[:, :L], r0, In, L))
            _, In1, q1 = Y[n + 1].shape
            SVt = s[:L, None] * Vt[:L, :]
            Y[n + 1] = np.asfortranarray(from_H(SVt @ H(Y[n + 1]), L, In1, q1))
    elif direction == "LRL":
        Y = _left_orth(X)
        nrm = float(np.linalg.norm(Y[N - 1]))
        delta = tol * nrm / math.sqrt(N - 1)
        for n in range(N - 1, 0, -1):
            r0, In, r1 = Y[n].shape
            U, s, Vt = np.linalg.svd(H(Y[n]).T, full_matrices=False)
            L = choose_rank(s, delta)
            sigmas.append(s.copy())
            Y[n] = np.asfortranarray(from_H(U[:, :L].T, L, In, r1))
            p0, Ip, _ = Y[n - 1].shape
            VS = Vt[:L, :].T * s[None, :L]
            Y[n - 1] = np.asfortranarray(from_V(V(Y[n - 1]) @ VS, p0, Ip, L))
        sigmas.reverse()
    else:
        raise ValueError("direction must be 'RLR' or 'LRL'")
    if return_info:
        return Y, {"norm": nrm, "delta": delta, "sigmas": sigmas}
    return Y


def diff_norm(A: TT, B: TT) -> float:
    """||A - B|| through the orthonormal-norm of the TT difference (§2.3):
    cancellation-free, unlike sqrt(||A||^2 - 2<A,B> + ||B||^2)."""
    return norm_ortho(add(1.0, A, -1.0, B))


# ---------------------------------------------------------------------------
# Brute force on small tensors (checks only)
# ---------------------------------------------------------------------------

def full(X: TT) -> np.ndarray:
    """Dense tensor X(i_1, ..., i_N) = X_1(i_1) ... X_N(i_N) (§2.1), as an
    I_1 x ... x I_N numpy array (index order = mode order)."""
    _check(X)
    T = X[0][0]                                   # I_1 x R_1
    for core in X[1:]:
        T = np.tensordot(T, core, axes=([T.ndim - 1], [0]))
    return T[..., 0]


def entry(X: TT, idx: Sequence[int]) -> float:
    """One entry: the chain product of the slices selected by ``idx`` (§2.1)."""
    v = np.ones((1, 1))
    for core, i in zip(X, idx):
        v = v @ core[:, int(i), :]
    return float(v[0, 0])


def tt_svd(T: np.ndarray, delta: float, return_sigmas: bool = False):
    """TT-SVD of a dense tensor, left to right, every link truncated with the
    same absolute Frobenius-tail threshold ``delta`` as :func:`choose_rank`.

    This is the textbook sequential SVD of successive unfoldings of the
    remainder (row index (r_{n-1}, i_n), columns the remaining modes); it
    touches no TT rounding code and serves as the brute-force reference.
    """
    shape = T.shape
    N = len(shape)
    cores: TT = []
    sig = []
    r = 1
    C = np.asarray(T, dtype=np.float64).reshape(1, -1)
    for n in range(N - 1):
        C = C.reshape(r * shape[n], -1)
        U, s, Vt = np.linalg.svd(C, full_matrices=False)
        L = choose_rank(s, delta)
        sig.append(s.copy())
        # row index of C is r_prev * I_n + i_n (C order) -> core(a, i, b) = U[a*I_n + i, b]
        cores.append(np.asfortranarray(U[:, :L].reshape(r, shape[n], L)))
        C = s[:L, None] * Vt[:L, :]
        r = L
    cores.append(np.asfortranarray(C.reshape(r, shape[N - 1], 1)))
    return (cores, sig) if return_sigmas else cores
