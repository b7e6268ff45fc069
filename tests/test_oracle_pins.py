"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these retypes an oracle formula: every check compares against a
dense brute-force tensor, a closed form, an invariant, a textbook routine on
the full matrix (TT-SVD, Eckart-Young), or the paper's own guarantee.
"""

import math

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def rand_tt(rng, I, r, scale=1.0):
    R = [1] + list(r) + [1]
    return [np.asfortranarray(scale * rng.standard_normal((R[n], I[n], R[n + 1]))) for n in range(len(I))]


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


SHAPES = [
    ([5, 4, 6], [3, 2]),
    ([3, 7, 2, 4], [2, 5, 3]),
    ([6], []),
    ([4, 1, 5], [2, 2]),          # I_n = 1 mode
    ([2, 3, 2, 2, 3], [2, 4, 3, 2]),
]


# ---------------------------------------------------------------- P4: brute force
@pytest.mark.parametrize("I,r", SHAPES)
def test_add_matches_full(I, r):
    rng = np.random.default_rng(1)
    X, Y = rand_tt(rng, I, r), rand_tt(rng, I, r[::-1] if len(r) else r)
    if len(r):
        Y = rand_tt(rng, I, [x + 1 for x in r])
    Z = O.add(1.5, X, -0.25, Y)
    assert rel(O.full(Z), 1.5 * O.full(X) - 0.25 * O.full(Y)) < 1e-13
    R = O.ranks(Z)
    assert R[1:-1] == [a + b for a, b in zip(O.ranks(X)[1:-1], O.ranks(Y)[1:-1])]


@pytest.mark.parametrize("I,r", SHAPES)
def test_hadamard_matches_full(I, r):
    rng = np.random.default_rng(2)
    X = rand_tt(rng, I, r)
    Y = rand_tt(rng, I, [x + 1 for x in r])
    Z = O.hadamard(X, Y)
    assert rel(O.full(Z), O.full(X) * O.full(Y)) < 1e-13
    assert O.ranks(Z)[1:-1] == [a * b for a, b in zip(O.ranks(X)[1:-1], O.ranks(Y)[1:-1])]


def test_hadamard_kronecker_index_convention():
    # Standard Kronecker product of the two slices (§3.2.2): block (a_x, b_x) of
    # Z(i) is X(i)[a_x, b_x] * Y(i).  Checked on a 2x2 (x) 2x2 slice by hand.
    X = [np.array([[[1.0, 2.0]]]).reshape(1, 1, 2, order="F"), np.array([[[3.0]], [[5.0]]]).reshape(2, 1, 1, order="F")]
    Y = [np.array([[[7.0, 11.0]]]).reshape(1, 1, 2, order="F"), np.array([[[13.0]], [[17.0]]]).reshape(2, 1, 1, order="F")]
    Z = O.hadamard(X, Y)
    assert Z[0][0, 0, :].tolist() == [7.0, 11.0, 14.0, 22.0]
    assert Z[1][:, 0, 0].tolist() == [39.0, 51.0, 65.0, 85.0]


@pytest.mark.parametrize("I,r", SHAPES)
def test_dot_and_norms_match_full(I, r):
    rng = np.random.default_rng(3)
    X = rand_tt(rng, I, r)
    Y = rand_tt(rng, I, [x + 2 for x in r])
    fx, fy = O.full(X), O.full(Y)
    assert abs(O.dot(X, Y) - np.sum(fx * fy)) <= 1e-12 * np.linalg.norm(fx) * np.linalg.norm(fy)
    n = np.linalg.norm(fx)
    assert abs(O.norm_gram(X) - n) <= 1e-12 * n
    assert abs(O.norm_gram_sym(X) - n) <= 1e-12 * n
    assert abs(O.norm_ortho(X) - n) <= 1e-13 * n
    # the norm sweep keeps only the triangular factors of Alg. 1: the same
    # value as ||X_1||_F of the explicitly orthonormalized train
    assert O.norm_ortho(X) == float(np.linalg.norm(O.orthogonalize(X, "right")[0]))


# ---------------------------------------------------------------- symmetric inner-product norm
@pytest.mark.parametrize("d,r", [(1, 1), (6, 6), (9, 4), (20, 20), (24, 7), (5, 0)])
def test_pivoted_cholesky_factors(d, r):
    rng = np.random.default_rng(40 + d + r)
    B = rng.standard_normal((d, r)) * np.logspace(0, -3, r) if r else np.zeros((d, 0))
    W = B @ B.T
    perm, L = O.pivoted_cholesky(W)
    k = L.shape[1]
    assert sorted(perm.tolist()) == list(range(d))
    assert k == r                                    # numerical rank of a rank-r PSD matrix
    assert np.array_equal(L, np.tril(L))
    dg = np.diag(L[:k, :k])
    assert np.all(dg > 0) and np.all(np.diff(dg) <= 1e-12 * max(dg[0] if k else 1.0, 1e-300))
    Wp = W[perm][:, perm]
    assert np.linalg.norm(Wp - L @ L.T) <= 1e-13 * max(np.linalg.norm(W), 1e-300)
    if 0 < r == d:
        # with the pivot order fixed, the Cholesky factor is unique: LAPACK's
        assert np.allclose(L, np.linalg.cholesky(Wp), rtol=0, atol=1e-12 * np.sqrt(np.max(np.diag(W))))


def test_norm_sym_rank_deficient_and_degenerate():
    rng = np.random.default_rng(44)
    Y = rand_tt(rng, [5, 6, 4, 7], [3, 4, 2])
    n = np.linalg.norm(O.full(Y))
    X = O.add(1.0, Y, 1.0, Y)                        # every W_n has rank R_n / 2
    assert abs(O.norm_gram_sym(X) - 2 * n) <= 1e-12 * n
    D = O.add(1.0, Y, -1.0, Y)                       # zero tensor in rank-8 form: cancellation level
    assert O.norm_gram_sym(D) <= 1e-6 * n
    Z = [np.zeros_like(c) for c in Y]                # zero cores: W_n = 0, empty factors
    assert O.norm_gram_sym(Z) == 0.0
    one = rand_tt(rng, [7], [])                      # N = 1
    assert abs(O.norm_gram_sym(one) - np.linalg.norm(one[0])) <= 1e-14 * np.linalg.norm(one[0])


def test_norm_sym_planted_mistakes_fail():
    rng = np.random.default_rng(45)
    X = rand_tt(rng, [4, 5, 3, 6], [3, 4, 2])
    n = np.linalg.norm(O.full(X))

    def variant(slip):
        W = O.V(X[0]).T @ O.V(X[0])
        for m in range(1, len(X)):
            r0, In, r1 = X[m].shape
            perm, L = O.pivoted_cholesky(W)
            Hx = O.H(X[m]) if slip == "no_perm" else O.H(X[m])[perm, :]
            F = L if slip == "L_not_LT" else L.T
            Z = O.from_H(F @ Hx, L.shape[1], In, r1)
            W = O.V(Z).T @ O.V(Z)
        return math.sqrt(max(W[0, 0], 0.0))

    assert abs(variant(None) - n) <= 1e-12 * n
    assert abs(variant("no_perm") - n) > 1e-6 * n
    assert abs(variant("L_not_LT") - n) > 1e-6 * n


def test_rank_one_closed_forms():
    # rank-1 TT u1 o u2 o u3: ||X|| = prod ||u_n||, <X, Y> = prod <u_n, v_n>
    rng = np.random.default_rng(4)
    us = [rng.standard_normal(m) for m in (5, 7, 3)]
    vs = [rng.standard_normal(m) for m in (5, 7, 3)]
    X = [u.reshape(1, -1, 1, order="F").copy(order="F") for u in us]
    Y = [v.reshape(1, -1, 1, order="F").copy(order="F") for v in vs]
    assert math.isclose(O.norm_ortho(X), np.prod([np.linalg.norm(u) for u in us]), rel_tol=1e-14)
    assert math.isclose(O.dot(X, Y), np.prod([u @ v for u, v in zip(us, vs)]), rel_tol=1e-13)


# ---------------------------------------------------------------- orthonormalization (§2.3)
@pytest.mark.parametrize("side", ["right", "left"])
@pytest.mark.parametrize("I,r", SHAPES)
def test_orthogonalize_invariants(side, I, r):
    rng = np.random.default_rng(5)
    X = rand_tt(rng, I, r, scale=3.0)
    Y = O.orthogonalize(X, side)
    assert rel(O.full(Y), O.full(X)) < 1e-13
    N = len(Y)
    if side == "right":
        for n in range(1, N):
            Hn = O.H(Y[n])
            assert np.linalg.norm(Hn @ Hn.T - np.eye(Hn.shape[0])) < 1e-13 * Hn.shape[0]
        assert math.isclose(np.linalg.norm(Y[0]), np.linalg.norm(O.full(X)), rel_tol=1e-13)
    else:
        for n in range(N - 1):
            Vn = O.V(Y[n])
            assert np.linalg.norm(Vn.T @ Vn - np.eye(Vn.shape[1])) < 1e-13 * Vn.shape[1]
        assert math.isclose(np.linalg.norm(Y[-1]), np.linalg.norm(O.full(X)), rel_tol=1e-13)


def test_thin_qr_rank_drop():
    # R_{n-1} > I_n R_n: the QR of H(X_n)^T is thin and the rank becomes I_n R_n
    rng = np.random.default_rng(6)
    X = rand_tt(rng, [6, 2], [5])
    Y = O.orthogonalize(X, "right")
    assert O.ranks(Y) == [1, 2, 1]
    assert rel(O.full(Y), O.full(X)) < 1e-13


# ---------------------------------------------------------------- P1: Y + Y rounds to 2Y
@pytest.mark.parametrize("direction", ["RLR", "LRL"])
def test_round_y_plus_y_is_2y_yy_small(direction):
    d = synth.yy_small()
    Y = d["Y"]
    X = O.add(1.0, Y, 1.0, Y)
    assert O.ranks(X) == [1, 10, 10, 10, 1]
    Xt = O.round_tt(X, d["tol"], direction)
    assert O.ranks(Xt) == [1, 5, 5, 5, 1]
    twoY = O.add(2.0, Y, 0.0, Y)
    assert O.diff_norm(Xt, twoY) <= 1e-12 * 2 * O.norm_ortho(Y)


# ---------------------------------------------------------------- P2: equivalence with TT-SVD of the full tensor
def _graded_tt(rng, I, r_big, r_small, eps_small):
    Y = rand_tt(rng, I, r_big)
    Z = rand_tt(rng, I, r_small)
    Z[0] = Z[0] * eps_small
    return O.add(1.0, Y, 1.0, Z)


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
@pytest.mark.parametrize("tol", [1e-1, 1e-3, 1e-6])
def test_round_equals_tt_svd(direction, tol):
    rng = np.random.default_rng(7)
    I = [4, 5, 3, 6]
    X = _graded_tt(rng, I, [2, 3, 2], [2, 2, 2], 1e-3)
    T = O.full(X)
    N = len(I)
    delta = tol * np.linalg.norm(T) / math.sqrt(N - 1)
    if direction == "RLR":
        ref, ref_sig = O.tt_svd(T, delta, return_sigmas=True)
        Tref = O.full(ref)
    else:
        Trev = np.transpose(T, axes=list(range(N))[::-1])
        ref, ref_sig = O.tt_svd(Trev, delta, return_sigmas=True)
        Tref = np.transpose(O.full(ref), axes=list(range(N))[::-1])
        ref_sig = ref_sig[::-1]
    Xt, info = O.round_tt(X, tol, direction, return_info=True)
    # ranks agree link by link (LRL ranks read right to left are TT-SVD ranks of the reversed tensor)
    got = O.ranks(Xt)
    want = O.ranks(ref) if direction == "RLR" else O.ranks(ref)[::-1]
    assert got == want
    assert rel(O.full(Xt), Tref) < 1e-12
    # gauge-invariant singular values agree (nonzero part)
    for s_tt, s_ref in zip(info["sigmas"], ref_sig):
        k = min(len(s_tt), len(s_ref))
        big = s_ref[:k] > 1e-10 * s_ref[0]
        assert np.allclose(s_tt[:k][big], s_ref[:k][big], rtol=1e-10, atol=0)


# ---------------------------------------------------------------- P3: N = 2 is the truncated matrix SVD
@pytest.mark.parametrize("tol", [0.3, 1e-2, 1e-8])
def test_round_n2_is_eckart_young(tol):
    rng = np.random.default_rng(8)
    F1 = rng.standard_normal((30, 6)) @ np.diag(10.0 ** -np.arange(6))
    F2 = rng.standard_normal((6, 25))
    A = F1 @ F2
    X = [np.asfortranarray(F1.reshape(1, 30, 6)), np.asfortranarray(F2.reshape(6, 25, 1))]
    assert rel(O.full(X), A) < 1e-14
    U, s, Vt = np.linalg.svd(A, full_matrices=False)      # Eckart-Young on the full matrix
    delta = tol * np.linalg.norm(A)
    L = O.choose_rank(s, delta)
    ref = (U[:, :L] * s[:L]) @ Vt[:L]
    Xt = O.round_tt(X, tol, "RLR")
    assert O.ranks(Xt)[1] == L
    assert np.linalg.norm(O.full(Xt) - ref) <= 1e-12 * np.linalg.norm(A)
    assert np.linalg.norm(A - ref) <= tol * np.linalg.norm(A) + 1e-15


# ---------------------------------------------------------------- P5, P6: orthonormal output and the error bound
@pytest.mark.parametrize("direction", ["RLR", "LRL"])
@pytest.mark.parametrize("tol", [0.5, 1e-2, 1e-5])
def test_round_output_orthonormal_and_bound(direction, tol):
    rng = np.random.default_rng(9)
    I = [3, 4, 5, 4, 3]
    X = _graded_tt(rng, I, [3, 4, 4, 3], [2, 3, 3, 2], 1e-2)
    Xt, info = O.round_tt(X, tol, direction, return_info=True)
    N = len(I)
    if direction == "RLR":
        for n in range(N - 1):
            Vn = O.V(Xt[n])
            assert np.linalg.norm(Vn.T @ Vn - np.eye(Vn.shape[1])) < 1e-13 * Vn.shape[1]
        assert math.isclose(np.linalg.norm(Xt[-1]), np.linalg.norm(O.full(Xt)), rel_tol=1e-12)
    else:
        for n in range(1, N):
            Hn = O.H(Xt[n])
            assert np.linalg.norm(Hn @ Hn.T - np.eye(Hn.shape[0])) < 1e-13 * Hn.shape[0]
        assert math.isclose(np.linalg.norm(Xt[0]), np.linalg.norm(O.full(Xt)), rel_tol=1e-12)
    T = O.full(X)
    err = np.linalg.norm(O.full(Xt) - T)
    assert err <= tol * np.linalg.norm(T) * (1 + 1e-12)
    for s in info["sigmas"]:
        L = O.choose_rank(s, info["delta"])
        assert math.sqrt(np.sum(s[L:] ** 2)) <= info["delta"]


# ---------------------------------------------------------------- P7: gauge invariance
def test_round_gauge_invariance():
    rng = np.random.default_rng(10)
    I = [4, 3, 5, 4]
    X = _graded_tt(rng, I, [3, 3, 3], [2, 2, 2], 1e-3)
    Xg = O.copy_tt(X)
    for n in range(len(I) - 1):
        r = Xg[n].shape[2]
        M = np.eye(r) + 0.3 * rng.standard_normal((r, r))
        Mi = np.linalg.inv(M)
        p0, In, _ = Xg[n].shape
        Xg[n] = np.asfortranarray(O.from_V(O.V(Xg[n]) @ M, p0, In, r))
        _, In1, q1 = Xg[n + 1].shape
        Xg[n + 1] = np.asfortranarray(O.from_H(Mi @ O.H(Xg[n + 1]), r, In1, q1))
    assert rel(O.full(Xg), O.full(X)) < 1e-12
    for tol in (1e-2, 1e-4):
        a, b = O.round_tt(X, tol), O.round_tt(Xg, tol)
        assert O.ranks(a) == O.ranks(b)
        assert rel(O.full(a), O.full(b)) < 1e-11


# ---------------------------------------------------------------- P8: identities
def test_identities():
    rng = np.random.default_rng(11)
    I = [4, 5, 3]
    X, Y = rand_tt(rng, I, [2, 3]), rand_tt(rng, I, [3, 2])
    one = [np.ones((1, m, 1), order="F") for m in I]
    YY = O.add(1.0, Y, 1.0, Y)
    assert math.isclose(O.norm_ortho(YY), 2 * O.norm_ortho(Y), rel_tol=1e-13)
    assert math.isclose(O.dot(X, Y), O.dot(Y, X), rel_tol=1e-13)
    assert rel(O.full(O.hadamard(X, one)), O.full(X)) < 1e-15
    assert math.isclose(O.dot(X, Y), O.dot(O.hadamard(X, Y), one), rel_tol=1e-12)
    assert math.isclose(O.norm_ortho(X) ** 2, O.dot(X, X), rel_tol=1e-12)


# ---------------------------------------------------------------- P9: idempotence and edge cases
def test_round_idempotent():
    rng = np.random.default_rng(12)
    X = _graded_tt(rng, [4, 4, 4, 4], [3, 3, 3], [2, 2, 2], 1e-3)
    a = O.round_tt(X, 1e-2)
    b = O.round_tt(a, 0.0)
    assert O.ranks(a) == O.ranks(b)
    assert rel(O.full(a), O.full(b)) < 1e-13


def test_round_edge_cases():
    rng = np.random.default_rng(13)
    # N = 1: copy
    X1 = rand_tt(rng, [7], [])
    assert np.array_equal(O.round_tt(X1, 0.5)[0], X1[0])
    # tol = 0 keeps the formal ranks of a generic TT
    X = rand_tt(rng, [5, 6, 5], [4, 4])
    assert O.ranks(O.round_tt(X, 0.0)) == O.ranks(X)
    # zero tensor -> rank-1 zero TT
    Z = [np.zeros_like(c) for c in X]
    Zt = O.round_tt(Z, 1e-3)
    assert O.ranks(Zt) == [1, 1, 1, 1]
    assert np.linalg.norm(O.full(Zt)) == 0.0
    # huge tolerance -> rank 1
    assert O.ranks(O.round_tt(X, 10.0)) == [1, 1, 1, 1]


def test_choose_rank_frobenius_tail():
    s = np.array([4.0, 3.0, 2.0, 1.0])
    # tails after L=1,2,3,4: sqrt(14), sqrt(5), 1, 0
    assert O.choose_rank(s, 1.0) == 3          # tie truncates (reading R2)
    assert O.choose_rank(s, 0.999) == 4
    assert O.choose_rank(s, math.sqrt(5)) == 2
    assert O.choose_rank(s, 100.0) == 1        # at least rank 1
    assert O.choose_rank(np.zeros(3), 0.0) == 1


def test_entry_matches_full():
    rng = np.random.default_rng(14)
    X = rand_tt(rng, [3, 4, 5], [2, 3])
    T = O.full(X)
    for idx in [(0, 0, 0), (2, 3, 4), (1, 2, 0)]:
        assert math.isclose(O.entry(X, idx), T[idx], rel_tol=1e-13, abs_tol=1e-15)


# ---------------------------------------------------------------- planted mistakes are caught
def test_planted_mistakes_fail_pins(monkeypatch):
    """Each plausible slip in the rounding code trips at least one pin above."""
    rng = np.random.default_rng(15)
    I = [4, 5, 3, 6]
    X = _graded_tt(rng, I, [2, 3, 2], [2, 2, 2], 1e-3)
    T = O.full(X)

    def fails(fn):
        try:
            Xt = fn(X, 1e-3)
        except Exception:
            return True
        delta = 1e-3 * np.linalg.norm(T) / math.sqrt(3)
        ref = O.tt_svd(T, delta)
        return O.ranks(Xt) != O.ranks(ref) or rel(O.full(Xt), O.full(ref)) > 1e-12

    good = lambda X, tol: O.round_tt(X, tol)
    assert not fails(good)

    # (a) singular values dropped when passing S V^T to the next core
    def no_sigma(X, tol):
        Y = O._right_orth(X)
        nrm = np.linalg.norm(Y[0]); delta = tol * nrm / math.sqrt(len(Y) - 1)
        for n in range(len(Y) - 1):
            r0, In, r1 = Y[n].shape
            U, s, Vt = np.linalg.svd(O.V(Y[n]), full_matrices=False)
            L = O.choose_rank(s, delta)
            Y[n] = O.from_V(U[:, :L], r0, In, L)
            _, In1, q1 = Y[n + 1].shape
            Y[n + 1] = O.from_H(Vt[:L] @ O.H(Y[n + 1]), L, In1, q1)
        return Y
    assert fails(no_sigma)

    # (b) R instead of R^T passed into the neighbour during orthonormalization
    def bad_orth(X):
        Y = O.copy_tt(X)
        for n in range(len(Y) - 1, 0, -1):
            r0, In, r1 = Y[n].shape
            Q, R = np.linalg.qr(O.H(Y[n]).T, mode="reduced")
            Y[n] = O.from_H(Q.T, Q.shape[1], In, r1)
            p0, Ip, _ = Y[n - 1].shape
            Y[n - 1] = O.from_V(O.V(Y[n - 1]) @ R, p0, Ip, Q.shape[1])
        return Y
    monkeypatch.setattr(O.tt_oracle, "_right_orth", bad_orth)
    assert fails(lambda X, tol: O.tt_oracle.round_tt(X, tol))
    monkeypatch.undo()

    # (c) threshold without the 1/sqrt(N-1) split
    def no_split(X, tol):
        return O.round_tt(X, tol * math.sqrt(len(X) - 1))
    assert fails(no_split)


# ---------------------------------------------------------------- Kronecker operator (§3.2.5)
def _kron_vec_full(A, X):
    """(A_1 (x) ... (x) A_N) applied to the full tensor, by brute force: the
    Kronecker product acts on vec(X) with the first index slowest, which is
    numpy's C order of full(X) (index order = mode order)."""
    T = O.full(X)
    K = A[0]
    for a in A[1:]:
        K = np.kron(K, a)
    return (K @ T.reshape(-1)).reshape(T.shape)


@pytest.mark.parametrize("I,r", SHAPES)
def test_apply_kron_matches_kronecker_product(I, r):
    rng = np.random.default_rng(31)
    X = rand_tt(rng, I, r)
    A = [rng.standard_normal((n, n)) for n in I]
    Y = O.apply_kron(A, X)
    assert O.ranks(Y) == O.ranks(X)
    ref = _kron_vec_full(A, X)
    assert rel(O.full(Y), ref) <= 1e-13


def test_apply_kron_identities():
    rng = np.random.default_rng(32)
    I = [5, 6, 4]
    X = rand_tt(rng, I, [3, 2])
    # identity operator; a scaled identity on one mode scales the tensor
    Y = O.apply_kron([np.eye(n) for n in I], X)
    assert all(np.array_equal(y, x) for y, x in zip(Y, X))
    A = [np.eye(n) for n in I]
    A[1] = 3.0 * np.eye(I[1])
    assert rel(O.full(O.apply_kron(A, X)), 3.0 * O.full(X)) <= 1e-15
    # (A (x) B)(C (x) D) = AC (x) BD: two applications equal one with the products
    A1 = [rng.standard_normal((n, n)) for n in I]
    A2 = [rng.standard_normal((n, n)) for n in I]
    two = O.apply_kron(A2, O.apply_kron(A1, X))
    one = O.apply_kron([b @ a for a, b in zip(A1, A2)], X)
    assert rel(O.full(two), O.full(one)) <= 1e-13
    # a transposed operator (the planted slip X_n A_n instead of A_n X_n) fails
    At = [a.T for a in A1]
    assert rel(O.full(O.apply_kron(At, X)), _kron_vec_full(A1, X)) > 1e-3
