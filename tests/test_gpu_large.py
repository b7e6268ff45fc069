"""GPU parity at ranks above 64 (the unfolding-based path, up to 256) against
the FP64 oracle: rounding of the Hadamard-then-round workload at reduced mode
sizes (A, B rank 16 with slice weights 2^-b, X = A * B of rank 256) in both
sweep orders and both precisions, sums of ranks 65..100, the rank-deficient
Y + Y; inner product, norms and orthonormalization at ranks up to 256.
"""
import numpy as np
import pytest

import oracle as O
import synth
from test_gpu_round import check_round, rand_tt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h(ttr):
    hd = ttr.Handle(0)
    yield hd
    hd.close()


@pytest.mark.parametrize("tol", [1e-6, 1e-3, 1e-9])
def test_hadamard_then_round_rank256(ttr, h, tol):
    N, I = 5, 20
    print(f"hadamard rank 16 x 16 -> 256, N={N} I={I}, round tol={tol}", flush=True)
    A = synth.random_tt(4, 0, "A", [I] * N, [16] * (N - 1), scaled=True, rank_weights=True)
    B = synth.random_tt(4, 0, "B", [I] * N, [16] * (N - 1), scaled=True, rank_weights=True)
    Xg = h.hadamard(ttr.TT.from_numpy(A), ttr.TT.from_numpy(B))
    assert Xg.R[1:-1] == [256] * (N - 1)
    X = Xg.to_numpy()
    assert O.diff_norm(X, O.hadamard(A, B)) <= 1e-14 * O.norm_ortho(X)
    got, ref = check_round(ttr, h, X, tol, "RLR", sig_rtol=1e-6, norm_rtol=1e-10)
    assert max(O.ranks(got)) < 256
    # bound of Alg. 2
    assert O.diff_norm(got, X) <= tol * O.norm_ortho(X) * (1 + 1e-6)


def test_sum_ranks_65_to_100(ttr, h):
    print("A + B with ranks 65..100", flush=True)
    rng = np.random.default_rng(900)
    I = [30, 25, 40, 35, 28]
    A = rand_tt(rng, I, [40, 50, 45, 30], scale=0.3)
    B = rand_tt(rng, I, [30, 45, 50, 40], scale=0.3)
    X = O.add(1.0, A, 1.0, B)
    assert max(O.ranks(X)) > 64
    got, ref = check_round(ttr, h, X, 1e-8, "RLR", norm_rtol=1e-10)


def test_y_plus_y_rank_80(ttr, h):
    print("Y + Y with Y of rank 40 (formal 80)", flush=True)
    rng = np.random.default_rng(901)
    I = [50, 45, 60, 40]
    Y = rand_tt(rng, I, [40, 40, 40])
    X = O.add(1.0, Y, 1.0, Y)
    got, ref = check_round(ttr, h, X, 1e-10, "RLR", norm_rtol=1e-10)
    assert O.ranks(got) == [1, 40, 40, 40, 1]
    twoY = O.add(2.0, Y, 0.0, Y)
    assert O.diff_norm(got, twoY) <= 1e-12 * O.norm_ortho(twoY)
    # left-orthonormal output cores
    for n in range(len(got) - 1):
        Vn = O.V(got[n])
        assert np.linalg.norm(Vn.T @ Vn - np.eye(Vn.shape[1])) < 1e-12


def test_thin_unfoldings(ttr, h):
    # ranks above I R at the ends: the boundary unfoldings are rank deficient
    print("ranks 70 with I = 8", flush=True)
    rng = np.random.default_rng(902)
    I = [8, 8, 8, 8]
    X = rand_tt(rng, I, [70, 70, 70])
    check_round(ttr, h, X, 1e-10, "RLR", norm_rtol=1e-10)


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
def test_large_rank_mixed(ttr, h, direction):
    # FP32 first Gram passes, FP64 refinement and small factorizations
    print(f"ranks > 64 in mixed precision {direction}", flush=True)
    rng = np.random.default_rng(903)
    I = [30, 25, 40, 35]
    X = O.add(1.0, rand_tt(rng, I, [40, 45, 30]), 1.0, rand_tt(rng, I, [35, 40, 45]))
    check_round(ttr, h, X, 1e-8, direction, rel=1e-8, prec="mixed", norm_rtol=1e-6, sig_rtol=1e-6)


@pytest.mark.parametrize("scale", [1e-30, 1e30])
def test_large_rank_mixed_far_from_unit_norm(ttr, h, scale):
    # the FP32 Gram passes rescale their data by a power of two, so tensors
    # whose entries square below or above FP32's range round as in FP64
    print(f"ranks > 64 in mixed precision, tensor scaled by {scale:g}", flush=True)
    rng = np.random.default_rng(908)
    I = [30, 25, 40, 35]
    X = O.add(1.0, rand_tt(rng, I, [40, 45, 30]), 1.0, rand_tt(rng, I, [35, 40, 45]))
    Z = rand_tt(rng, I, [3, 3, 3])
    Z[0] *= 1e-5
    X = O.add(1.0, X, 1.0, Z)
    X[0] = X[0] * scale
    check_round(ttr, h, X, 1e-4, "RLR", rel=1e-8, prec="mixed", norm_rtol=1e-6, sig_rtol=1e-6)


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
def test_large_rank_mirror_order(ttr, h, direction):
    # the mirror sweep order (LRL) at ranks above 64, against the oracle's LRL
    print(f"ranks 70..100 {direction}", flush=True)
    rng = np.random.default_rng(904)
    I = [12, 20, 15, 18, 10]
    X = O.add(1.0, rand_tt(rng, I, [70, 50, 60, 40], scale=0.5), 1.0, rand_tt(rng, I, [30, 45, 20, 35], scale=0.5))
    Z = rand_tt(rng, I, [5, 5, 5, 5], scale=0.5)
    Z[0] *= 1e-5
    X = O.add(1.0, X, 1.0, Z)
    got, ref = check_round(ttr, h, X, 1e-4, direction, norm_rtol=1e-10, sig_rtol=1e-6)
    assert max(O.ranks(X)) > 64


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_hadamard_rank256_both_orders(ttr, h, direction, prec):
    N, I = 4, 40
    print(f"hadamard rank 256, N={N} I={I}, {direction} {prec}", flush=True)
    A = synth.random_tt(4, 1, "A", [I] * N, [16] * (N - 1), scaled=True, rank_weights=True)
    B = synth.random_tt(4, 1, "B", [I] * N, [16] * (N - 1), scaled=True, rank_weights=True)
    X = h.hadamard(ttr.TT.from_numpy(A), ttr.TT.from_numpy(B)).to_numpy()
    rel = 1e-10 if prec == "fp64" else 1e-8
    got, ref = check_round(ttr, h, X, 1e-6, direction, rel=rel, prec=prec, sig_rtol=1e-6,
                           norm_rtol=1e-10 if prec == "fp64" else 1e-6)
    assert max(O.ranks(got)) < 256


LARGE_SHAPES = [
    ([30, 25, 40, 35], [80, 100, 70]),
    ([9, 300, 200, 7], [9, 256, 7]),          # rank 256 between thin end cores
    ([50, 40, 60], [65, 120]),
]


@pytest.mark.parametrize("I,r", LARGE_SHAPES)
def test_large_rank_dot_and_norms(ttr, h, I, r):
    print(f"dot / norms at ranks {r}", flush=True)
    rng = np.random.default_rng(905)
    X = rand_tt(rng, I, r, scale=0.1)
    Y = rand_tt(rng, I, [max(1, x // 2) for x in r], scale=0.1)
    gx, gy = ttr.TT.from_numpy(X), ttr.TT.from_numpy(Y)
    ref = O.dot(X, Y)
    scale = O.norm_ortho(X) * O.norm_ortho(Y)
    assert abs(h.dot(gx, gy) - ref) <= 1e-12 * scale
    assert abs(h.dot(gy, gx) - ref) <= 1e-12 * scale
    n = O.norm_ortho(X)
    assert abs(h.norm(gx, "gram") - n) <= 1e-12 * n
    assert abs(h.norm(gx, "ortho") - n) <= 1e-12 * n
    with pytest.raises(ttr.TTRError) as e:
        h.norm(gx, "sym")
    assert e.value.code == 7


def test_large_rank_norm_small_difference(ttr, h):
    # the orthonormalization norm resolves ||(X + 1e-9 Z) - X|| at ranks > 64
    print("norm of a difference tensor at ranks > 64", flush=True)
    rng = np.random.default_rng(906)
    I = [20, 30, 25, 15]
    X = rand_tt(rng, I, [40, 50, 35])
    Z = rand_tt(rng, I, [3, 3, 3])
    D = O.add(1.0, O.add(1.0, X, 1e-9, Z), -1.0, X)
    assert max(O.ranks(D)) > 64
    ref = 1e-9 * O.norm_ortho(Z)
    assert abs(h.norm(ttr.TT.from_numpy(D), "ortho") - ref) <= 1e-6 * ref


@pytest.mark.parametrize("side", ["right", "left"])
@pytest.mark.parametrize("I,r", LARGE_SHAPES)
def test_large_rank_orthogonalize(ttr, h, side, I, r):
    print(f"orthogonalize {side} ranks {r}", flush=True)
    rng = np.random.default_rng(907)
    X = rand_tt(rng, I, r, scale=2.0)
    g = ttr.TT.from_numpy(X)
    h.orthogonalize(g, side)
    Y = g.to_numpy()
    N = len(Y)
    nrm = O.norm_ortho(X)
    assert O.diff_norm(Y, X) <= 1e-13 * nrm * max(1, N)
    if side == "right":
        for n in range(1, N):
            Hn = O.H(Y[n])
            assert np.linalg.norm(Hn @ Hn.T - np.eye(Hn.shape[0])) < 1e-13 * Hn.shape[0]
    else:
        for n in range(N - 1):
            Vn = O.V(Y[n])
            assert np.linalg.norm(Vn.T @ Vn - np.eye(Vn.shape[1])) < 1e-13 * Vn.shape[1]
    # the oracle's Householder sweep gives the same ranks on generic inputs
    assert O.ranks(Y) == O.ranks(O.orthogonalize(X, side))


def test_hadamard_workload_full_N_reduced_I(ttr, h):
    # the Hadamard-then-round workload at its full N = 10 and ranks 16 x 16 -> 256,
    # with I = 96 instead of 16384 so that the oracle stays within seconds
    print("hadamard workload N=10 I=96 tol 1e-6", flush=True)
    d = synth.hadamard_r256(I_override=96)
    Xg = h.hadamard(ttr.TT.from_numpy(d["A"]), ttr.TT.from_numpy(d["B"]))
    X = Xg.to_numpy()
    got, ref = check_round(ttr, h, X, d["tol"], "RLR", sig_rtol=1e-6, norm_rtol=1e-10)
    print(f"  ranks {O.ranks(got)}", flush=True)


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_large_rank_explicit_factors(ttr, h, direction, prec):
    # explicit orthonormal factors (§3.4 Alg. 5, §4.3.2) at rank 256
    N, I = 4, 40
    print(f"hadamard rank 256, explicit factors, {direction} {prec}", flush=True)
    A = synth.random_tt(4, 2, "A", [I] * N, [16] * (N - 1), scaled=True, rank_weights=True)
    B = synth.random_tt(4, 2, "B", [I] * N, [16] * (N - 1), scaled=True, rank_weights=True)
    X = h.hadamard(ttr.TT.from_numpy(A), ttr.TT.from_numpy(B)).to_numpy()
    g = ttr.TT.from_numpy(X)
    Yg = h.round(g, 1e-6, direction + "_EXPLICIT", prec)
    got = Yg.to_numpy()
    ref = O.round_tt(X, 1e-6, direction)
    assert O.ranks(got) == O.ranks(ref), (O.ranks(got), O.ranks(ref))
    rel = O.diff_norm(got, ref) / O.norm_ortho(ref)
    print(f"  ranks {O.ranks(got)[1:-1]} rel diff {rel:.3e}", flush=True)
    assert rel <= (1e-10 if prec == "fp64" else 1e-8)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("ra,rb", [(16, 16), (7, 9), (3, 16)])
def test_round_hadamard_implicit(ttr, h, prec, ra, rb):
    # rounding of A * B without forming it (§3.2.2, closing remark) against the
    # oracle's rounding of the formed product
    N, I = 5, 30
    print(f"implicit Hadamard rounding, ranks {ra} x {rb}, {prec}", flush=True)
    A = synth.random_tt(4, 3, "A", [I] * N, [ra] * (N - 1), scaled=True, rank_weights=True)
    B = synth.random_tt(4, 3, "B", [I] * N, [rb] * (N - 1), scaled=True, rank_weights=True)
    gA, gB = ttr.TT.from_numpy(A), ttr.TT.from_numpy(B)
    Yg, nrm = h.round_hadamard(gA, gB, 1e-6, "RLR", prec, return_norm=True)
    got = Yg.to_numpy()
    X = O.hadamard(A, B)
    ref, info = O.round_tt(X, 1e-6, "RLR", return_info=True)
    assert O.ranks(got) == O.ranks(ref), (O.ranks(got), O.ranks(ref))
    rel = O.diff_norm(got, ref) / O.norm_ortho(ref)
    print(f"  ranks {O.ranks(got)[1:-1]} rel diff {rel:.3e}", flush=True)
    assert rel <= (1e-10 if prec == "fp64" else 1e-8)
    assert abs(nrm - info["norm"]) <= (1e-10 if prec == "fp64" else 1e-6) * info["norm"]
    with pytest.raises(ttr.TTRError) as e:
        h.round_hadamard(gA, gB, 1e-6, "LRL", prec)
    assert e.value.code == 7


@pytest.mark.parametrize("N", [1, 2, 3])
def test_round_hadamard_implicit_short_trains(ttr, h, N):
    # the boundary cases of the implicit product: N = 1 (the product itself),
    # N = 2 (one link: only the last core is formed), N = 3, at tol 0 and 1e-3
    rng = np.random.default_rng(940 + N)
    I = [23, 17, 29][:N]
    A = rand_tt(rng, I, [5, 4][: N - 1])
    B = rand_tt(rng, I, [3, 6][: N - 1])
    X = O.hadamard(A, B)
    for tol in (0.0, 1e-3):
        print(f"implicit Hadamard rounding N={N} tol={tol}", flush=True)
        got = h.round_hadamard(ttr.TT.from_numpy(A), ttr.TT.from_numpy(B), tol).to_numpy()
        ref = O.round_tt(X, tol, "RLR")
        assert O.ranks(got) == O.ranks(ref), (O.ranks(got), O.ranks(ref))
        assert O.diff_norm(got, ref) <= 1e-10 * O.norm_ortho(ref)
