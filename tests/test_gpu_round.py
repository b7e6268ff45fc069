"""GPU parity of TT rounding (Alg. 2, RLR and LRL) against the FP64 oracle.

Tensors are compared through the oracle's cancellation-free difference norm
(singular vectors are not unique; App. A makes the tensor and the per-link
singular values gauge-invariant).  FP64 bar: equal ranks and
||X~_gpu - X~_oracle|| <= 1e-10 ||X~_oracle||.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu

REL = 1e-10


def rand_tt(rng, I, r, scale=1.0):
    R = [1] + list(r) + [1]
    return [np.asfortranarray(scale * rng.standard_normal((R[n], I[n], R[n + 1]))) for n in range(len(I))]


@pytest.fixture(scope="module")
def h(ttr):
    hd = ttr.Handle(0)
    yield hd
    hd.close()


def check_round(ttr, h, X, tol, direction, rel=REL, sig_rtol=1e-9, prec="fp64", norm_rtol=1e-12):
    g = ttr.TT.from_numpy(X)
    Yg, nrm = h.round(g, tol, direction, prec, return_norm=True)
    got = Yg.to_numpy()
    ref, info = O.round_tt(X, tol, direction, return_info=True)
    assert O.ranks(got) == O.ranks(ref), (O.ranks(got), O.ranks(ref))
    nref = O.norm_ortho(ref)
    d = O.diff_norm(got, ref)
    print(f"  ranks {O.ranks(got)[1:-1]} rel diff {d / max(nref, 1e-300):.3e}", flush=True)
    assert d <= rel * max(nref, 1e-300), (d, nref)
    assert math.isclose(nrm, info["norm"], rel_tol=norm_rtol)
    st = h.round_stats()
    for l, (s_gpu, s_ref) in enumerate(zip(st["sigmas"], info["sigmas"])):
        k = min(len(s_gpu), len(s_ref))
        big = np.asarray(s_ref[:k]) > 1e-6 * s_ref[0]
        assert np.allclose(np.asarray(s_gpu[:k])[big], np.asarray(s_ref[:k])[big], rtol=sig_rtol), l
    return got, ref


def orthonormality(cores, direction):
    """max_n ||V_n^T V_n - I||_F (RLR, n < N) or ||H_n H_n^T - I||_F (LRL, n > 1)."""
    worst = 0.0
    N = len(cores)
    for n in (range(N - 1) if direction == "RLR" else range(1, N)):
        M = O.V(cores[n]) if direction == "RLR" else O.H(cores[n]).T
        worst = max(worst, float(np.linalg.norm(M.T @ M - np.eye(M.shape[1]))))
    return worst


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
def test_round_yy_small_y_plus_y(ttr, h, direction):
    print(f"round yy_small Y+Y {direction}", flush=True)
    d = synth.yy_small()
    Y = d["Y"]
    X = O.add(1.0, Y, 1.0, Y)
    got, ref = check_round(ttr, h, X, d["tol"], direction)
    assert O.ranks(got) == [1, 5, 5, 5, 1]
    twoY = O.add(2.0, Y, 0.0, Y)
    assert O.diff_norm(got, twoY) <= 1e-12 * O.norm_ortho(twoY)
    # output orthonormality (RLR: left-orthonormal cores 1..N-1)
    N = len(got)
    if direction == "RLR":
        for n in range(N - 1):
            Vn = O.V(got[n])
            assert np.linalg.norm(Vn.T @ Vn - np.eye(Vn.shape[1])) < 1e-13 * Vn.shape[1]
    else:
        for n in range(1, N):
            Hn = O.H(got[n])
            assert np.linalg.norm(Hn @ Hn.T - np.eye(Hn.shape[0])) < 1e-13 * Hn.shape[0]


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
def test_round_sum_r40_shape_small_I(ttr, h, direction):
    # the A+B workload's structure (N=16, ranks 20 + 20 -> 40, scaled) at I = 512
    print(f"round A+B N=16 I=512 {direction}", flush=True)
    d = synth.sum_r40(I_override=512)
    X = O.add(1.0, d["A"], 1.0, d["B"])
    got, ref = check_round(ttr, h, X, d["tol"], direction)
    assert O.ranks(got)[1:-1] == [40] * 15


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
def test_round_sum_r50_shape_small_I(ttr, h, direction):
    # the A + B + 1e-6 C workload's structure (ranks 50) at I = 400
    print(f"round A+B+1e-6C N=16 I=400 {direction}", flush=True)
    d = synth.sum_r50(I_override=400)
    X = O.add(1.0, O.add(1.0, d["A"], 1.0, d["B"]), 1.0, d["C"])
    h.set_profiling(True)
    got, ref = check_round(ttr, h, X, d["tol"], direction, sig_rtol=1e-6)
    prof = h.profile()
    h.set_profiling(False)
    assert O.ranks(got)[1:-1] == [50] * 15
    # the 1e-6 part makes every truncation step ill conditioned: the refinement
    # runs on a materialized core with the matrix-core kernels
    assert prof["k_gram_fac"]["count"] >= 14, prof["k_gram_fac"]
    assert prof["k_apply_fac2"]["count"] >= 14, prof["k_apply_fac2"]
    assert prof["k_gram"]["count"] == 0 and prof["k_apply"]["count"] == 0
    # output orthonormality (RLR: left-orthonormal cores 1..N-1)
    # same bound as the oracle's orthonormality pin (1e-13 R), here with a
    # condition number of ~1e6 in every truncation step
    worst = orthonormality(got, direction)
    print(f"  output orthonormality {worst:.2e}", flush=True)
    assert worst < 1e-13 * 50


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
def test_round_batched_members(ttr, h, direction):
    # a few members of the batched workload (Y + Y + 1e-9 E), full size
    shapes = synth.batched_shapes(512)
    for t in (0, 1, 7, 100):
        I, r = shapes[t]
        print(f"round Y+Y+E member {t} I={I} r={r} {direction}", flush=True)
        Yc = synth.random_tt(3, t, "Y", I, r, scaled=True)
        E = synth.random_tt(3, t, "E", I, [2] * 7, scaled=True, first_core_factor=1e-9)
        X = O.add(1.0, O.add(1.0, Yc, 1.0, Yc), 1.0, E)
        got, ref = check_round(ttr, h, X, synth.TOL[3], direction, sig_rtol=1e-6)
        assert O.ranks(got)[1:-1] == list(r)


@pytest.mark.parametrize("tol", [0.5, 1e-2, 1e-5, 1e-9])
@pytest.mark.parametrize("direction", ["RLR", "LRL"])
def test_round_graded_spectrum(ttr, h, tol, direction):
    # content at 1e-3, 1e-6, 1e-9 of the leading part: truncation bites at
    # different links depending on tol
    print(f"round graded tol={tol} {direction}", flush=True)
    rng = np.random.default_rng(200)
    I = [30, 45, 37, 50, 28]
    X = rand_tt(rng, I, [5, 6, 6, 4])
    for eps, r in ((1e-3, [3, 3, 3, 3]), (1e-6, [2, 2, 2, 2]), (1e-9, [2, 3, 2, 2])):
        Z = rand_tt(rng, I, r)
        Z[0] = Z[0] * eps
        X = O.add(1.0, X, 1.0, Z)
    check_round(ttr, h, X, tol, direction, sig_rtol=1e-5)


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
def test_round_edge_cases(ttr, h, direction):
    rng = np.random.default_rng(201)
    print(f"round edge cases {direction}", flush=True)
    # N = 2 (one link), I_n = 1 modes, tol = 0 on a generic TT, huge tol
    check_round(ttr, h, rand_tt(rng, [33, 41], [7]), 1e-3, direction)
    check_round(ttr, h, rand_tt(rng, [7, 1, 9, 1, 5], [3, 3, 4, 2]), 1e-4, direction)
    check_round(ttr, h, rand_tt(rng, [20, 30, 25], [4, 5]), 0.0, direction)
    got, ref = check_round(ttr, h, rand_tt(rng, [20, 30, 25], [4, 5]), 10.0, direction)
    assert O.ranks(got) == [1, 1, 1, 1]
    # N = 1: copy
    X1 = rand_tt(rng, [17], [])
    g = ttr.TT.from_numpy(X1)
    out = h.round(g, 0.1, direction).to_numpy()
    assert np.array_equal(out[0], X1[0])
    # zero tensor: rank-1 zero TT
    Z = [np.zeros_like(c) for c in rand_tt(rng, [10, 12, 9], [3, 4])]
    out = h.round(ttr.TT.from_numpy(Z), 1e-3, direction).to_numpy()
    assert O.ranks(out) == [1, 1, 1, 1]
    assert all(np.count_nonzero(c) == 0 for c in out)


def test_round_error_bound_and_idempotence(ttr, h):
    print("round bound + idempotence", flush=True)
    rng = np.random.default_rng(202)
    I = [60, 70, 50, 40]
    X = rand_tt(rng, I, [6, 8, 5])
    Z = rand_tt(rng, I, [3, 3, 3])
    Z[0] *= 1e-2
    X = O.add(1.0, X, 1.0, Z)
    tol = 3e-3
    g = ttr.TT.from_numpy(X)
    Yg = h.round(g, tol)
    Y = Yg.to_numpy()
    assert O.diff_norm(Y, X) <= tol * O.norm_ortho(X)
    Y2 = h.round(Yg, 0.0).to_numpy()
    assert O.ranks(Y2) == O.ranks(Y)
    assert O.diff_norm(Y2, Y) <= 1e-13 * O.norm_ortho(Y)


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_round_explicit_factors(ttr, h, direction, prec):
    # the explicit variants of §4.3.2: orthonormal cores written first (§3.4
    # Alg. 5), truncation over the written cores; same result as the oracle's
    # rounding in the same sweep order
    print(f"round, explicit orthonormal factors, {direction} {prec}", flush=True)
    rng = np.random.default_rng(210)
    I = [300, 250, 400, 280, 350]
    X = O.add(1.0, rand_tt(rng, I, [20, 25, 18, 22], scale=0.2), 1.0, rand_tt(rng, I, [15, 10, 20, 12], scale=0.2))
    Z = rand_tt(rng, I, [4, 4, 4, 4], scale=0.2)
    Z[0] *= 1e-6
    X = O.add(1.0, X, 1.0, Z)
    g = ttr.TT.from_numpy(X)
    Yg, nrm = h.round(g, 1e-5, direction + "_EXPLICIT", prec, return_norm=True)
    got = Yg.to_numpy()
    ref, info = O.round_tt(X, 1e-5, direction, return_info=True)
    assert O.ranks(got) == O.ranks(ref), (O.ranks(got), O.ranks(ref))
    rel = O.diff_norm(got, ref) / O.norm_ortho(ref)
    print(f"  ranks {O.ranks(got)[1:-1]} rel diff {rel:.3e}", flush=True)
    assert rel <= (1e-10 if prec == "fp64" else 1e-8)
    assert math.isclose(nrm, info["norm"], rel_tol=1e-12 if prec == "fp64" else 1e-6)
    # output orthonormality as for the implicit variant
    assert orthonormality(got, direction) < (1e-12 if prec == "fp64" else 1e-6)


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
@pytest.mark.parametrize("rank", [5, 80])
def test_round_tol0_rank_deficient_against_oracle(ttr, h, direction, rank):
    # tol = 0 on Y + Y (every unfolding exactly rank deficient): the oracle's
    # Householder QR keeps the formal ranks with rounding-level singular
    # values, the GPU keeps the numerical ranks.  Both must give the same
    # tensor (2Y), and the GPU's ranks must be the oracle's count of singular
    # values above rounding level (1e-12 sigma_1) at each link.
    print(f"round tol=0 Y+Y rank {rank} {direction}", flush=True)
    rng = np.random.default_rng(211 + rank)
    I = [30, 40, 35, 25] if rank == 5 else [12, 10, 9, 11]
    Yc = rand_tt(rng, I, [rank] * 3)
    X = O.add(1.0, Yc, 1.0, Yc)
    Yg = h.round(ttr.TT.from_numpy(X), 0.0, direction).to_numpy()
    ref, info = O.round_tt(X, 0.0, direction, return_info=True)
    num = [1] + [int(np.sum(np.asarray(s) > 1e-12 * s[0])) for s in info["sigmas"]] + [1]
    assert O.ranks(ref) != num  # the oracle keeps rounding-level directions
    assert O.ranks(Yg) == num, (O.ranks(Yg), num, O.ranks(ref))
    assert O.diff_norm(Yg, ref) <= 1e-12 * O.norm_ortho(ref)


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
def test_round_long_train_stats(ttr, h, direction):
    # N = 70 cores: more links than the per-link statistics hold (64); links
    # past that are not reported and nothing past the statistics is written
    # (the handle keeps working)
    print(f"round N=70 {direction}", flush=True)
    rng = np.random.default_rng(230)
    N = 70
    I = [2] * N
    Yc = rand_tt(rng, I, [2] * (N - 1))
    X = O.add(1.0, Yc, 1.0, rand_tt(rng, I, [2] * (N - 1), scale=1e-3))
    got = h.round(ttr.TT.from_numpy(X), 1e-2, direction).to_numpy()
    ref, info = O.round_tt(X, 1e-2, direction, return_info=True)
    assert O.ranks(got) == O.ranks(ref)
    assert O.diff_norm(got, ref) <= 1e-10 * O.norm_ortho(ref)
    st = h.round_stats()
    assert len(st["sigmas"]) == 64 and len(st["tail2"]) == 64
    for l in range(64):
        s_ref = np.asarray(info["sigmas"][l])
        s_gpu = np.asarray(st["sigmas"][l])
        k = min(len(s_gpu), len(s_ref))
        if k:
            big = s_ref[:k] > 1e-6 * s_ref[0]
            assert np.allclose(s_gpu[:k][big], s_ref[:k][big], rtol=1e-9), l
    # the handle still works
    check_round(ttr, h, rand_tt(rng, [20, 30, 25], [4, 5]), 1e-3, direction)
