"""GPU parity of TT rounding at ranks above 64 (the GEMM-based path, up to
256) against the FP64 oracle: the Hadamard-then-round workload at reduced mode
sizes (A, B rank 16 with slice weights 2^-b, X = A * B of rank 256), sums of
ranks 65..100, and the rank-deficient Y + Y.
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


def test_large_rank_mixed_runs_fp64(ttr, h):
    print("ranks > 64 with prec mixed", flush=True)
    rng = np.random.default_rng(903)
    I = [30, 25, 40, 35]
    X = O.add(1.0, rand_tt(rng, I, [40, 45, 30]), 1.0, rand_tt(rng, I, [35, 40, 45]))
    check_round(ttr, h, X, 1e-8, "RLR", prec="mixed", norm_rtol=1e-10)


def test_large_rank_lrl_unsupported(ttr, h):
    rng = np.random.default_rng(904)
    X = rand_tt(rng, [10, 10, 10], [70, 70])
    with pytest.raises(ttr.TTRError) as e:
        h.round(ttr.TT.from_numpy(X), 1e-8, "LRL")
    assert e.value.code == 7


def test_hadamard_workload_full_N_reduced_I(ttr, h):
    # the Hadamard-then-round workload at its full N = 10 and ranks 16 x 16 -> 256,
    # with I = 96 instead of 16384 so that the oracle stays within seconds
    print("hadamard workload N=10 I=96 tol 1e-6", flush=True)
    d = synth.hadamard_r256(I_override=96)
    Xg = h.hadamard(ttr.TT.from_numpy(d["A"]), ttr.TT.from_numpy(d["B"]))
    X = Xg.to_numpy()
    got, ref = check_round(ttr, h, X, d["tol"], "RLR", sig_rtol=1e-6, norm_rtol=1e-10)
    print(f"  ranks {O.ranks(got)}", flush=True)
