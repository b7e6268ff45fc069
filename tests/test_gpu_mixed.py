"""GPU parity of the mixed-precision TT rounding (TTR_MIXED) against the FP64
oracle.

In TTR_MIXED the first Gram pass of every QR-by-Gram factorization runs on the
FP32 matrix cores (slices rounded to FP32 on load, FP32 products and
accumulation); refinement passes, every small factorization and every written
core stay FP64.  A factorization is accepted once its factor is orthonormal to
about 1e-5, so the tensor keeps FP64 accuracy (each R factor is the exact
inverse of the applied basis change) while the output cores are orthonormal
only to that level.  Bar: equal ranks and
||X~_gpu - X~_oracle|| <= 1e-8 ||X~_oracle||.
"""
import numpy as np
import pytest

import oracle as O
import synth
from test_gpu_round import check_round, orthonormality, rand_tt

pytestmark = pytest.mark.gpu

REL_MIXED = 1e-8
ORTH_MIXED = 1e-4


@pytest.fixture(scope="module")
def h(ttr):
    hd = ttr.Handle(0)
    yield hd
    hd.close()


def run(ttr, h, X, tol, direction, orth=ORTH_MIXED):
    h.set_profiling(True)
    got, ref = check_round(ttr, h, X, tol, direction, rel=REL_MIXED, sig_rtol=1e-4, prec="mixed",
                           norm_rtol=1e-6)
    prof = h.profile()
    h.set_profiling(False)
    worst = orthonormality(got, direction)
    print(f"  output orthonormality {worst:.2e}", flush=True)
    assert worst < orth
    # the first passes really ran on the FP32 matrix cores
    assert prof["k_gram_right_factor_f32"]["count"] + prof["k_gram_left_factor_f32"]["count"] >= len(X) - 1
    return got, ref, prof


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
def test_mixed_yy_small_y_plus_y(ttr, h, direction):
    print(f"mixed yy_small Y+Y {direction}", flush=True)
    d = synth.yy_small()
    Y = d["Y"]
    X = O.add(1.0, Y, 1.0, Y)
    got, ref, _ = run(ttr, h, X, d["tol"], direction)
    assert O.ranks(got) == [1, 5, 5, 5, 1]


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
def test_mixed_sum_r40_shape(ttr, h, direction):
    print(f"mixed A+B N=16 I=512 {direction}", flush=True)
    d = synth.sum_r40(I_override=512)
    X = O.add(1.0, d["A"], 1.0, d["B"])
    got, ref, prof = run(ttr, h, X, d["tol"], direction)
    assert O.ranks(got)[1:-1] == [40] * 15
    # well conditioned: one FP32 pass per factorization, no FP64 Gram pass
    assert prof["k_gram_right_factor"]["count"] + prof["k_gram_left_factor"]["count"] == 0


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
def test_mixed_sum_r50_shape(ttr, h, direction):
    # A + B + 1e-6 C: FP32 cannot resolve the 1e-6 part (sigma^2 ~ 1e-12), the
    # FP64 refinement pass on the materialized core recovers it
    print(f"mixed A+B+1e-6C N=16 I=400 {direction}", flush=True)
    d = synth.sum_r50(I_override=400)
    X = O.add(1.0, O.add(1.0, d["A"], 1.0, d["B"]), 1.0, d["C"])
    got, ref, prof = run(ttr, h, X, d["tol"], direction)
    assert O.ranks(got)[1:-1] == [50] * 15
    # refinement passes on materialized cores, all on the matrix cores (RLR: in
    # the truncation sweep; LRL: in the orthonormalization sweep, where the
    # scaled first core sits)
    assert prof["k_gram_fac"]["count"] >= 14
    assert prof["k_gram"]["count"] == 0 and prof["k_apply"]["count"] == 0


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
def test_mixed_batched_members(ttr, h, direction):
    shapes = synth.batched_shapes(512)
    for t in (0, 1, 7, 100):
        I, r = shapes[t]
        print(f"mixed Y+Y+E member {t} I={I} r={r} {direction}", flush=True)
        Yc = synth.random_tt(3, t, "Y", I, r, scaled=True)
        E = synth.random_tt(3, t, "E", I, [2] * 7, scaled=True, first_core_factor=1e-9)
        X = O.add(1.0, O.add(1.0, Yc, 1.0, Yc), 1.0, E)
        got, ref, _ = run(ttr, h, X, synth.TOL[3], direction)
        assert O.ranks(got)[1:-1] == list(r)


@pytest.mark.parametrize("tol", [0.5, 1e-2, 1e-5])
@pytest.mark.parametrize("direction", ["RLR", "LRL"])
def test_mixed_graded_spectrum(ttr, h, tol, direction):
    print(f"mixed graded tol={tol} {direction}", flush=True)
    rng = np.random.default_rng(200)
    I = [30, 45, 37, 50, 28]
    X = rand_tt(rng, I, [5, 6, 6, 4])
    for eps, r in ((1e-3, [3, 3, 3, 3]), (1e-6, [2, 2, 2, 2]), (1e-9, [2, 3, 2, 2])):
        Z = rand_tt(rng, I, r)
        Z[0] = Z[0] * eps
        X = O.add(1.0, X, 1.0, Z)
    run(ttr, h, X, tol, direction)


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
@pytest.mark.parametrize("scale", [1e-30, 1e30, 1e-100])
def test_mixed_far_from_unit_norm(ttr, h, direction, scale):
    # the FP32 Gram passes scale their data and factor by powers of two chosen
    # from the largest entries, so products whose squares leave FP32's range
    # round as in FP64.  1e+-30 is spread over the cores (the triangular
    # factors passed between cores carry the tensor's scale into the products
    # C = M T); 1e-100 sits in one core.
    print(f"mixed precision, tensor scaled by {scale:g} {direction}", flush=True)
    rng = np.random.default_rng(909)
    I = [40, 30, 50, 35]
    X = O.add(1.0, rand_tt(rng, I, [7, 9, 8]), 1.0, rand_tt(rng, I, [6, 5, 7]))
    Z = rand_tt(rng, I, [2, 2, 2])
    Z[0] *= 1e-6
    X = O.add(1.0, X, 1.0, Z)
    if scale > 1e-50:
        X = [c * scale ** (1.0 / len(X)) for c in X]
    else:
        X[0] = X[0] * scale
    run(ttr, h, X, 1e-8, direction)
