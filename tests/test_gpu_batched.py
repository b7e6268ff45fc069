"""GPU parity of the batched rounding (ttr_round_batched: one captured graph
for many tensors, decisions on the device) against the FP64 oracle.

Inputs follow the batched workload (Y + Y + 1e-9 E with per-tensor mode sizes
and ranks), with mode sizes capped so the oracle stays fast.  Bar as for the
single path: equal ranks, ||X~_gpu - X~_oracle|| <= 1e-10 ||X~_oracle|| in FP64
and 1e-8 in mixed precision.
"""
import numpy as np
import pytest

import oracle as O
import synth
from test_gpu_round import rand_tt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h(ttr):
    hd = ttr.Handle(0)
    yield hd
    hd.close()


def batch_inputs(count, I_cap, start=0):
    shapes = synth.batched_shapes(512)
    Xs, rs = [], []
    for t in range(start, start + count):
        I, r = shapes[t]
        I = [min(x, I_cap) for x in I]
        Y = synth.random_tt(3, t, "Y", I, r, scaled=True)
        E = synth.random_tt(3, t, "E", I, [2] * 7, scaled=True, first_core_factor=1e-9)
        Xs.append(O.add(1.0, O.add(1.0, Y, 1.0, Y), 1.0, E))
        rs.append(list(r))
    return Xs, rs


def run_batched(ttr, h, Xs, tols, prec="fp64", tune=False):
    g = [ttr.TT.from_numpy(X) for X in Xs]
    Ys, ranks = h.round_batched(g, tols, prec, tune=tune)
    ttr.Handle.sync_ranks(Ys, ranks)
    return g, Ys, [Y.to_numpy() for Y in Ys]


def check_against_oracle(Xs, got, tols, rel):
    worst = 0.0
    for t, (X, Yg) in enumerate(zip(Xs, got)):
        tol = tols[t] if isinstance(tols, (list, tuple)) else tols
        ref = O.round_tt(X, tol, "RLR")
        assert O.ranks(Yg) == O.ranks(ref), (t, O.ranks(Yg), O.ranks(ref))
        d = O.diff_norm(Yg, ref) / max(O.norm_ortho(ref), 1e-300)
        worst = max(worst, d)
        assert d <= rel, (t, d)
    return worst


@pytest.mark.parametrize("prec,rel", [("fp64", 1e-10), ("mixed", 1e-8)])
def test_batched_y_plus_y_plus_e(ttr, h, prec, rel):
    print(f"batched Y+Y+E 24 tensors I<=160 {prec}", flush=True)
    Xs, rs = batch_inputs(24, 160)
    _, _, got = run_batched(ttr, h, Xs, synth.TOL[3], prec)
    for Yg, r in zip(got, rs):
        assert O.ranks(Yg)[1:-1] == r
    worst = check_against_oracle(Xs, got, synth.TOL[3], rel)
    print(f"  worst rel diff {worst:.2e}", flush=True)


def test_batched_replay_is_deterministic_and_matches_single(ttr, h):
    print("batched replay vs single path", flush=True)
    Xs, _ = batch_inputs(12, 120, start=100)
    g = [ttr.TT.from_numpy(X) for X in Xs]
    Ys, ranks = h.round_batched(g, synth.TOL[3])
    first = [c.clone() for Y in Ys for c in Y.cores]
    r1 = ranks.clone()
    Ys, ranks = h.round_batched(g, synth.TOL[3], outs=Ys, ranks=ranks)  # graph replay
    second = [c for Y in Ys for c in Y.cores]
    assert bool((r1 == ranks).all())
    for a, b in zip(first, second):
        assert bool((a == b).all())
    ttr.Handle.sync_ranks(Ys, ranks)
    for X, Yb in zip(g, Ys):
        Ysg = h.round(X, synth.TOL[3])
        assert Ysg.R == Yb.R
        ref = Ysg.to_numpy()
        assert O.diff_norm(Yb.to_numpy(), ref) <= 1e-10 * O.norm_ortho(ref)


@pytest.mark.parametrize("prec,rel", [("fp64", 1e-10), ("mixed", 1e-8)])
def test_batched_graded_mixed_tolerances(ttr, h, prec, rel):
    # tensors with content at 1e-3, 1e-6, 1e-9 and per-tensor tolerances:
    # truncation and multi-pass factorizations in both sweeps
    print(f"batched graded spectra {prec}", flush=True)
    rng = np.random.default_rng(300)
    Xs, tols = [], []
    for t in range(10):
        I = [int(x) for x in rng.integers(20, 60, size=5)]
        X = rand_tt(rng, I, [int(x) for x in rng.integers(2, 7, size=4)])
        for eps in (1e-3, 1e-6, 1e-9):
            Z = rand_tt(rng, I, [int(x) for x in rng.integers(1, 4, size=4)])
            Z[0] = Z[0] * eps
            X = O.add(1.0, X, 1.0, Z)
        Xs.append(X)
        tols.append([0.5, 1e-2, 1e-5, 1e-4, 0.1][t % 5])
    _, _, got = run_batched(ttr, h, Xs, tols, prec)
    worst = check_against_oracle(Xs, got, tols, rel)
    print(f"  worst rel diff {worst:.2e}", flush=True)


def test_batched_autotuner(ttr, h):
    print("batched autotuner", flush=True)
    Xs, rs = batch_inputs(16, 200, start=300)
    _, _, got = run_batched(ttr, h, Xs, synth.TOL[3], tune=True)
    plan = h.batch_plan()
    assert plan["count"] == 16 and len(plan["candidates"]) == 8
    best = min(plan["candidates"], key=lambda c: c["ms"])
    assert (plan["spw_target"], plan["grid_cap"]) == (best["spw"], best["grid"])
    assert plan["graph_nodes"] > 0
    for Yg, r in zip(got, rs):
        assert O.ranks(Yg)[1:-1] == r


def test_batched_argument_errors(ttr, h):
    import ctypes
    print("batched argument errors", flush=True)
    Xs, _ = batch_inputs(2, 64)
    g = [ttr.TT.from_numpy(X) for X in Xs]
    lib = ttr.load()
    outs = [ttr.TT.empty(X.I, [X.R[n] * X.I[n] * X.R[n + 1] for n in range(X.N)]) for X in g]
    import torch
    ranks = torch.zeros((2, 9), dtype=torch.int64, device="cuda")

    def call(xs_list, count, direction=ttr.TTR_RLR, tl=1e-7):
        xs = (ttr._TTStruct * len(xs_list))(*[X._struct() for X in xs_list])
        ys = (ttr._TTStruct * len(xs_list))(*[Y._struct() for Y in outs[: len(xs_list)]])
        tv = (ctypes.c_double * max(count, 1))(*([tl] * max(count, 1)))
        return lib.ttr_round_batched(h.h, count, xs, tv, direction, ttr.TTR_FP64, ys,
                                     ctypes.c_void_p(ranks.data_ptr()), 0)

    assert call(g, 2, direction=ttr.TTR_LRL) == 7   # RLR only
    assert call(g, 0) == 1                           # empty batch
    assert call(g, 2, tl=-1.0) == 1                  # negative tolerance
    short = ttr.TT.from_numpy(g[1].to_numpy()[:5])   # N = 5 in a batch of N = 8
    short.R[-1] = 1
    assert call([g[0], short], 2) == 2


def test_batched_workspace_through_torch_allocator(ttr):
    # the batched plan's workspace comes from the registered allocator and the
    # results are unchanged
    import torch
    print("batched allocator", flush=True)
    Xs, rs = batch_inputs(16, 256, start=16)
    tol = synth.TOL[3]
    hd = ttr.Handle(0)
    stream = torch.cuda.current_stream(0)
    live = {}

    def alloc(n):
        p = torch.cuda.caching_allocator_alloc(n, 0, stream)
        live[p] = n
        return p

    def free(p):
        live.pop(p)
        torch.cuda.caching_allocator_delete(p)

    hd.set_allocator(alloc, free)
    _, _, got = run_batched(ttr, hd, Xs, tol)
    assert live  # the plan's workspace is held through the allocator
    for X, r, Yg in zip(Xs, rs, got):
        assert O.ranks(Yg) == [1] + r + [1]
    check_against_oracle(Xs, got, tol, 1e-10)
    hd.set_allocator(None, None)
    assert not live  # and handed back
    hd.close()


def test_batched_replan_while_previous_batch_runs(ttr):
    # batch A is enqueued and, without waiting, a different batch B is
    # submitted on the same handle under the torch allocator: building B's plan
    # frees A's plan, which must wait for A's replay first.  Both results
    # against the oracle.
    import torch
    print("batched re-plan while a replay runs", flush=True)
    XA, rA = batch_inputs(12, 200, start=40)
    XB, rB = batch_inputs(9, 150, start=60)
    tol = synth.TOL[3]
    hd = ttr.Handle(0)
    hd.use_torch_allocator()
    gA = [ttr.TT.from_numpy(X) for X in XA]
    gB = [ttr.TT.from_numpy(X) for X in XB]
    YA, ranksA = hd.round_batched(gA, tol)   # asynchronous
    YB, ranksB = hd.round_batched(gB, tol)   # a new plan at once
    torch.cuda.synchronize()
    ttr.Handle.sync_ranks(YA, ranksA)
    ttr.Handle.sync_ranks(YB, ranksB)
    for Y, r in zip(YA, rA):
        assert Y.R == [1] + r + [1]
    for Y, r in zip(YB, rB):
        assert Y.R == [1] + r + [1]
    check_against_oracle(XA, [Y.to_numpy() for Y in YA], tol, 1e-10)
    check_against_oracle(XB, [Y.to_numpy() for Y in YB], tol, 1e-10)
    hd.close()


def test_batched_cores_not_16_byte_aligned(ttr, h):
    # inputs and outputs that start 8 bytes into their allocations: the paired
    # 16-byte loads of the batched kernels check each tensor's alignment
    import torch
    print("batched, cores at 8-byte offsets", flush=True)
    Xs, _ = batch_inputs(12, 96, start=40)

    def offset_tt(cores_np=None, I=None, caps=None):
        cores = []
        if cores_np is not None:
            R = [1]
            for c in cores_np:
                flat = torch.from_numpy(np.ascontiguousarray(np.asarray(c).reshape(-1, order="F")))
                buf = torch.empty(flat.numel() + 1, dtype=torch.float64, device="cuda")
                buf[1:].copy_(flat)
                cores.append(buf[1:])
                R.append(int(c.shape[2]))
            return ttr.TT(cores, [int(c.shape[1]) for c in cores_np], R)
        for c in caps:
            cores.append(torch.empty(int(c) + 1, dtype=torch.float64, device="cuda")[1:])
        return ttr.TT(cores, I, [1] * (len(I) + 1))

    g = [offset_tt(X) for X in Xs]
    outs = [offset_tt(I=X.I, caps=[X.R[n] * X.I[n] * X.R[n + 1] for n in range(X.N)]) for X in g]
    assert all(c.data_ptr() % 16 == 8 for X in g + outs for c in X.cores)
    Ys, ranks = h.round_batched(g, synth.TOL[3], "fp64", outs=outs)
    ttr.Handle.sync_ranks(Ys, ranks)
    check_against_oracle(Xs, [Y.to_numpy() for Y in Ys], synth.TOL[3], 1e-10)
