"""GPU parity in the launch geometry of the benchmark workloads.

* Oracle parity at I = 32768 (N = 4): every streaming pass over an interior
  core runs on 512 workgroups (the FP64 cap; 1024 for the FP32 passes), and
  each Gram pass ends in the fixed-order reduction of 512 (1024) partial
  Grams -- the grid the full-size rounds use.  Equal ranks, relative
  difference <= 1e-10 (FP64) / 1e-8 (mixed), per-link singular values.
* The A + B workload at its full size (N = 16, I = 262144, 47 GB): nothing
  can be dropped (X has exact rank 40 and tol = 1e-8), so the rounding must
  return X itself; sampled entries of the result are compared with the
  oracle's entries of X (Alg. 2's bound with no truncation), output cores are
  checked for orthonormality, and the discarded tails must be zero.
* The Hadamard workload's ranks (16 x 16 -> 256) at I = 512: oracle parity of
  ranks, tensor and every singular value above 1e-6 sigma_1 at each link.
* 64 members of the batched workload at their full mode sizes (up to 4096),
  through one ttr_round_batched call: ranks and sampled entries against the
  oracle's rounding of each member.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth
from test_gpu_round import check_round

pytestmark = pytest.mark.gpu

_CACHE = {}


@pytest.fixture(scope="module")
def h(ttr):
    hd = ttr.Handle(0)
    yield hd
    hd.close()
    _CACHE.clear()


def _oracle_round(key, X, tol, direction):
    if key not in _CACHE:
        _CACHE[key] = O.round_tt(X, tol, direction, return_info=True)
    return _CACHE[key]


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_sum_r40_512_workgroups(ttr, h, direction, prec):
    print(f"A+B ranks 40, N=4, I=32768 (512-workgroup passes) {direction} {prec}", flush=True)
    d = synth.sum_r40(I_override=32768, N=4)
    X = O.add(1.0, d["A"], 1.0, d["B"])
    ref, info = _oracle_round(("r40", direction), X, d["tol"], direction)
    g = ttr.TT.from_numpy(X)
    Yg, nrm = h.round(g, d["tol"], direction, prec, return_norm=True)
    got = Yg.to_numpy()
    assert O.ranks(got) == O.ranks(ref) == [1, 40, 40, 40, 1]
    rel = O.diff_norm(got, ref) / O.norm_ortho(ref)
    print(f"  rel diff {rel:.3e}", flush=True)
    assert rel <= (1e-10 if prec == "fp64" else 1e-8)
    # the norm that sets the threshold comes from the first link's Gram; in
    # mixed precision that Gram is accumulated in FP32 (relative error ~1e-7)
    assert math.isclose(nrm, info["norm"], rel_tol=1e-12 if prec == "fp64" else 1e-6)
    st = h.round_stats()
    # no truncation can happen here: the discarded tails are zero
    assert all(t == 0.0 for t in st["tail2"])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_sum_r50_512_workgroups(ttr, h, prec):
    # A + B + 1e-6 C: every truncation step needs a refinement pass
    print(f"A+B+1e-6C ranks 50, N=4, I=32768 {prec}", flush=True)
    d = synth.sum_r50(I_override=32768, N=4)
    X = O.add(1.0, O.add(1.0, d["A"], 1.0, d["B"]), 1.0, d["C"])
    ref, info = _oracle_round(("r50", "RLR"), X, d["tol"], "RLR")
    Yg = h.round(ttr.TT.from_numpy(X), d["tol"], "RLR", prec)
    got = Yg.to_numpy()
    assert O.ranks(got) == O.ranks(ref) == [1, 50, 50, 50, 1]
    rel = O.diff_norm(got, ref) / O.norm_ortho(ref)
    print(f"  rel diff {rel:.3e}", flush=True)
    assert rel <= (1e-10 if prec == "fp64" else 1e-8)
    st = h.round_stats()
    for l, (s_gpu, s_ref) in enumerate(zip(st["sigmas"], info["sigmas"])):
        k = min(len(s_gpu), len(s_ref))
        if k == 0:
            continue  # the step proved that nothing can be dropped
        big = np.asarray(s_ref[:k]) > 1e-6 * s_ref[0]
        assert np.allclose(np.asarray(s_gpu[:k])[big], np.asarray(s_ref[:k])[big], rtol=1e-6), l


def _sample_entries_device(T, idx):
    """Entries of a device TT at the multi-indices idx (rows), gathered slice by
    slice on the device and multiplied on the host."""
    S, N = idx.shape
    v = np.ones((S, 1))
    for n in range(N):
        r0, r1 = T.R[n], T.R[n + 1]
        t3 = T.cores[n][: r0 * T.I[n] * r1].view(r1, T.I[n], r0)     # [b][i][a]
        sl = t3[:, idx[:, n], :].permute(1, 2, 0).cpu().numpy()     # [s][a][b]
        v = np.einsum("sa,sab->sb", v, sl)
    return v[:, 0]


@pytest.mark.parametrize("direction", ["RLR", "LRL"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_sum_r40_full_size(ttr, h, direction, prec):
    import torch
    print(f"A+B ranks 40, N=16, I=262144 (47 GB) {direction} {prec}", flush=True)
    if "full40" not in _CACHE:
        d = synth.sum_r40()
        A = ttr.TT.from_numpy(d["A"])
        B = ttr.TT.from_numpy(d["B"])
        rng = np.random.default_rng(11)
        idx = rng.integers(0, 262144, size=(512, 16))
        # the oracle's entries of X = A + B (the exact rounding result here),
        # one by one: its sum of the two single-entry TTs at each multi-index
        ex = np.array([O.entry(O.add(1.0, _slices(d["A"], row), 1.0, _slices(d["B"], row)), [0] * 16)
                       for row in idx])
        del d
        X = h.add(1.0, A, 1.0, B)
        del A, B
        torch.cuda.empty_cache()
        _CACHE["full40"] = (X, idx, ex)
    X, idx, ex = _CACHE["full40"]
    Y = h.round(X, synth.TOL[1], direction, prec)
    torch.cuda.synchronize()
    assert Y.R == [1] + [40] * 15 + [1]
    ey = _sample_entries_device(Y, idx)
    rms = math.sqrt(float(np.mean(ex * ex)))
    err = float(np.max(np.abs(ey - ex))) / rms
    print(f"  max entry diff / rms entry {err:.3e}", flush=True)
    assert err <= (1e-10 if prec == "fp64" else 1e-8)
    # output orthonormality of two interior cores
    for n in (1, 9):
        a, b = Y.R[n], Y.R[n + 1]
        core = Y.cores[n][: a * Y.I[n] * b]
        if direction == "RLR":
            M = core.view(b, a * Y.I[n]).t()
            G = M.t() @ M
        else:
            M = core.view(b * Y.I[n], a).t()
            G = M @ M.t()
        e = float(torch.linalg.matrix_norm(G - torch.eye(G.shape[0], dtype=G.dtype, device=G.device)).item())
        assert e < (1e-12 if prec == "fp64" else 1e-4), (n, e)
    st = h.round_stats()
    assert all(t == 0.0 for t in st["tail2"])
    del Y
    torch.cuda.empty_cache()
    if direction == "LRL" and prec == "mixed":
        _CACHE.pop("full40", None)
        torch.cuda.empty_cache()


def _slices(cores, row):
    """The TT of the single entry at multi-index `row` (one slice per core)."""
    return [c[:, [int(i)], :] for c, i in zip(cores, row)]


def test_hadamard_rank256_I512(ttr, h):
    N, I = 6, 512
    print(f"hadamard ranks 16 x 16 -> 256, N={N} I={I}, tol 1e-6", flush=True)
    d = synth.hadamard_r256(I_override=I, N=N)
    Xg = h.hadamard(ttr.TT.from_numpy(d["A"]), ttr.TT.from_numpy(d["B"]))
    X = Xg.to_numpy()
    got, ref = check_round(ttr, h, X, d["tol"], "RLR", sig_rtol=1e-6, norm_rtol=1e-10)
    st = h.round_stats()
    # singular values are reported at full width: the cut (~210) is inside
    assert all(len(s) > O.ranks(ref)[l + 1] for l, s in enumerate(st["sigmas"]) if len(s)), \
        [len(s) for s in st["sigmas"]]
    nrm = st["norm"]
    assert math.sqrt(sum(st["tail2"])) <= d["tol"] * nrm


def test_round_hadamard_implicit_I512(ttr, h):
    # the Hadamard workload's factors (N = 6, I = 512) rounded without forming
    # A * B: ranks, tensor and singular values against the oracle
    N, I = 6, 512
    print(f"implicit Hadamard rounding N={N} I={I}", flush=True)
    d = synth.hadamard_r256(I_override=I, N=N)
    Yg = h.round_hadamard(ttr.TT.from_numpy(d["A"]), ttr.TT.from_numpy(d["B"]), d["tol"])
    got = Yg.to_numpy()
    X = O.hadamard(d["A"], d["B"])
    ref, info = O.round_tt(X, d["tol"], "RLR", return_info=True)
    assert O.ranks(got) == O.ranks(ref)
    rel = O.diff_norm(got, ref) / O.norm_ortho(ref)
    print(f"  rel diff {rel:.3e}", flush=True)
    assert rel <= 1e-10
    st = h.round_stats()
    for l, (s_gpu, s_ref) in enumerate(zip(st["sigmas"], info["sigmas"])):
        k = min(len(s_gpu), len(s_ref))
        if k == 0:
            continue
        big = np.asarray(s_ref[:k]) > 1e-6 * s_ref[0]
        assert np.allclose(np.asarray(s_gpu[:k])[big], np.asarray(s_ref[:k])[big], rtol=1e-6), l


@pytest.mark.parametrize("part", [0, 1, 2, 3])
def test_batched_members_full_size(ttr, h, part):
    # 64 members of the batched workload, full mode sizes (64..4096), rounded in
    # one batched call; members 16*part .. 16*part+15 are checked here
    import torch
    count = 64
    if "batch64" not in _CACHE:
        shapes = synth.batched_shapes(512)[:count]
        Xs_np, Xs = [], []
        for t, (I, r) in enumerate(shapes):
            Yc = synth.random_tt(3, t, "Y", I, r, scaled=True)
            E = synth.random_tt(3, t, "E", I, [2] * 7, scaled=True, first_core_factor=1e-9)
            Xn = O.add(1.0, O.add(1.0, Yc, 1.0, Yc), 1.0, E)
            Xs_np.append(Xn)
            Xs.append(ttr.TT.from_numpy(Xn))
        Ys, ranks = h.round_batched(Xs, synth.TOL[3], "fp64")
        torch.cuda.synchronize()
        rk = ranks.cpu().tolist()
        _CACHE["batch64"] = (shapes, Xs_np, Ys, rk)
    shapes, Xs_np, Ys, rk = _CACHE["batch64"]
    rng = np.random.default_rng(12)
    for t in range(16 * part, 16 * part + 16):
        I, r = shapes[t]
        print(f"  member {t} I={I} r={r}", flush=True)
        ref = O.round_tt(Xs_np[t], synth.TOL[3], "RLR")
        assert rk[t] == O.ranks(ref) == [1] + list(r) + [1], (t, rk[t], O.ranks(ref))
        Y = Ys[t]
        Y.R = list(rk[t])
        idx = np.stack([rng.integers(0, i, size=64) for i in I], axis=1)
        ey = _sample_entries_device(Y, idx)
        eo = np.array([O.entry(ref, row) for row in idx])
        rms = math.sqrt(float(np.mean(eo * eo)))
        err = float(np.max(np.abs(ey - eo))) / rms
        assert err <= 1e-10, (t, err)
    if part == 3:
        _CACHE.pop("batch64", None)
