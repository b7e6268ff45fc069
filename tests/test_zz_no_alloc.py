"""ttr_dot_noalloc: the inner product (§3.2.3, eq. (4)) with no allocation,
through the C ABI.  Its value must be ttr_dot's bit for bit (same kernels,
same summation order) and within the oracle's bar (1e-12 relative), on two
calls in a row, the second with a smaller input, and on replays of a captured
HIP graph."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


def rand_tt(rng, I, r):
    R = [1] + list(r) + [1]
    return [np.asfortranarray(rng.standard_normal((R[n], I[n], R[n + 1]))) for n in range(len(I))]


@pytest.fixture(scope="module")
def h(ttr):
    hd = ttr.Handle(0)
    yield hd
    hd.close()


def test_dot_noalloc_matches_dot_twice(ttr, h):
    import torch
    rng = np.random.default_rng(77)
    # first call: ragged ranks up to 64, mode sizes spanning many workgroups
    I1 = [3000, 4100, 2500, 3333, 700]
    X1 = rand_tt(rng, I1, [37, 64, 50, 9])
    Y1 = rand_tt(rng, I1, [21, 33, 64, 40])
    # second call: a smaller input (fewer cores, smaller modes and ranks)
    I2 = [90, 130, 77]
    X2 = rand_tt(rng, I2, [5, 11])
    Y2 = rand_tt(rng, I2, [7, 3])
    for Xn, Yn in ((X1, Y1), (X2, Y2)):
        print(f"dot_noalloc I={[c.shape[1] for c in Xn]}", flush=True)
        Xg, Yg = ttr.TT.from_numpy(Xn), ttr.TT.from_numpy(Yn)
        out = h.dot_noalloc(Xg, Yg)
        torch.cuda.synchronize()
        v_noalloc = float(out.item())
        v_dot = h.dot(Xg, Yg)
        assert v_noalloc == v_dot, (v_noalloc, v_dot)
        ref = O.dot(Xn, Yn)
        scale = O.norm_ortho(Xn) * O.norm_ortho(Yn)
        assert abs(v_noalloc - ref) <= 1e-12 * scale, (v_noalloc, ref)


def test_dot_noalloc_rejects_large_ranks(ttr, h):
    rng = np.random.default_rng(78)
    X = rand_tt(rng, [10, 10, 10], [70, 70])
    Xg = ttr.TT.from_numpy(X)
    with pytest.raises(ttr.TTRError) as e:
        h.dot_noalloc(Xg, Xg)
    assert e.value.code == 7


def test_dot_noalloc_in_captured_graph(ttr):
    import torch
    rng = np.random.default_rng(79)
    I = [500, 800, 600, 400]
    X = rand_tt(rng, I, [12, 30, 17])
    Y = rand_tt(rng, I, [8, 25, 40])
    Xg, Yg = ttr.TT.from_numpy(X), ttr.TT.from_numpy(Y)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        hg = ttr.Handle(0)        # bound to the side stream
        hg.dot_noalloc(Xg, Yg, out=out)   # warm-up outside the capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            hg.sync_stream()      # the capture stream
            hg.dot_noalloc(Xg, Yg, out=out)
    torch.cuda.synchronize()
    eager = hg.dot(Xg, Yg)
    for rep in range(4):
        out.fill_(0.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert float(out.item()) == eager, (rep, float(out.item()), eager)
        # eager work between replays
        assert hg.dot(Xg, Xg) > 0
    hg.close()
